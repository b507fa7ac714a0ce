// k_cell.hpp -- per-cell kernels of the double-precision path: primitives
// and the Courant timestep, gradients with slope limiting, and the
// conservative update. One lane per cell; cells are in space-filling-curve
// order so that a wavefront's neighbours are close in memory.
#pragma once

#include "common.hpp"

namespace mm {

// Block-wide minimum of one double per lane; result valid in lane 0.
__device__ __forceinline__ double block_min(double v) {
    __shared__ double red[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBlock / 64; k++) v = fmin(v, red[k]);
    }
    return v;
}

// Step (ii) and the timestep bound of step (v) (Section 7.1):
//   rho = m/V, v = p/m, P = (g-1)(E - m v^2/2)/V;
//   dt_i = C R_i / (c_i + |v_i - w_i|), R_i the radius of the cell's volume.
// Cells with m <= 0 are vacuum (W = 0) and impose no timestep limit.
template <int D>
__global__ void __launch_bounds__(kBlock) k_prim_cfl(int64_t n, double gamma, double cfl, const double *__restrict__ V,
                                                     const double *__restrict__ Q, const double *__restrict__ mvel,
                                                     double *__restrict__ W, double *__restrict__ dt_part) {
    constexpr int NV = D + 2;
    const int64_t i = xcd_global_id();
    double dti = INFINITY;
    if (i < n) {
        const double m = Q[i];
        if (!(m > 0.0)) {
            for (int c = 0; c < NV; c++) W[c * n + i] = 0.0;
        } else {
            const double vol = V[i];
            const double inv_m = 1.0 / m;
            double v[D], ke = 0.0, rel = 0.0;
            for (int k = 0; k < D; k++) {
                v[k] = Q[(1 + k) * n + i] * inv_m;
                ke += v[k] * v[k];
                const double dv = v[k] - mvel[k * n + i];
                rel += dv * dv;
            }
            const double rho = m / vol;
            const double P = (gamma - 1.0) * (Q[(NV - 1) * n + i] - 0.5 * m * ke) / vol;
            W[i] = rho;
            for (int k = 0; k < D; k++) W[(1 + k) * n + i] = v[k];
            W[(NV - 1) * n + i] = P;
            if (rho > 0.0 && P > 0.0) {
                const double R = (D == 3) ? cbrt(vol * (3.0 / (4.0 * M_PI))) : sqrt(vol * (1.0 / M_PI));
                dti = cfl * R / (sqrt(gamma * P / rho) + sqrt(rel));
            }
        }
    }
    dti = block_min(dti);
    if (threadIdx.x == 0) dt_part[xcd_tile()] = dti;
}

__global__ void __launch_bounds__(1024) k_min_final(int64_t nparts, const double *part, double *out) {
    __shared__ double red[16];
    double v = INFINITY;
    for (int64_t k = threadIdx.x; k < nparts; k += 1024) v = fmin(v, part[k]);
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 16; k++) v = fmin(v, red[k]);
        out[0] = v;
    }
}

// Step (iii), Section 3.1. Gradient estimate exact to linear order on a
// Voronoi mesh, summed over the cell's faces in ascending face order:
//   V_i grad phi_i += s (A/|d|) [ (phi_R - phi_L) c + (phi_L + phi_R)/2 d ],
// s = +1 where i is the left cell and -1 where it is the right one. Then the
// limiter: per primitive, alpha_i = min(1, min_faces psi) with
//   psi = (phi_max - phi_i)/D if D > 0, (phi_min - phi_i)/D if D < 0, 1 else,
// D = grad phi_i . (f - s_i), phi_min/max over the face neighbours and i;
// |D| <= 1e-13 max(|phi_i|, phi_max - phi_min) counts as D = 0.
// f - s_i = c + d/2 - delta_i for the left cell, c - d/2 - delta_i for the right.
template <int D>
__global__ void __launch_bounds__(kBlock) k_grad_limit(int64_t n, int64_t nf, const int32_t *__restrict__ off,
                                                       const int32_t *__restrict__ ent, const int32_t *__restrict__ nbr,
                                                       const double *__restrict__ geo, const double *__restrict__ V,
                                                       const double *__restrict__ coff, const double *__restrict__ W,
                                                       double *__restrict__ G) {
    constexpr int NV = D + 2;
    const int64_t i = xcd_global_id();
    if (i >= n) return;
    double wi[NV], mn[NV], mx[NV], acc[NV][D];
    for (int c = 0; c < NV; c++) {
        wi[c] = W[c * n + i];
        mn[c] = wi[c];
        mx[c] = wi[c];
        for (int k = 0; k < D; k++) acc[c][k] = 0.0;
    }
    const int32_t b = off[i], e = off[i + 1];
    for (int32_t q = b; q < e; q++) {
        const int32_t en = ent[q];
        const int64_t f = en >> 1;
        const bool right = en & 1;
        const int32_t j = nbr[q];
        const double a = geo[f] * geo[nf + f];
        double d[D], cc[D];
        for (int k = 0; k < D; k++) {
            d[k] = geo[(2 + k) * nf + f];
            cc[k] = geo[(2 + D + k) * nf + f];
        }
        for (int c = 0; c < NV; c++) {
            const double wj = W[c * n + j];
            const double pl = right ? wj : wi[c];
            const double pr = right ? wi[c] : wj;
            const double dp = pr - pl, sp = 0.5 * (pl + pr);
            for (int k = 0; k < D; k++) {
                const double g = a * (dp * cc[k] + sp * d[k]);
                acc[c][k] = right ? acc[c][k] - g : acc[c][k] + g;
            }
            mn[c] = fmin(mn[c], wj);
            mx[c] = fmax(mx[c], wj);
        }
    }
    const double inv_v = 1.0 / V[i];
    double dl[D], alpha[NV];
    for (int k = 0; k < D; k++) dl[k] = coff[k * n + i];
    for (int c = 0; c < NV; c++) {
        alpha[c] = 1.0;
        for (int k = 0; k < D; k++) acc[c][k] *= inv_v;
    }
    for (int32_t q = b; q < e; q++) {
        const int32_t en = ent[q];
        const int64_t f = en >> 1;
        const double h = (en & 1) ? -0.5 : 0.5;
        double dx[D];
        for (int k = 0; k < D; k++) dx[k] = geo[(2 + D + k) * nf + f] + h * geo[(2 + k) * nf + f] - dl[k];
        for (int c = 0; c < NV; c++) {
            double dphi = 0.0;
            for (int k = 0; k < D; k++) dphi += acc[c][k] * dx[k];
            const double tol = 1e-13 * fmax(fabs(wi[c]), mx[c] - mn[c]);
            double psi = 1.0;
            if (dphi > tol) psi = (mx[c] - wi[c]) / dphi;
            else if (dphi < -tol) psi = (mn[c] - wi[c]) / dphi;
            alpha[c] = fmin(alpha[c], psi);
        }
    }
    for (int c = 0; c < NV; c++)
        for (int k = 0; k < D; k++) G[(c * D + k) * n + i] = alpha[c] * acc[c][k];
}

// Step (vii): Q_i <- Q_i - sum over faces where i is left + sum where i is
// right, in ascending face order (Section 3, discrete update). A non-finite
// result raises the flag.
template <int D>
__global__ void __launch_bounds__(kBlock) k_update(int64_t n, int64_t nf, const int32_t *__restrict__ off,
                                                   const int32_t *__restrict__ ent, const double *__restrict__ flux,
                                                   double *__restrict__ Q, int32_t *__restrict__ flags) {
    constexpr int NV = D + 2;
    const int64_t i = xcd_global_id();
    if (i >= n) return;
    double acc[NV];
    for (int c = 0; c < NV; c++) acc[c] = Q[c * n + i];
    const int32_t b = off[i], e = off[i + 1];
    for (int32_t q = b; q < e; q++) {
        const int32_t en = ent[q];
        const int64_t f = en >> 1;
        if (en & 1) {
            for (int c = 0; c < NV; c++) acc[c] += flux[c * nf + f];
        } else {
            for (int c = 0; c < NV; c++) acc[c] -= flux[c * nf + f];
        }
    }
    bool fin = true;
    for (int c = 0; c < NV; c++) {
        Q[c * n + i] = acc[c];
        fin = fin && isfinite(acc[c]);
    }
    if (!fin) atomicOr(flags, 1);
}

}  // namespace mm
