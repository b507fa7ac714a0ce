// k_flux.hpp -- the face-flux kernel of the double-precision path, one lane
// per face (Section 3.3), and the block-level diagnostics it feeds.
#pragma once

#include "common.hpp"
#include "riemann.hpp"

namespace mm {

// Device-side diagnostic accumulators (mirrors mm_diag's counters).
struct DiagDev {
    unsigned long long newton_iters, newton_max, unconverged, vacuum, positivity_fallback, fp64_fallback,
        guess_fallback, wave_iter_max_sum;
};

// Per-lane counters reduced over the block and added once per block.
struct LaneDiag {
    unsigned iters = 0, unconv = 0, vacuum = 0, posfb = 0, fp64fb = 0, guessfb = 0;
};

__device__ __forceinline__ unsigned wave_sum(unsigned v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ unsigned wave_max(unsigned v) {
    for (int off = 32; off > 0; off >>= 1) { unsigned o = __shfl_xor(v, off, 64); v = o > v ? o : v; }
    return v;
}

__device__ __forceinline__ void flush_diag(const LaneDiag &d, bool active, DiagDev *out) {
    __shared__ unsigned red[kBlock / 64][8];
    const unsigned it = active ? d.iters : 0u;
    const unsigned s_it = wave_sum(it), m_it = wave_max(it);
    const unsigned s_un = wave_sum(d.unconv), s_va = wave_sum(d.vacuum), s_pf = wave_sum(d.posfb);
    const unsigned s_64 = wave_sum(d.fp64fb), s_gf = wave_sum(d.guessfb);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        red[w][0] = s_it; red[w][1] = m_it; red[w][2] = s_un; red[w][3] = s_va;
        red[w][4] = s_pf; red[w][5] = s_64; red[w][6] = s_gf; red[w][7] = m_it;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        unsigned mx = 0;
        for (int k = 0; k < kBlock / 64; k++) {
            for (int q = 0; q < 8; q++) t[q] += red[k][q];
            mx = red[k][1] > mx ? red[k][1] : mx;
        }
        atomicAdd(&out->newton_iters, t[0]);
        atomicMax(&out->newton_max, (unsigned long long)mx);
        atomicAdd(&out->wave_iter_max_sum, t[7]);
        if (t[2]) atomicAdd(&out->unconverged, t[2]);
        if (t[3]) atomicAdd(&out->vacuum, t[3]);
        if (t[4]) atomicAdd(&out->positivity_fallback, t[4]);
        if (t[5]) atomicAdd(&out->fp64_fallback, t[5]);
        if (t[6]) atomicAdd(&out->guess_fallback, t[6]);
    }
}

// Linear extrapolation to the face centroid and half a step forward in time
// in the face frame (Section 3.3): with v' = v - w_f and dx = f - s_K,
//   rho'' = rho + grad rho.dx - dt/2 (v'.grad rho + rho div v)
//   v''   = v'  + (grad v) dx  - dt/2 ((v'.grad) v + grad P / rho)
//   P''   = P   + grad P.dx    - dt/2 (v'.grad P + gamma P div v),
// the time derivative taken from the primitive Euler equations at the
// cell's own face-frame state.
template <int D>
__device__ __forceinline__ void half_step64(const double *__restrict__ W, const double *__restrict__ G, int64_t n,
                                            int64_t i, const double *wf, const double *dx, double gamma, double hdt,
                                            double out[D + 2], double cen[D + 2]) {
    constexpr int NV = D + 2;
    double g[NV][D];
    for (int c = 0; c < NV; c++)
        for (int k = 0; k < D; k++) g[c][k] = G[(c * D + k) * n + i];
    const double rho = W[i], P = W[(NV - 1) * n + i];
    double v[D];
    for (int k = 0; k < D; k++) v[k] = W[(1 + k) * n + i] - wf[k];
    double div = 0.0;
    for (int k = 0; k < D; k++) div += g[1 + k][k];
    double s = 0.0, t = 0.0;
    for (int k = 0; k < D; k++) { s += g[0][k] * dx[k]; t += v[k] * g[0][k]; }
    out[0] = rho + s - hdt * (t + rho * div);
    const double inv_rho = 1.0 / rho;
    for (int a = 0; a < D; a++) {
        s = 0.0; t = 0.0;
        for (int k = 0; k < D; k++) { s += g[1 + a][k] * dx[k]; t += v[k] * g[1 + a][k]; }
        out[1 + a] = v[a] + s - hdt * (t + g[NV - 1][a] * inv_rho);
    }
    s = 0.0; t = 0.0;
    for (int k = 0; k < D; k++) { s += g[NV - 1][k] * dx[k]; t += v[k] * g[NV - 1][k]; }
    out[NV - 1] = P + s - hdt * (t + gamma * P * div);
    cen[0] = rho;
    for (int k = 0; k < D; k++) cen[1 + k] = v[k];
    cen[NV - 1] = P;
}

// Steps (vi) of Section 3 for one face per lane, all in double:
// face-frame extrapolation of both sides (positivity fallback to the
// unextrapolated face-frame states if a density or pressure would not be
// positive), normal/transverse split, exact Riemann solution at x/t = 0,
// upwind transverse velocity, and the moving-face flux in the lab frame
//   (m_f, Pi + m_f w, eps + Pi.w + m_f |w|^2/2),
//   m_f = rho_F u_F, Pi = m_f v_F + P_F n, eps = m_f |v_F|^2/2 + u_F P_F g/(g-1).
// Output: flux[c][f] = dt A_f Fhat_c.
template <int D>
__global__ void __launch_bounds__(kBlock) k_face_flux64(int64_t n, int64_t nf, const int32_t *__restrict__ fL,
                                                        const int32_t *__restrict__ fR, const double *__restrict__ geo,
                                                        const double *__restrict__ wfa, const double *__restrict__ coff,
                                                        const double *__restrict__ W, const double *__restrict__ G,
                                                        const double *__restrict__ dt_ptr, double dt_val, double gamma,
                                                        double tol, int maxit, double *__restrict__ flux, DiagDev *diag) {
    constexpr int NV = D + 2;
    const int64_t f = xcd_global_id();
    const bool active = f < nf;
    LaneDiag ld;
    if (active) {
        const double dt = dt_ptr ? *dt_ptr : dt_val;
        const double hdt = 0.5 * dt;
        const int32_t l = fL[f], r = fR[f];
        const double A = geo[f], inv = geo[nf + f];
        double d[D], cc[D], nrm[D], w[D];
        for (int k = 0; k < D; k++) {
            d[k] = geo[(2 + k) * nf + f];
            cc[k] = geo[(2 + D + k) * nf + f];
            nrm[k] = d[k] * inv;
            w[k] = wfa[k * nf + f];
        }
        double xl[NV], xr[NV], cl[NV], cr[NV], dx[D];
        for (int k = 0; k < D; k++) dx[k] = cc[k] + 0.5 * d[k] - coff[k * n + l];
        half_step64<D>(W, G, n, l, w, dx, gamma, hdt, xl, cl);
        for (int k = 0; k < D; k++) dx[k] = cc[k] - 0.5 * d[k] - coff[k * n + r];
        half_step64<D>(W, G, n, r, w, dx, gamma, hdt, xr, cr);
        if (!(xl[0] > 0.0 && xl[NV - 1] > 0.0 && xr[0] > 0.0 && xr[NV - 1] > 0.0)) {
            for (int c = 0; c < NV; c++) { xl[c] = cl[c]; xr[c] = cr[c]; }
            ld.posfb = 1;
        }
        double uL = 0.0, uR = 0.0;
        for (int k = 0; k < D; k++) { uL += xl[1 + k] * nrm[k]; uR += xr[1 + k] * nrm[k]; }

        const GasConst<double> kg(gamma);
        const bool lvac = !(xl[0] > 0.0 && xl[NV - 1] > 0.0);
        const bool rvac = !(xr[0] > 0.0 && xr[NV - 1] > 0.0);
        Side<double> SL = make_side<double>(lvac ? 1.0 : xl[0], uL, lvac ? 1.0 : xl[NV - 1], kg);
        Side<double> SR = make_side<double>(rvac ? 1.0 : xr[0], uR, rvac ? 1.0 : xr[NV - 1], kg);
        FaceState<double> fs;
        int kase = RC_NORMAL;
        if (!vacuum_cases<double>(xl[0], uL, xl[NV - 1], xr[0], uR, xr[NV - 1], kg, SL, SR, lvac, rvac, fs, kase)) {
            double ps;
            bool conv;
            const double p0 = standard_guess<double>(SL, SR, kg);
            const int it = newton_star<double>(SL, SR, kg, p0, tol, maxit, ps, conv);
            ld.iters = it;
            ld.unconv = conv ? 0 : 1;
            const double us = star_velocity<double>(SL, SR, ps, kg);
            fs = sample0<double>(SL, SR, ps, us, kg);
        } else {
            ld.vacuum = 1;
        }
        // lab-frame moving-face flux
        const double *xs = fs.side ? xr : xl;
        const double us_side = fs.side ? uR : uL;
        double vF[D], v2 = 0.0, w2 = 0.0, Piw = 0.0, Pi[D];
        const double mf = fs.rho * fs.u;
        for (int k = 0; k < D; k++) {
            vF[k] = fs.u * nrm[k] + (xs[1 + k] - us_side * nrm[k]);
            v2 += vF[k] * vF[k];
            w2 += w[k] * w[k];
            Pi[k] = mf * vF[k] + fs.P * nrm[k];
            Piw += Pi[k] * w[k];
        }
        const double eps = mf * 0.5 * v2 + fs.u * fs.P * kg.g_over_gm1;
        const double scale = dt * A;
        flux[f] = scale * mf;
        for (int k = 0; k < D; k++) flux[(1 + k) * nf + f] = scale * (Pi[k] + mf * w[k]);
        flux[(NV - 1) * nf + f] = scale * (eps + Piw + 0.5 * mf * w2);
    }
    if (diag) flush_diag(ld, active, diag);
}

}  // namespace mm
