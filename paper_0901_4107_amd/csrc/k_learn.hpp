// k_learn.hpp -- the learned Newton guess: training kernels (fp32 forward,
// backward and Adam), packing of the trained parameters into the bf16
// matrix-core form, a test hook for the fused inference, the batched
// Riemann solver (labels for training; the 16M-problem benchmark) and the
// harvester of face-frame Riemann problems from a hydro step.
#pragma once

#include "common.hpp"
#include "k_flux.hpp"
#include "layout.hpp"
#include "mlp.hpp"
#include "riemann.hpp"

namespace mm {

constexpr int kMlpTile = 32;  // samples per training block

// Forward and backward of the MSE loss sum_s (y_s - t_s)^2 / n_total over a
// tile of samples; writes this block's gradient (and loss) partial sums.
// h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), y = h2 . w3 + b3.
__global__ void __launch_bounds__(kBlock) k_mlp_grad_partial(int64_t n, float inv_ntot, const float *__restrict__ prm,
                                                             const float *__restrict__ X, const float *__restrict__ T,
                                                             float *__restrict__ part) {
    __shared__ float sp[kMlpParams];
    __shared__ float sx[kMlpTile][3];
    __shared__ float h1[kMlpTile][kMlpHidden];
    __shared__ float h2[kMlpTile][kMlpHidden];
    __shared__ float dz2[kMlpTile][kMlpHidden];
    __shared__ float dy[kMlpTile];
    const int tid = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * kMlpTile;
    for (int q = tid; q < kMlpParams; q += kBlock) sp[q] = prm[q];
    for (int q = tid; q < kMlpTile * 3; q += kBlock) {
        const int64_t s = s0 + q / 3;
        sx[q / 3][q % 3] = s < n ? X[s * 3 + q % 3] : 0.0f;
    }
    __syncthreads();
    const float *W1 = sp + kMlpOffW1, *b1 = sp + kMlpOffB1, *W2 = sp + kMlpOffW2, *b2 = sp + kMlpOffB2,
                *w3 = sp + kMlpOffW3;
    for (int q = tid; q < kMlpTile * kMlpHidden; q += kBlock) {
        const int s = q / kMlpHidden, h = q % kMlpHidden;
        float z = b1[h];
        for (int k = 0; k < 3; k++) z += sx[s][k] * W1[k * kMlpHidden + h];
        h1[s][h] = z > 0.0f ? z : 0.0f;
    }
    __syncthreads();
    for (int q = tid; q < kMlpTile * kMlpHidden; q += kBlock) {
        const int s = q / kMlpHidden, h = q % kMlpHidden;
        float z = b2[h];
        for (int k = 0; k < kMlpHidden; k++) z += h1[s][k] * W2[k * kMlpHidden + h];
        h2[s][h] = z > 0.0f ? z : 0.0f;
    }
    __syncthreads();
    if (tid < kMlpTile) {
        const int64_t s = s0 + tid;
        float y = sp[kMlpOffB3];
        for (int h = 0; h < kMlpHidden; h++) y += h2[tid][h] * w3[h];
        dy[tid] = s < n ? 2.0f * (y - T[s]) * inv_ntot : 0.0f;
        // loss contribution of the sample (the partial's last slot sums them)
        dz2[tid][0] = s < n ? (y - T[s]) * (y - T[s]) * inv_ntot : 0.0f;
    }
    __syncthreads();
    float *out = part + (int64_t)blockIdx.x * (kMlpParams + 1);
    if (tid == 0) {
        float l = 0.0f, d3 = 0.0f;
        for (int s = 0; s < kMlpTile; s++) { l += dz2[s][0]; d3 += dy[s]; }
        out[kMlpParams] = l;
        out[kMlpOffB3] = d3;
    }
    __syncthreads();
    for (int h = tid; h < kMlpHidden; h += kBlock) {
        float g = 0.0f;
        for (int s = 0; s < kMlpTile; s++) g += dy[s] * h2[s][h];
        out[kMlpOffW3 + h] = g;
    }
    for (int q = tid; q < kMlpTile * kMlpHidden; q += kBlock) {
        const int s = q / kMlpHidden, h = q % kMlpHidden;
        dz2[s][h] = h2[s][h] > 0.0f ? dy[s] * w3[h] : 0.0f;
    }
    __syncthreads();
    for (int q = tid; q < kMlpHidden * kMlpHidden; q += kBlock) {
        const int k = q / kMlpHidden, h = q % kMlpHidden;
        float g = 0.0f;
        for (int s = 0; s < kMlpTile; s++) g += h1[s][k] * dz2[s][h];
        out[kMlpOffW2 + q] = g;
    }
    for (int h = tid; h < kMlpHidden; h += kBlock) {
        float g = 0.0f;
        for (int s = 0; s < kMlpTile; s++) g += dz2[s][h];
        out[kMlpOffB2 + h] = g;
    }
    __syncthreads();
    // dz1 = (dz2 W2^T) * [h1 > 0], stored over h2 (no longer needed)
    for (int q = tid; q < kMlpTile * kMlpHidden; q += kBlock) {
        const int s = q / kMlpHidden, k = q % kMlpHidden;
        float g = 0.0f;
        for (int h = 0; h < kMlpHidden; h++) g += W2[k * kMlpHidden + h] * dz2[s][h];
        h2[s][k] = h1[s][k] > 0.0f ? g : 0.0f;
    }
    __syncthreads();
    for (int q = tid; q < 3 * kMlpHidden; q += kBlock) {
        const int k = q / kMlpHidden, h = q % kMlpHidden;
        float g = 0.0f;
        for (int s = 0; s < kMlpTile; s++) g += sx[s][k] * h2[s][h];
        out[kMlpOffW1 + q] = g;
    }
    for (int h = tid; h < kMlpHidden; h += kBlock) {
        float g = 0.0f;
        for (int s = 0; s < kMlpTile; s++) g += h2[s][h];
        out[kMlpOffB1 + h] = g;
    }
}

// Sum the block partials in block order (deterministic): grad [kMlpParams],
// then loss.
__global__ void k_mlp_reduce(int64_t nblocks, const float *__restrict__ part, float *__restrict__ grad) {
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q > kMlpParams) return;
    float s = 0.0f;
    for (int64_t b = 0; b < nblocks; b++) s += part[b * (kMlpParams + 1) + q];
    grad[q] = s;
}

// Adam (bias-corrected) on the parameter vector.
__global__ void k_mlp_adam(float *__restrict__ prm, const float *__restrict__ grad, float *__restrict__ m1,
                           float *__restrict__ m2, float lr, float beta1, float beta2, float eps, float c1, float c2) {
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= kMlpParams) return;
    const float g = grad[q];
    const float a = beta1 * m1[q] + (1.0f - beta1) * g;
    const float b = beta2 * m2[q] + (1.0f - beta2) * g * g;
    m1[q] = a;
    m2[q] = b;
    prm[q] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

// fp32 forward (reference form of the network; evaluation).
__global__ void __launch_bounds__(kBlock) k_mlp_forward(int64_t n, const float *__restrict__ prm,
                                                        const float *__restrict__ X, float *__restrict__ Y) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    float x[3] = {X[s * 3], X[s * 3 + 1], X[s * 3 + 2]};
    float h1[kMlpHidden];
    for (int h = 0; h < kMlpHidden; h++) {
        float z = prm[kMlpOffB1 + h];
        for (int k = 0; k < 3; k++) z += x[k] * prm[kMlpOffW1 + k * kMlpHidden + h];
        h1[h] = z > 0.0f ? z : 0.0f;
    }
    float y = prm[kMlpOffB3];
    for (int h = 0; h < kMlpHidden; h++) {
        float z = prm[kMlpOffB2 + h];
        for (int k = 0; k < kMlpHidden; k++) z += h1[k] * prm[kMlpOffW2 + k * kMlpHidden + h];
        y += (z > 0.0f ? z : 0.0f) * prm[kMlpOffW3 + h];
    }
    Y[s] = y;
}

// Pack trained parameters into the per-lane matrix-core operand order of
// MlpPacked (one block of 256 threads).
__global__ void k_mlp_pack(const float *__restrict__ prm, MlpPacked *__restrict__ out) {
    for (int q = threadIdx.x; q < 4 * 64; q += blockDim.x) {
        const int t = q / 64, l = q % 64;
        const int h = 16 * t + (l & 15);
        bf16x4_t v;
        for (int j = 0; j < 4; j++) {
            const int k = 4 * (l >> 4) + j;
            float w = 0.0f;
            if (k < 3) w = prm[kMlpOffW1 + k * kMlpHidden + h];
            else if (k == 3) w = prm[kMlpOffB1 + h];
            v[j] = f2bf(w);
        }
        out->a1[t][l] = v;
    }
    for (int q = threadIdx.x; q < 8 * 64; q += blockDim.x) {
        const int t = q / 128, s = (q / 64) % 2, l = q % 64;
        const int hout = 16 * t + (l & 15);
        bf16x8_t v;
        for (int j = 0; j < 8; j++) v[j] = (__bf16)prm[kMlpOffW2 + mlp_l2_unit(s, l >> 4, j) * kMlpHidden + hout];
        out->a2[t][s][l] = v;
    }
    for (int h = threadIdx.x; h < kMlpHidden; h += blockDim.x) {
        out->b2[h] = prm[kMlpOffB2 + h];
        out->w3[h] = prm[kMlpOffW3 + h];
    }
    if (threadIdx.x == 0) out->b3 = prm[kMlpOffB3];
}

// Test hook: the fused bf16 inference on given features [n][3].
__global__ void __launch_bounds__(kBlock) k_mlp_infer(int64_t n, const MlpPacked *__restrict__ P,
                                                      const float *__restrict__ X, float *__restrict__ Y) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool ok = s < n;
    const float x0 = ok ? X[s * 3] : 0.0f, x1 = ok ? X[s * 3 + 1] : 0.0f, x2 = ok ? X[s * 3 + 2] : 0.0f;
    const float y = mlp_wave_infer(P, x0, x1, x2);
    if (ok) Y[s] = y;
}

// Batched 1D Riemann problems: states [6][n] (rho_L, u_L, P_L, rho_R, u_R,
// P_R, double), problems [i0, i0 + nc) of them solved in precision T with
// the standard or learned guess; out [n][5] = (rho_F, u_F, P_F, p*, p_std)
// with p* = -1 where no star state exists (vacuum); iters [n] optional. In
// float, hard problems (as for faces) are appended to hard_list (a split
// list of chunk-local indices, sub-list capacity cap) for k_riemann_hard.
template <typename T, bool LEARNED>
__global__ void __launch_bounds__(kBlock) k_riemann_batch(int64_t n, int64_t i0, int64_t nc,
                                                          const double *__restrict__ st, GasConst<T> kt, T tol,
                                                          int maxit, const MlpPacked *mlp, double *__restrict__ out,
                                                          int32_t *__restrict__ iters, int32_t *__restrict__ hard_list,
                                                          int64_t cap, DiagDev *diag) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool ok = q < nc;
    const int64_t i = i0 + q;
    T s[6];
    for (int k = 0; k < 6; k++) s[k] = ok ? (T)st[k * n + i] : (T)1;
    T pl = no_guess<T>();
    if constexpr (LEARNED) {
        const bool want = ok && wants_learned<T>(s[0], s[1], s[2], s[3], s[4], s[5], kt.g);
        pl = learned_guess_wave<T>(mlp, want, s[0], s[1], s[2], s[3], s[4], s[5], (float)kt.g);
    }
    LaneDiag ld;
    bool hard = false;
    if (ok) {
        const bool f32 = sizeof(T) == 4;
        FaceState<T> fs = solve_face<T>(s[0], s[1], s[2], s[3], s[4], s[5], kt, tol, maxit, pl, f32, ld, hard);
        if (!hard) {
            out[i * 5 + 0] = fs.rho;
            out[i * 5 + 1] = fs.u;
            out[i * 5 + 2] = fs.P;
            out[i * 5 + 3] = fs.pstar;
            out[i * 5 + 4] = fs.pstd;
        }
        if (iters) iters[i] = (int32_t)ld.iters;
    }
    if constexpr (sizeof(T) == 4) list_append(hard_list, cap, hard, (int32_t)q);
    if (diag) flush_diag(ld, diag);
}

// Double re-solve of the hard problems listed by k_riemann_batch<float>
// (from the double inputs, standard guess); their iteration counts add to
// the float ones. A fixed grid (a multiple of kLists blocks) walks the list.
__global__ void __launch_bounds__(kBlock) k_riemann_hard(int64_t n, int64_t i0, const double *__restrict__ st,
                                                         GasConst<double> kd, double tol64,
                                                         const int32_t *__restrict__ hard_list, int64_t cap,
                                                         double *__restrict__ out, int32_t *__restrict__ iters,
                                                         DiagDev *diag) {
    const ListWalk lw = list_walk(hard_list, cap);
    LaneDiag ld;
    for (int64_t q = lw.start; q < lw.count; q += lw.stride) {
        const int64_t i = i0 + lw.items[q];
        const uint32_t before = ld.iters;
        bool h2;
        FaceState<double> fd = solve_face<double>(st[i], st[n + i], st[2 * n + i], st[3 * n + i], st[4 * n + i],
                                                  st[5 * n + i], kd, tol64, 50, no_guess<double>(), false, ld, h2);
        ld.fp64fb += 1;
        out[i * 5 + 0] = fd.rho;
        out[i * 5 + 1] = fd.u;
        out[i * 5 + 2] = fd.P;
        out[i * 5 + 3] = fd.pstar;
        out[i * 5 + 4] = fd.pstd;
        if (iters) iters[i] += (int32_t)(ld.iters - before);
    }
    if (diag) flush_diag(ld, diag);
}

// Face-frame Riemann inputs of every face from double reconstruction
// records (the harvester): out [6][F] float = rho_L, u_L, P_L, rho_R, u_R, P_R
// after extrapolation and the positivity fallback.
template <int D>
__global__ void __launch_bounds__(kBlock) k_face_states64(int64_t nf, const int32_t *__restrict__ fL,
                                                          const int32_t *__restrict__ fR,
                                                          const double *__restrict__ frec,
                                                          const double *__restrict__ wf64,
                                                          const double *__restrict__ prim,
                                                          const double *__restrict__ grad, double dt, double gamma,
                                                          float *__restrict__ out) {
    using Y = Lay<D>;
    constexpr int NV = D + 2;
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f >= nf) return;
    double fr[Y::FREC], w[D];
    load_rec<Y::FREC>(frec + f * Y::FREC, fr);
    load_rec<Y::WSTRIDE>(wf64 + f * Y::WSTRIDE, w);
    const double hl = 0.5 * fr[Y::FELL];
    double nrm[D], gL[D], gR[D];
    for (int k = 0; k < D; k++) {
        nrm[k] = fr[Y::FN + k];
        gL[k] = fr[Y::FC + k] + hl * nrm[k];
        gR[k] = fr[Y::FC + k] - hl * nrm[k];
    }
    const CellRec<D, double> rl = load_cell<D>(prim, grad, fL[f]);
    const CellRec<D, double> rr = load_cell<D>(prim, grad, fR[f]);
    double xl[NV], xr[NV], cl[NV], cr[NV], vf[D];
    for (int k = 0; k < D; k++) vf[k] = rl.p[Y::W + 1 + k] - w[k];
    half_step<D, double>(rl, vf, gL, gamma, 0.5 * dt, xl, cl);
    for (int k = 0; k < D; k++) vf[k] = rr.p[Y::W + 1 + k] - w[k];
    half_step<D, double>(rr, vf, gR, gamma, 0.5 * dt, xr, cr);
    if (!(xl[0] > 0.0 && xl[NV - 1] > 0.0 && xr[0] > 0.0 && xr[NV - 1] > 0.0))
        for (int c = 0; c < NV; c++) { xl[c] = cl[c]; xr[c] = cr[c]; }
    double uL = 0.0, uR = 0.0;
    for (int k = 0; k < D; k++) { uL += xl[1 + k] * nrm[k]; uR += xr[1 + k] * nrm[k]; }
    out[0 * nf + f] = (float)xl[0];
    out[1 * nf + f] = (float)uL;
    out[2 * nf + f] = (float)xl[NV - 1];
    out[3 * nf + f] = (float)xr[0];
    out[4 * nf + f] = (float)uR;
    out[5 * nf + f] = (float)xr[NV - 1];
}

}  // namespace mm
