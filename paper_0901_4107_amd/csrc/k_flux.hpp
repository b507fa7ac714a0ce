// k_flux.hpp -- the face-flux kernels, one lane per face (Section 3.3), in
// double precision and in the mixed form, and the block-level diagnostics
// they feed.
//
// Per face: gather the two cells' reconstruction records, go to the face's
// rest frame, extrapolate each side to the face centroid and half a step
// forward in time, split velocities into the component along the L->R
// normal and the transverse rest, solve the Riemann problem exactly and
// sample it at x/t = 0, take the transverse velocity from the upwind side,
// and form the moving-face flux in the lab frame
//   (m_f, Pi + m_f w, eps + Pi.w + m_f |w|^2/2),
//   m_f = rho_F u_F, Pi = m_f v_F + P_F n, eps = m_f |v_F|^2/2 + u_F P_F g/(g-1).
// If an extrapolated density or pressure is not positive on either side,
// both sides use their unextrapolated face-frame states (counted).
// Output: flux[f][c] = dt A_f Fhat_c.
#pragma once

#include "common.hpp"
#include "k_update.hpp"
#include "layout.hpp"
#include "mlp.hpp"
#include "riemann.hpp"

namespace mm {


struct LaneDiag {
    unsigned iters = 0, itmax = 0, unconv = 0, vacuum = 0, posfb = 0, fp64fb = 0, guessfb = 0;
    // add another lane record's counts
    __device__ void add(const LaneDiag &o) {
        iters += o.iters;
        itmax = o.itmax > itmax ? o.itmax : itmax;
        unconv += o.unconv;
        vacuum += o.vacuum;
        posfb += o.posfb;
        fp64fb += o.fp64fb;
        guessfb += o.guessfb;
    }
};

// Wavefront reductions with DPP moves (every lane of the wavefront active):
// quad swaps, half-row and row mirrors leave each 16-lane row's total in
// all its lanes; the row broadcasts (lane 15 into rows 1 and 3, lane 31 into
// rows 2 and 3) then accumulate the whole wavefront in row 3, read from
// lane 63. Rows a broadcast does not write keep 'old' = 0, the identity of
// both operations.
template <int CTRL, int ROWS> __device__ __forceinline__ unsigned dpp_u32(unsigned v) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, false);
}
template <typename Op> __device__ __forceinline__ unsigned wave_reduce(unsigned v, Op op) {
    v = op(v, dpp_u32<0xB1, 0xF>(v));    // quad_perm [1,0,3,2]
    v = op(v, dpp_u32<0x4E, 0xF>(v));    // quad_perm [2,3,0,1]
    v = op(v, dpp_u32<0x141, 0xF>(v));   // row_half_mirror
    v = op(v, dpp_u32<0x140, 0xF>(v));   // row_mirror
    v = op(v, dpp_u32<0x142, 0xA>(v));   // row_bcast:15
    v = op(v, dpp_u32<0x143, 0xC>(v));   // row_bcast:31
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ unsigned wave_sum(unsigned v) {
    return wave_reduce(v, [](unsigned a, unsigned b) { return a + b; });
}
__device__ __forceinline__ unsigned wave_max(unsigned v) {
    return wave_reduce(v, [](unsigned a, unsigned b) { return a > b ? a : b; });
}

// Reduce the lanes' counters over the block; one set of atomics per block.
// The wavefront maximum of the lanes' iteration counts goes to
// wave_iter_max_sum, the largest count of a single problem to newton_max.
__device__ __forceinline__ void flush_diag(const LaneDiag &d, DiagDev *slots) {
    DiagDev *out = slots + (blockIdx.x & (kDiagSlots - 1));
    __shared__ unsigned red[kBlock / 64][8];
    const unsigned s_it = wave_sum(d.iters), m_it = wave_max(d.iters), m_one = wave_max(d.itmax);
    const unsigned s_un = wave_sum(d.unconv), s_va = wave_sum(d.vacuum), s_pf = wave_sum(d.posfb);
    const unsigned s_64 = wave_sum(d.fp64fb), s_gf = wave_sum(d.guessfb);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        red[w][0] = s_it; red[w][1] = m_it; red[w][2] = s_un; red[w][3] = s_va;
        red[w][4] = s_pf; red[w][5] = s_64; red[w][6] = s_gf; red[w][7] = m_one;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t[7] = {0, 0, 0, 0, 0, 0, 0};
        unsigned mx = 0;
        for (int k = 0; k < kBlock / 64; k++) {
            for (int q = 0; q < 7; q++) t[q] += red[k][q];
            mx = red[k][7] > mx ? red[k][7] : mx;
        }
        atomicAdd(&out->newton_iters, t[0]);
        atomicMax(&out->newton_max, (unsigned long long)mx);
        atomicAdd(&out->wave_iter_max_sum, t[1]);
        if (t[2]) atomicAdd(&out->unconverged, t[2]);
        if (t[3]) atomicAdd(&out->vacuum, t[3]);
        if (t[4]) atomicAdd(&out->positivity_fallback, t[4]);
        if (t[5]) atomicAdd(&out->fp64_fallback, t[5]);
        if (t[6]) atomicAdd(&out->guess_fallback, t[6]);
    }
}

// Face-frame extrapolation of one side from its reconstruction record:
// with v' the face-frame velocity and dx = f - s_K,
//   rho'' = rho + grad rho.dx - dt/2 (v'.grad rho + rho div v)
//   v''   = v'  + (grad v) dx  - dt/2 ((v'.grad) v + grad P / rho)
//   P''   = P   + grad P.dx    - dt/2 (v'.grad P + gamma P div v),
// the time derivative from the primitive Euler equations at the cell's own
// face-frame state. cen receives that unextrapolated state.
template <int D, typename T> struct CellRec {
    T p[Lay<D>::PREC];   // primitive record
    T g[Lay<D>::GREC];   // gradient record
};

// Gather one cell's records with 16-byte loads.
template <int D, typename T>
__device__ __forceinline__ CellRec<D, T> load_cell(const T *__restrict__ prim, const T *__restrict__ grad, int64_t i) {
    CellRec<D, T> c;
    load_rec<Lay<D>::PREC>(prim + i * Lay<D>::PREC, c.p);
    load_rec<Lay<D>::GREC>(grad + i * Lay<D>::GREC, c.g);
    return c;
}

// A window of cell records staged in LDS by the block: cells
// [c0, c0 + kWin), PREC + GREC floats each, c0 the left cell of the block's
// first face. Faces are sorted by left cell and cells run along a
// space-filling curve, so the window holds every left cell of the block's
// faces and about two thirds of their right cells (on Poisson meshes);
// those records come from LDS, the rest from memory.
constexpr int kWin = 128;
struct Window {
    const float *buf;
    int64_t c0;
};

template <int D>
__device__ __forceinline__ CellRec<D, float> load_cell_w(const float *__restrict__ prim, const float *__restrict__ grad,
                                                         int64_t i, const Window &w) {
    constexpr int RF = Lay<D>::PREC + Lay<D>::GREC;
    const int64_t k = i - w.c0;
    if (w.buf && k >= 0 && k < kWin) {
        CellRec<D, float> c;
        lds_cfloat *r = (lds_cfloat *)w.buf + k * RF;
        load_rec_lds<Lay<D>::PREC>(r, c.p);
        load_rec_lds<Lay<D>::GREC>(r + Lay<D>::PREC, c.g);
        return c;
    }
    return load_cell<D>(prim, grad, i);
}

// Every thread of the block calls it (it holds a barrier); f0 the block's
// first face, n the number of cells.
template <int D>
__device__ __forceinline__ Window stage_window(float *buf, int64_t f0, int64_t nf, const int32_t *__restrict__ fL,
                                               const float *__restrict__ prim, const float *__restrict__ grad,
                                               int64_t n) {
    constexpr int RF = Lay<D>::PREC + Lay<D>::GREC, P4 = Lay<D>::PREC / 4;
    const int64_t c0 = f0 < nf ? fL[f0] : 0;
    for (int e = threadIdx.x; e < kWin * RF / 4; e += kBlock) {
        const int cell = e / (RF / 4), part = e % (RF / 4);
        const int64_t j = c0 + cell;
        f32x4u v = {0.0f, 0.0f, 0.0f, 0.0f};
        if (j < n)
            v = part < P4 ? *reinterpret_cast<const f32x4u *>(prim + j * Lay<D>::PREC + part * 4)
                          : *reinterpret_cast<const f32x4u *>(grad + j * Lay<D>::GREC + (part - P4) * 4);
        *reinterpret_cast<f32x4u *>(buf + cell * RF + part * 4) = v;
    }
    __syncthreads();
    return Window{buf, c0};
}

template <int D, typename T>
__device__ __forceinline__ void half_step(const CellRec<D, T> &r, const T *vface, const T *gfr, T gamma, T hdt,
                                          T out[D + 2], T cen[D + 2]) {
    using Y = Lay<D>;
    constexpr int NV = D + 2;
    T g[NV][D], dx[D], v[D];
    for (int c = 0; c < NV; c++)
        for (int k = 0; k < D; k++) g[c][k] = r.g[c * D + k];
    for (int k = 0; k < D; k++) {
        dx[k] = gfr[k] - r.p[Y::DL + k];
        v[k] = vface[k];
    }
    const T rho = r.p[Y::W], P = r.p[Y::W + NV - 1];
    T div = (T)0;
    for (int k = 0; k < D; k++) div += g[1 + k][k];
    T s = (T)0, t = (T)0;
    for (int k = 0; k < D; k++) { s += g[0][k] * dx[k]; t += v[k] * g[0][k]; }
    out[0] = rho + s - hdt * (t + rho * div);
    const T inv_rho = (T)1 / rho;
    for (int a = 0; a < D; a++) {
        s = (T)0; t = (T)0;
        for (int k = 0; k < D; k++) { s += g[1 + a][k] * dx[k]; t += v[k] * g[1 + a][k]; }
        out[1 + a] = v[a] + s - hdt * (t + g[NV - 1][a] * inv_rho);
    }
    s = (T)0; t = (T)0;
    for (int k = 0; k < D; k++) { s += g[NV - 1][k] * dx[k]; t += v[k] * g[NV - 1][k]; }
    out[NV - 1] = P + s - hdt * (t + gamma * P * div);
    cen[0] = rho;
    for (int k = 0; k < D; k++) cen[1 + k] = v[k];
    cen[NV - 1] = P;
}

// Solve one face's Riemann problem in precision T with the standard or the
// learned starting guess. The learned guess is the standard one times
// exp(corr), corr the network's output (NaN: no learned guess). Returns the
// sampled state; fills the counters. `hard` (mixed path only) reports a face
// that needs the double solve: a strong rarefaction or near-vacuum problem,
// a tiny guess, or no convergence.
template <typename T>
__device__ __forceinline__ FaceState<T> solve_face(T rhoL, T uL, T PL, T rhoR, T uR, T PR, const GasConst<T> &kg,
                                                   T tol, int maxit, T corr, bool check_hard,
                                                   LaneDiag &ld, bool &hard) {
    hard = false;
    const bool lvac = !(rhoL > (T)0 && PL > (T)0);
    const bool rvac = !(rhoR > (T)0 && PR > (T)0);
    Side<T> SL = make_side<T>(lvac ? (T)1 : rhoL, uL, lvac ? (T)1 : PL, kg);
    Side<T> SR = make_side<T>(rvac ? (T)1 : rhoR, uR, rvac ? (T)1 : PR, kg);
    FaceState<T> fs;
    T vac_num = (T)0;
    if (vacuum_cases<T>(kg, SL, SR, lvac, rvac, fs, vac_num)) {
        ld.vacuum += 1;
        fs.pstar = (T)-1;
        fs.pstd = (T)-1;
        return fs;
    }
    const T p_std = standard_guess<T>(SL, SR, kg, vac_num);
    const bool learned = corr == corr;
    const T p0 = learned ? p_std * (T)__expf((float)corr) : p_std;
    fs.pstd = p_std;
    if (check_hard) {
        const T pmin = SL.P < SR.P ? SL.P : SR.P;
        if (vac_num < (T)0.5 * (SL.c + SR.c) || p0 < (T)1e-3 * pmin) { hard = true; return fs; }
    }
    Star<T> st = newton_star<T>(SL, SR, kg, p0, tol, maxit);
    int it = st.iters;
    if (!st.conv && learned) {
        // the learned guess failed: restart from the standard guess
        ld.guessfb += 1;
        st = newton_star<T>(SL, SR, kg, p_std, tol, maxit);
        it += st.iters;
    }
    ld.iters += it;
    ld.itmax = (unsigned)it > ld.itmax ? (unsigned)it : ld.itmax;
    if (!st.conv) {
        if (check_hard) { hard = true; return fs; }
        ld.unconv += 1;
    }
    fs = sample0<T>(SL, SR, st, kg);
    fs.pstar = st.ps;
    fs.pstd = p_std;
    return fs;
}

template <typename T> __device__ __forceinline__ T no_guess() { return (T)__builtin_nan(""); }

// Whether a problem takes the learned guess: both sides non-vacuum, no
// vacuum generated, a strong problem (a density or pressure ratio of at
// least e, or a velocity jump of at least 0.4 (c_L + c_R): below that every
// scaled feature is under 0.2, where the standard guess is already far more
// accurate than the network), and a standard guess that is not already
// good: neither the primitive-variable estimate in its accepted regime
// (mild pressure ratio, estimate between the pressures) nor the
// two-rarefaction estimate when both waves are rarefactions (then it is the
// exact root; that case is f(p_min) >= 0, f increasing, where only the
// higher-pressure side contributes:
// (2 c_max/(g-1)) ((p_min/p_max)^z - 1) + u_R - u_L >= 0).
template <typename T>
__device__ __forceinline__ bool wants_learned(T rhoL, T uL, T PL, T rhoR, T uR, T PR, T gamma) {
    if (!(rhoL > (T)0 && PL > (T)0 && rhoR > (T)0 && PR > (T)0)) return false;
    const T pmin = PL < PR ? PL : PR, pmax = PL < PR ? PR : PL;
    const T rmin = rhoL < rhoR ? rhoL : rhoR, rmax = rhoL < rhoR ? rhoR : rhoL;
    const bool ratio = rmax >= (T)kMlpGateRatio * rmin || pmax >= (T)kMlpGateRatio * pmin;
    const T cL2 = gamma * PL / rhoL, cR2 = gamma * PR / rhoR;
    const T du = uR - uL;
    // a mild problem leaves before any root: without a strong ratio the jump
    // must reach kMlpGateDu (c_L + c_R) >= kMlpGateDu sqrt(c_L^2 + c_R^2); the
    // margin 0.99 keeps this test from rejecting a face the exact one below
    // would accept
    if (!ratio && du * du < (T)(0.99 * kMlpGateDu * kMlpGateDu) * (cL2 + cR2)) return false;
    const T cL = mm_sqrt(cL2), cR = mm_sqrt(cR2);
    if (!(cL + cR - (T)0.5 * (gamma - (T)1) * du > (T)0)) return false;
    const T adu = du < (T)0 ? -du : du;
    if (!(ratio || adu >= (T)kMlpGateDu * (cL + cR))) return false;
    const T ppv = (T)0.5 * (PL + PR) - (T)0.125 * du * (rhoL + rhoR) * (cL + cR);
    if (pmax <= (T)2 * pmin && ppv >= pmin && ppv <= pmax) return false;
    if (ppv < pmin) {
        const T cmax = PL < PR ? cR : cL;
        const T z = (gamma - (T)1) / ((T)2 * gamma);
        const T fmin = (T)2 * cmax / (gamma - (T)1) * (mm_pow(pmin / pmax, z) - (T)1) + du;
        if (fmin >= (T)0) return false;
    }
    return true;
}

// Block-wide staging of the learned guess (the double flux kernels; the
// float ones and the batch use the per-wavefront form below): the problems
// of a block that want the network are compacted, so only ceil(count / 64)
// wavefronts evaluate it, each for 64 problems. Every thread of the block
// takes part in each phase (they hold barriers):
//   learn_count  how many threads of the block want the network (the same
//                for the whole block), and this thread's slot among them;
//   learn_put    a wanting thread stores its features in its slot;
//   learn_run    the network over the stored features;
//   learn_get    the network's ln(p* / p_standard) for a wanting thread
//                (NaN when out of range or not wanted).
struct LearnLds {
    float x[3][kBlock];
    float y[kBlock];
    int cnt[kBlock / 64];
};

__device__ __forceinline__ int learn_count(LearnLds &sh, bool want, int &slot) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long m = __ballot(want);
    if (lane == 0) sh.cnt[wv] = __popcll(m);
    __syncthreads();
    int base = 0, total = 0;
    for (int w = 0; w < kBlock / 64; w++) {
        const int c = sh.cnt[w];
        base += w < wv ? c : 0;
        total += c;
    }
    slot = base + __popcll(m & ((1ull << lane) - 1ull));
    return total;
}

template <typename T>
__device__ __forceinline__ void learn_put(LearnLds &sh, int slot, T rhoL, T uL, T PL, T rhoR, T uR, T PR,
                                          float gamma) {
    float x0, x1, x2;
    mlp_features((float)rhoL, (float)uL, (float)PL, (float)rhoR, (float)uR, (float)PR, gamma, x0, x1, x2);
    sh.x[0][slot] = x0;
    sh.x[1][slot] = x1;
    sh.x[2][slot] = x2;
}

__device__ __forceinline__ void learn_run(LearnLds &sh, const MlpPacked *P, int total) {
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (wv * 64 < total) {   // uniform per wavefront
        const int k = wv * 64 + lane;
        const bool ok = k < total;
        const float y = mlp_wave_infer(P, ok ? sh.x[0][k] : 0.0f, ok ? sh.x[1][k] : 0.0f, ok ? sh.x[2][k] : 0.0f);
        if (ok) sh.y[k] = y;
    }
    __syncthreads();
}

template <typename T> __device__ __forceinline__ T learn_get(const LearnLds &sh, bool want, int slot) {
    if (!want) return no_guess<T>();
    // the network predicts ln(p* / p_standard) / kMlpScaleY
    const float corr = kMlpScaleY * sh.y[slot];
    return (corr > -20.0f && corr < 20.0f) ? (T)corr : no_guess<T>();
}

// The learned guess for the problems of a block in one call (every thread
// of the block calls it); NaN for threads with want = false.
template <typename T>
__device__ __forceinline__ T learned_guess(const MlpPacked *P, bool want, T rhoL, T uL, T PL, T rhoR, T uR, T PR,
                                           float gamma) {
    __shared__ LearnLds sh;
    if (P == nullptr) return no_guess<T>();
    int slot;
    const int total = learn_count(sh, want, slot);
    T corr = no_guess<T>();
    if (total > 0) {   // the same for the whole block
        if (want) learn_put<T>(sh, slot, rhoL, uL, PL, rhoR, uR, PR, gamma);
        learn_run(sh, P, total);
        corr = learn_get<T>(sh, want, slot);
    }
    __syncthreads();   // every thread has read the staging before a next call rewrites it
    return corr;
}

// The learned guess for the problems of one wavefront, with no barrier and
// no LDS (every lane of the wavefront calls it, full exec mask): the lanes
// that want the network are packed to the front by lane reads, the network
// runs over ceil(count / 32) passes of 32 columns, and each result is read
// back by its lane. The other wavefronts of the block run on meanwhile.
// NaN for lanes with want = false.
template <typename T>
__device__ __forceinline__ T learned_guess_wave(const MlpPacked *P, bool want, T rhoL, T uL, T PL, T rhoR, T uR,
                                                T PR, float gamma) {
    const unsigned long long m = __ballot(want);
    if (P == nullptr || m == 0ull) return no_guess<T>();   // the same for the whole wavefront
    const int lane = threadIdx.x & 63;
    const int count = __popcll(m);
    float x0 = 0.0f, x1 = 0.0f, x2 = 0.0f;
    if (want) mlp_features((float)rhoL, (float)uL, (float)PL, (float)rhoR, (float)uR, (float)PR, gamma, x0, x1, x2);
    // lane j < count takes the j-th wanting lane: the smallest s with
    // popcount(m & (2^(s+1) - 1)) = j + 1, by bisection on s
    int s = 0;
    for (int step = 32; step > 0; step >>= 1) {
        const int t = s + step - 1;
        if (__popcll(m & (t >= 63 ? ~0ull : ((2ull << t) - 1ull))) <= lane) s += step;
    }
    const bool has = lane < count;
    const float y0 = __shfl(x0, s, 64), y1 = __shfl(x1, s, 64), y2 = __shfl(x2, s, 64);
    const float y = mlp_wave_infer(P, has ? y0 : 0.0f, has ? y1 : 0.0f, has ? y2 : 0.0f, count > 32 ? 2 : 1);
    const float back = __shfl(y, __popcll(m & ((1ull << lane) - 1ull)), 64);
    if (!want) return no_guess<T>();
    // the network predicts ln(p* / p_standard) / kMlpScaleY
    const float corr = kMlpScaleY * back;
    return (corr > -20.0f && corr < 20.0f) ? (T)corr : no_guess<T>();
}

// Section 3.5 (poorly resolved cold flows), per face: the entropy flux is
// the mass flux times A_U = P_U / rho_U^gamma of the upwind side of the
// Riemann problem, the side the face state is sampled from (AU = 0 for a
// vacuum side, whose mass flux vanishes). The face's Mach number is the
// larger over its two sides of sqrt((g+1)/(2g) p*/p_K + (g-1)/(2g)): on a
// side the star pressure exceeds, the Mach number of the shock moving into
// it; on a rarefied side below 1, which keeps the value continuous where
// p* crosses p_K. 0 without a star state (vacuum cases).
template <typename T>
__device__ __forceinline__ void entropy_terms(const FaceState<T> &fs, T rhoL, T PL, T rhoR, T PR,
                                              const GasConst<T> &k, T &AU, T &mach) {
    const T rhoU = fs.side ? rhoR : rhoL, PU = fs.side ? PR : PL;
    AU = rhoU > (T)0 ? PU / mm_pow(rhoU, k.g) : (T)0;
    mach = (T)0;
    if (fs.pstar > (T)0) {
        const T mL = mm_sqrt(k.zs1 * fs.pstar / PL + k.zs2), mR = mm_sqrt(k.zs1 * fs.pstar / PR + k.zs2);
        mach = mL > mR ? mL : mR;
    }
}

// A face's values besides its D + 2 fluxes (EM the entropy mode): the
// entropy flux (EM >= 1) and the Mach number (EM == 1; the energy switch
// does not read it, and its record ends before it).
struct FaceX {
    double v[2];
};

// One face's record, face-major (the Rec<D, EM>::FM values).
template <int D, int EM>
__device__ __forceinline__ void store_face(double *p, const double (&F)[D + 2], const FaceX &X) {
    using RC = Rec<D, EM>;
    double r[RC::FM];
    for (int c = 0; c < D + 2; c++) r[c] = F[c];
    for (int c = D + 2; c < RC::FM; c++) r[c] = X.v[c - D - 2];
    store_rec<RC::FM>(p, r);
}

// One point of the individual-timestep integration (Section 7.2) as the
// face kernels see it: per-cell bins and record times (in ticks), the
// point's tick ti (read from the info block at the start of a kernel), and
// dt_max = 2^levels ticks.
struct TbView {
    const int8_t *bin;
    const int64_t *trec;
    int64_t ti;
    double dt_max;
    int32_t levels;
    const int32_t *info;   // the timeline's info block (tick, halt and run flags)
    // Face (l, r) is integrated over fdt = 2^min(bin_l, bin_r) ticks; each
    // side is predicted from its record to the middle of that step,
    // (ti - trec) ticks + fdt/2.
    __device__ __forceinline__ void face(int64_t l, int64_t r, double &fdt, double &hl, double &hr) const {
        const int bl = bin[l], br = bin[r];
        fdt = ldexp(dt_max, (bl < br ? bl : br) - levels);
        const double tick = ldexp(dt_max, -levels);
        hl = (double)(ti - trec[l]) * tick + 0.5 * fdt;
        hr = (double)(ti - trec[r]) * tick + 0.5 * fdt;
    }
};

// Lab-frame moving-face flux in double from the sampled face-frame state
// (rho_F, u_F, P_F), the upwind transverse velocity tv, the normal n and
// the face velocity w, times scale (dt A).
template <int D>
__device__ __forceinline__ void lab_flux(double rho, double u, double P, const double *tv, const double *nrm,
                                         const double *w, double g_over_gm1, double scale, double (&out)[D + 2]) {
    constexpr int NV = D + 2;
    const double mf = rho * u;
    double v2 = 0.0, w2 = 0.0, Piw = 0.0, Pi[D];
    for (int k = 0; k < D; k++) {
        const double vF = u * nrm[k] + tv[k];
        v2 += vF * vF;
        w2 += w[k] * w[k];
        Pi[k] = mf * vF + P * nrm[k];
        Piw += Pi[k] * w[k];
    }
    const double eps = mf * 0.5 * v2 + u * P * g_over_gm1;
    out[0] = scale * mf;
    for (int k = 0; k < D; k++) out[1 + k] = scale * (Pi[k] + mf * w[k]);
    out[NV - 1] = scale * (eps + Piw + 0.5 * mf * w2);
}

// What the face bodies read besides the records: the static field
// (GRAV, Section 5.2; accel [D][n], g = -grad Phi), the mixed form's
// reference velocity W0, by value (a kernel argument the lab-frame flux
// takes from scalar registers), and its faces' w_f - W0 ([F][D] floats).
struct FaceAux {
    const double *accel;
    int64_t n;
    double w0[3] = {0.0, 0.0, 0.0};
    const float *wrel = nullptr;
};

// Double-precision flux of face f (dt A Fhat into F), the body of the face
// kernel. The left and right states are predicted over hdtL and hdtR (dt/2
// each in a global step; with individual timesteps each side's record age
// plus half the face's step). Every thread of the block calls it (the
// learned staging holds barriers); active = false does no face. LEARNED
// compiles the fused network in; the standard-guess instantiation carries
// none of its registers. EM >= 1 adds the entropy flux and the shock Mach
// number (X). GRAV adds the half-step
// kick hdt g_K of the static field to each side's predicted velocity; a
// face that falls back to its unextrapolated states takes none.
template <int D, bool LEARNED, int EM, bool GRAV>
__device__ __forceinline__ void face_flux64(bool active, int64_t f, const int32_t *__restrict__ fL,
                                            const int32_t *__restrict__ fR, const double *__restrict__ frec,
                                            const double *__restrict__ wf64, const double *__restrict__ prim, const double *__restrict__ grad,
                                            double dt, double hdtL, double hdtR, const GasConst<double> &kg,
                                            double tol, int maxit, const MlpPacked *mlp, const FaceAux &aux,
                                            LaneDiag &ld, double (&F)[D + 2], FaceX &X) {
    using Y = Lay<D>;
    constexpr int NV = D + 2;
    double A = 0.0, nrm[D], w[D], xl[NV], xr[NV], uL = 0.0, uR = 0.0;
    for (int c = 0; c < NV; c++) { xl[c] = 1.0; xr[c] = 1.0; }
    if (active) {
        double fr[Y::FREC];
        load_rec<Y::FREC>(frec + f * Y::FREC, fr);
        load_rec<Y::WSTRIDE>(wf64 + f * Y::WSTRIDE, w);
        const int64_t l = fL[f], r = fR[f];
        const CellRec<D, double> rl = load_cell<D>(prim, grad, l);
        const CellRec<D, double> rr = load_cell<D>(prim, grad, r);
        A = fr[Y::FA];
        const double hl = 0.5 * fr[Y::FELL];
        double gL[D], gR[D];
        for (int k = 0; k < D; k++) {
            nrm[k] = fr[Y::FN + k];
            const double c = fr[Y::FC + k];
            gL[k] = c + hl * nrm[k];   // f - r_L
            gR[k] = c - hl * nrm[k];   // f - r_R
        }
        double cl[NV], cr[NV], vf[D];
        for (int k = 0; k < D; k++) vf[k] = rl.p[Y::W + 1 + k] - w[k];
        half_step<D, double>(rl, vf, gL, kg.g, hdtL, xl, cl);
        for (int k = 0; k < D; k++) vf[k] = rr.p[Y::W + 1 + k] - w[k];
        half_step<D, double>(rr, vf, gR, kg.g, hdtR, xr, cr);
        if constexpr (GRAV) {
            for (int k = 0; k < D; k++) {
                xl[1 + k] += hdtL * aux.accel[k * aux.n + l];
                xr[1 + k] += hdtR * aux.accel[k * aux.n + r];
            }
        }
        if (!(xl[0] > 0.0 && xl[NV - 1] > 0.0 && xr[0] > 0.0 && xr[NV - 1] > 0.0)) {
            for (int c = 0; c < NV; c++) { xl[c] = cl[c]; xr[c] = cr[c]; }
            ld.posfb += 1;
        }
        for (int k = 0; k < D; k++) { uL += xl[1 + k] * nrm[k]; uR += xr[1 + k] * nrm[k]; }
    }
    // learned guess for the block's compacted problems
    double pl = no_guess<double>();
    if constexpr (LEARNED) {
        const bool want = active && wants_learned<double>(xl[0], uL, xl[NV - 1], xr[0], uR, xr[NV - 1], kg.g);
        pl = learned_guess<double>(mlp, want, xl[0], uL, xl[NV - 1], xr[0], uR, xr[NV - 1], (float)kg.g);
    }
    if (active) {
        bool hard;
        FaceState<double> fs = solve_face<double>(xl[0], uL, xl[NV - 1], xr[0], uR, xr[NV - 1], kg, tol, maxit,
                                                  pl, false, ld, hard);
        const double *xs = fs.side ? xr : xl;
        const double un = fs.side ? uR : uL;
        double tv[D];
        for (int k = 0; k < D; k++) tv[k] = xs[1 + k] - un * nrm[k];
        lab_flux<D>(fs.rho, fs.u, fs.P, tv, nrm, w, kg.g_over_gm1, dt * A, F);
        if constexpr (EM != 0) {
            double AU, mach;
            entropy_terms<double>(fs, xl[0], xl[NV - 1], xr[0], xr[NV - 1], kg, AU, mach);
            X.v[0] = F[0] * AU;
            X.v[1] = mach;
        }
    }
}

// Double-precision face flux kernel: one lane per face, records
// face-major (Rec<D, EM>::FM values per face).
template <int D, bool LEARNED, int EM, bool GRAV>
__global__ void __launch_bounds__(kBlock) k_face_flux64(int64_t nf, const int32_t *__restrict__ fL,
                                                        const int32_t *__restrict__ fR, const double *__restrict__ frec, const double *__restrict__ wf64,
                                                        const double *__restrict__ prim, const double *__restrict__ grad,
                                                        const double *__restrict__ dt_ptr, double dt_val,
                                                        GasConst<double> kg, double tol, int maxit,
                                                        const MlpPacked *mlp, double *__restrict__ flux, DiagDev *diag,
                                                        FaceAux aux) {
    constexpr int NV = D + 2;
    const int64_t f = xcd_global_id();
    const bool active = f < nf;
    LaneDiag ld;
    const double dt = dt_ptr ? *dt_ptr : dt_val;
    double F[NV];
    FaceX X;
    face_flux64<D, LEARNED, EM, GRAV>(active, f, fL, fR, frec, wf64, prim, grad, dt, 0.5 * dt, 0.5 * dt, kg, tol, maxit,
                                      mlp, aux, ld, F, X);
    if (active) store_face<D, EM>(flux + f * Rec<D, EM>::FM, F, X);
    if (diag) flush_diag(ld, diag);
}

// Float face-frame states of one face for the mixed path: reconstruction,
// frame transform and half step on velocities relative to the face (the
// cell record holds v_K - W0 and the face record w_f - W0, both rounded
// from double, so v_K - w_f never forms a lab-frame velocity in float).
template <int D> struct MixedFace {
    float xl[D + 2], xr[D + 2], uL, uR, nrm[D], A;
    bool posfb;
};

template <int D, int EM, bool GRAV>
__device__ __forceinline__ MixedFace<D> mixed_face_states(int64_t f, const int32_t *__restrict__ fL,
                                                          const int32_t *__restrict__ fR,
                                                          const float *__restrict__ mrec,
                                                          const float *__restrict__ prim,
                                                          const float *__restrict__ grad, float hdtL, float hdtR,
                                                          float gam, const FaceAux &aux,
                                                          const Window &win = Window{nullptr, 0}) {
    using Y = Lay<D>;
    constexpr int NV = D + 2;
    MixedFace<D> o;
    float fr[Y::MREC], wo[D];
    load_rec<Y::MREC>(mrec + f * Y::MREC, fr);
    load_rec<D>(aux.wrel + f * D, wo);
    const int64_t l = fL[f], r = fR[f];
    const CellRec<D, float> rl = load_cell_w<D>(prim, grad, l, win);
    const CellRec<D, float> rr = load_cell_w<D>(prim, grad, r, win);
    o.A = fr[Y::FA];
    const float hl = 0.5f * fr[Y::FELL];
    float gL[D], gR[D], cl[NV], cr[NV], vf[D];
    for (int k = 0; k < D; k++) {
        o.nrm[k] = fr[Y::FN + k];
        const float c = fr[Y::FC + k];
        gL[k] = c + hl * o.nrm[k];
        gR[k] = c - hl * o.nrm[k];
    }
    // v_K - w_f = (v_K - W0) - (w_f - W0)
    for (int k = 0; k < D; k++) vf[k] = rl.p[Y::W + 1 + k] - wo[k];
    half_step<D, float>(rl, vf, gL, gam, hdtL, o.xl, cl);
    for (int k = 0; k < D; k++) vf[k] = rr.p[Y::W + 1 + k] - wo[k];
    half_step<D, float>(rr, vf, gR, gam, hdtR, o.xr, cr);
    if constexpr (GRAV) {   // the half-step kick of a static field (Section 5.2)
        for (int k = 0; k < D; k++) {
            o.xl[1 + k] += hdtL * (float)aux.accel[k * aux.n + l];
            o.xr[1 + k] += hdtR * (float)aux.accel[k * aux.n + r];
        }
    }
    o.posfb = !(o.xl[0] > 0.0f && o.xl[NV - 1] > 0.0f && o.xr[0] > 0.0f && o.xr[NV - 1] > 0.0f);
    if (o.posfb)
        for (int c = 0; c < NV; c++) { o.xl[c] = cl[c]; o.xr[c] = cr[c]; }
    o.uL = 0.0f;
    o.uR = 0.0f;
    for (int k = 0; k < D; k++) { o.uL += o.xl[1 + k] * o.nrm[k]; o.uR += o.xr[1 + k] * o.nrm[k]; }
    return o;
}

// The lab-frame flux of a mixed face: the face velocity is W0 + (w_f - W0)
// as the face record holds it, the one the face frame was formed with, so
// the transform there and back is exact.
template <int D>
__device__ __forceinline__ void mixed_lab_flux(const MixedFace<D> &m, double rho, double u, double P, int side,
                                               int64_t f, const FaceAux &aux, double g_over_gm1, double dt,
                                               double (&out)[D + 2]) {
    const float *xs = side ? m.xr : m.xl;
    const float un = side ? m.uR : m.uL;
    float wo[D];
    load_rec<D>(aux.wrel + f * D, wo);
    double tv[D], nd[D], w[D];
    for (int k = 0; k < D; k++) {
        tv[k] = (double)(xs[1 + k] - un * m.nrm[k]);
        nd[k] = (double)m.nrm[k];
        w[k] = aux.w0[k] + (double)wo[k];
    }
    lab_flux<D>(rho, u, P, tv, nd, w, g_over_gm1, dt * (double)m.A, out);
}

// LDS the learned guess of the mixed kernel parks the two face states in
// while the network runs (floats; each lane its own slots).
template <int D> constexpr int stash_floats() { return 2 * (D + 2) * kBlock; }

// Mixed-precision flux of face f (dt A Fhat into F): float face states and
// float Newton; the lab-frame flux and everything after it in double. Faces
// the float solve judges hard (strong rarefaction or near vacuum, tiny
// guess, no convergence) come back with hard = true and no flux. The body
// of the face kernel; active = false does no face, but every lane of a
// wavefront calls it (the learned guess works across the wavefront). Only a
// wavefront with a face the gate passes runs the network, over its gated
// faces compacted by lane reads (learned_guess_wave); meanwhile the two
// face states wait in the lane's own LDS slots (stash: 2(D+2) kBlock floats,
// apart from the window) and the normal and area are read again from the
// face record, so the network's registers come on top of few live values.
// No barrier: the other wavefronts of the block run on.
template <int D, bool LEARNED, int EM, bool GRAV>
__device__ __forceinline__ void face_flux_mixed(bool active, int64_t f, const int32_t *__restrict__ fL,
                                                const int32_t *__restrict__ fR, const float *__restrict__ mrec,
                                                const float *__restrict__ prim,
                                                const float *__restrict__ grad, double dt, double hdtL, double hdtR,
                                                const GasConst<float> &kf, double g_over_gm1, float tol32, int maxit,
                                                const MlpPacked *mlp, const FaceAux &aux, float *stash,
                                                LaneDiag &ld, bool &hard, double (&F)[D + 2], FaceX &X,
                                                const Window &win = Window{nullptr, 0}) {
    constexpr int NV = D + 2;
    hard = false;
    MixedFace<D> m;
    if (active) {
        m = mixed_face_states<D, EM, GRAV>(f, fL, fR, mrec, prim, grad, (float)hdtL, (float)hdtR, kf.g, aux, win);
        ld.posfb += m.posfb ? 1 : 0;
    } else {
        for (int c = 0; c < NV; c++) { m.xl[c] = 1.0f; m.xr[c] = 1.0f; }
        m.uL = 0.0f;
        m.uR = 0.0f;
    }
    float pl = no_guess<float>();
    if constexpr (LEARNED) {
        const bool want =
            active && wants_learned<float>(m.xl[0], m.uL, m.xl[NV - 1], m.xr[0], m.uR, m.xr[NV - 1], kf.g);
        if (mlp && __ballot(want) != 0ull) {   // the same for the whole wavefront
            const int t = threadIdx.x;
            for (int c = 0; c < NV; c++) { stash[c * kBlock + t] = m.xl[c]; stash[(NV + c) * kBlock + t] = m.xr[c]; }
            pl = learned_guess_wave<float>(mlp, want, m.xl[0], m.uL, m.xl[NV - 1], m.xr[0], m.uR, m.xr[NV - 1], kf.g);
            for (int c = 0; c < NV; c++) { m.xl[c] = stash[c * kBlock + t]; m.xr[c] = stash[(NV + c) * kBlock + t]; }
            float fr[2 + D];   // A, |d|, n
            load_rec<2 + D>(mrec + (active ? f : 0) * Lay<D>::MREC, fr);
            m.A = fr[Lay<D>::FA];
            m.uL = 0.0f;
            m.uR = 0.0f;
            for (int k = 0; k < D; k++) {
                m.nrm[k] = fr[Lay<D>::FN + k];
                m.uL += m.xl[1 + k] * m.nrm[k];
                m.uR += m.xr[1 + k] * m.nrm[k];
            }
        }
    }
    if (active) {
        FaceState<float> fs = solve_face<float>(m.xl[0], m.uL, m.xl[NV - 1], m.xr[0], m.uR, m.xr[NV - 1], kf, tol32,
                                                maxit, pl, true, ld, hard);
        if (!hard) {
            mixed_lab_flux<D>(m, fs.rho, fs.u, fs.P, fs.side, f, aux, g_over_gm1, dt, F);
            if constexpr (EM != 0) {
                float AU, mach;
                entropy_terms<float>(fs, m.xl[0], m.xl[NV - 1], m.xr[0], m.xr[NV - 1], kf, AU, mach);
                X.v[0] = F[0] * (double)AU;
                X.v[1] = (double)mach;
            }
        }
    }
}

// Mixed-precision face flux kernel: one lane per face, records face-major;
// hard faces are appended to a split list (wave-aggregated) and left to
// k_face_flux_hard. Held to 7 wavefronts per SIMD.
template <int D, bool LEARNED, int EM, bool GRAV>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7))) k_face_flux_mixed(int64_t nf, const int32_t *__restrict__ fL,
                                                            const int32_t *__restrict__ fR,
                                                            const float *__restrict__ mrec,
                                                            const float *__restrict__ prim,
                                                            const float *__restrict__ grad,
                                                            const double *__restrict__ dt_ptr, double dt_val,
                                                            GasConst<float> kf, double g_over_gm1, float tol32,
                                                            int maxit, const MlpPacked *mlp,
                                                            double *__restrict__ flux, int32_t *__restrict__ hard_list,
                                                            int64_t cap, DiagDev *diag, FaceAux aux) {
    constexpr int NV = D + 2;
    constexpr int SW = kWin * (Lay<D>::PREC + Lay<D>::GREC);
    // the staged window of cell records, and apart from it the learned
    // guess's parking slots
    __shared__ float wbuf[SW];
    __shared__ float stash[LEARNED ? stash_floats<D>() : 1];
    const int64_t f = xcd_global_id();
    const bool active = f < nf;
    const Window win = stage_window<D>(wbuf, xcd_tile() * kBlock, nf, fL, prim, grad, aux.n);
    LaneDiag ld;
    bool hard;
    const double dt = dt_ptr ? *dt_ptr : dt_val;
    double F[NV];
    FaceX X;
    face_flux_mixed<D, LEARNED, EM, GRAV>(active, f, fL, fR, mrec, prim, grad, dt, 0.5 * dt, 0.5 * dt, kf,
                                          g_over_gm1, tol32, maxit, mlp, aux, stash, ld, hard, F, X, win);
    if (active && !hard) store_face<D, EM>(flux + f * Rec<D, EM>::FM, F, X);
    list_append(hard_list, cap, hard, (int32_t)f);
    if (diag) flush_diag(ld, diag);
}

// The double solve of a hard face: the float face states recomputed by the
// same code (hence identical), the Riemann problem in double, the lab-frame
// flux; over the prediction intervals hl, hr and the step dt.
template <int D, int EM, bool GRAV>
__device__ __forceinline__ void hard_face(int64_t f, const int32_t *__restrict__ fL, const int32_t *__restrict__ fR,
                                          const float *__restrict__ mrec,
                                          const float *__restrict__ prim, const float *__restrict__ grad, double dt,
                                          double hl, double hr, float gam, const GasConst<double> &kg, double tol64,
                                          const FaceAux &aux, LaneDiag &ld, double (&F)[D + 2], FaceX &X) {
    constexpr int NV = D + 2;
    const MixedFace<D> m =
        mixed_face_states<D, EM, GRAV>(f, fL, fR, mrec, prim, grad, (float)hl, (float)hr, gam, aux);
    bool h2;
    FaceState<double> fd = solve_face<double>(m.xl[0], m.uL, m.xl[NV - 1], m.xr[0], m.uR, m.xr[NV - 1], kg, tol64,
                                              50, no_guess<double>(), false, ld, h2);
    ld.fp64fb += 1;
    mixed_lab_flux<D>(m, fd.rho, fd.u, fd.P, fd.side, f, aux, kg.g_over_gm1, dt, F);
    if constexpr (EM != 0) {
        double AU, mach;
        entropy_terms<double>(fd, (double)m.xl[0], (double)m.xl[NV - 1], (double)m.xr[0], (double)m.xr[NV - 1], kg,
                              AU, mach);
        X.v[0] = F[0] * AU;
        X.v[1] = mach;
    }
}

// Double re-solve of the hard faces listed by k_face_flux_mixed (a split
// list of sub-list capacity cap), face-major records. A fixed grid
// walks the list, so the launch needs no host-side count. With tb.bin set
// (individual timesteps) each face takes its step and prediction intervals
// from the timeline.
template <int D, int EM, bool GRAV>
__global__ void __launch_bounds__(kBlock) k_face_flux_hard(const int32_t *__restrict__ fL,
                                                           const int32_t *__restrict__ fR,
                                                           const float *__restrict__ mrec,
                                                           const float *__restrict__ prim,
                                                           const float *__restrict__ grad,
                                                           const double *__restrict__ dt_ptr, double dt_val,
                                                           float gam, GasConst<double> kg, double tol64,
                                                           const int32_t *__restrict__ hard_list, int64_t cap,
                                                           double *__restrict__ flux, DiagDev *diag, FaceAux aux,
                                                           TbView tb) {
    constexpr int NV = D + 2;
    const ListWalk lw = list_walk(hard_list, cap);
    if (tb.bin) tb.ti = tb64(tb.info, TB_TI);
    LaneDiag ld;
    for (int64_t q = lw.start; q < lw.count; q += lw.stride) {
        const int64_t f = lw.items[q];
        double dt = dt_ptr ? *dt_ptr : dt_val, hl = 0.5 * dt, hr = 0.5 * dt;
        if (tb.bin) tb.face(fL[f], fR[f], dt, hl, hr);
        double F[NV];
        FaceX X;
        hard_face<D, EM, GRAV>(f, fL, fR, mrec, prim, grad, dt, hl, hr, gam, kg, tol64, aux, ld, F, X);
        store_face<D, EM>(flux + f * Rec<D, EM>::FM, F, X);
    }
    if (diag) flush_diag(ld, diag);
}

// Individual timesteps: the active faces of a point, listed in a split
// list, each integrated over its own step (TbView). Each block walks its
// sub-list in block-uniform rounds, since the learned staging holds
// barriers. Double path.
template <int D, bool LEARNED>
__global__ void __launch_bounds__(kBlock) k_face_flux64_list(const int32_t *__restrict__ list, int64_t cap,
                                                             const int32_t *__restrict__ fL,
                                                             const int32_t *__restrict__ fR,
                                                             const double *__restrict__ frec, const double *__restrict__ wf64,
                                                             const double *__restrict__ prim,
                                                             const double *__restrict__ grad, TbView tb,
                                                             GasConst<double> kg, double tol, int maxit,
                                                             const MlpPacked *mlp, double *__restrict__ flux,
                                                             DiagDev *diag) {
    constexpr int NV = D + 2;
    const int c = blockIdx.x % kLists;
    const int32_t *items = list + (int64_t)kLists * kListPad + c * cap;
    tb.ti = tb64(tb.info, TB_TI);
    const int64_t count = (!tb.info[TB_LIVE] || tb.info[TB_ERR]) ? 0 : list[c * kListPad];
    const int64_t stride = (int64_t)(gridDim.x / kLists) * kBlock;
    LaneDiag ld;
    for (int64_t base = (int64_t)(blockIdx.x / kLists) * kBlock; base < count; base += stride) {
        const int64_t q = base + threadIdx.x;
        const bool active = q < count;
        const int64_t f = active ? items[q] : 0;
        double fdt = 0.0, hl = 0.0, hr = 0.0;
        if (active) tb.face(fL[f], fR[f], fdt, hl, hr);
        double F[NV];
        FaceX X;
        face_flux64<D, LEARNED, 0, false>(active, f, fL, fR, frec, wf64, prim, grad, fdt, hl, hr, kg, tol, maxit, mlp,
                                          FaceAux{nullptr, 0}, ld, F, X);
        if (active) store_face<D, 0>(flux + f * NV, F, X);
    }
    if (diag) flush_diag(ld, diag);
}

// The same on the mixed path: hard faces go to the split hard list (the
// sub-list of the block's residue, which holds at most as many items as
// the face sub-list the block walks) for k_face_flux_hard. The learned
// instantiation runs at 4 wavefronts per SIMD, where it needs no spill
// (1% faster per timeline cycle than 5 with 16 bytes spilled).
template <int D, bool LEARNED>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(LEARNED ? 4 : 5)))
k_face_flux_mixed_list(const int32_t *__restrict__ list, int64_t cap, const int32_t *__restrict__ fL,
                       const int32_t *__restrict__ fR, const float *__restrict__ mrec,
                       const float *__restrict__ prim,
                       const float *__restrict__ grad, TbView tb, GasConst<float> kf, double g_over_gm1,
                       float tol32, int maxit, const MlpPacked *mlp, double *__restrict__ flux,
                       int32_t *__restrict__ hard_list, DiagDev *diag, FaceAux aux) {
    constexpr int NV = D + 2;
    __shared__ float stash[LEARNED ? stash_floats<D>() : 1];
    const int c = blockIdx.x % kLists;
    const int32_t *items = list + (int64_t)kLists * kListPad + c * cap;
    tb.ti = tb64(tb.info, TB_TI);
    const int64_t count = (!tb.info[TB_LIVE] || tb.info[TB_ERR]) ? 0 : list[c * kListPad];
    const int64_t stride = (int64_t)(gridDim.x / kLists) * kBlock;
    LaneDiag ld;
    for (int64_t base = (int64_t)(blockIdx.x / kLists) * kBlock; base < count; base += stride) {
        const int64_t q = base + threadIdx.x;
        const bool active = q < count;
        const int64_t f = active ? items[q] : 0;
        double fdt = 0.0, hl = 0.0, hr = 0.0;
        if (active) tb.face(fL[f], fR[f], fdt, hl, hr);
        bool hard;
        double F[NV];
        FaceX X;
        face_flux_mixed<D, LEARNED, 0, false>(active, f, fL, fR, mrec, prim, grad, fdt, hl, hr, kf,
                                              g_over_gm1, tol32, maxit, mlp, aux,
                                              stash, ld, hard, F, X);
        if (active && !hard) store_face<D, 0>(flux + f * NV, F, X);
        list_append(hard_list, cap, active && hard, (int32_t)f);
    }
    if (diag) flush_diag(ld, diag);
}

}  // namespace mm
