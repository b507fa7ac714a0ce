// k_cell.hpp -- per-cell kernels: primitives and the Courant timestep,
// gradients with slope limiting, the entropy row's start, mesh motion (the
// conservative update is in k_update.hpp).
//
// The gradient and update kernels give each cell a group of GS lanes
// (4; a wavefront serves 16 cells) that walk the cell's
// face-side list together: consecutive lanes read consecutive side records,
// and the per-cell sums, minima and maxima are butterfly reductions inside
// the group (no atomics, fixed order, so results are bitwise reproducible).
#pragma once

#include "common.hpp"
#include "layout.hpp"
#include "riemann.hpp"

namespace mm {

template <int D> struct Group { static constexpr int GS = 4; };

// Cross-lane moves inside 16-lane rows by DPP (no LDS round trip):
// quad_perm xor 1 and xor 2, then row_half_mirror (lane i <- 7 - i within 8)
// and row_mirror (i <- 15 - i). After the quad steps every lane of a quad
// holds the quad's result, so the mirrors combine whole quads and halves:
// all GS lanes of a group end with the group's result.
enum : int { DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140 };

template <int CTRL> __device__ __forceinline__ float dpp(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double dpp(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <int GS, typename T, typename Op> __device__ __forceinline__ T grp_reduce(T v, Op op) {
    static_assert(GS == 4 || GS == 8 || GS == 16, "group size");
    v = op(v, dpp<DPP_XOR1>(v));
    v = op(v, dpp<DPP_XOR2>(v));
    if (GS >= 8) v = op(v, dpp<DPP_HALF_MIRROR>(v));
    if (GS >= 16) v = op(v, dpp<DPP_MIRROR>(v));
    return v;
}
template <int GS, typename T> __device__ __forceinline__ T grp_sum(T v) {
    return grp_reduce<GS>(v, [](T a, T b) { return a + b; });
}
template <int GS, typename T> __device__ __forceinline__ T grp_max(T v) {
    return grp_reduce<GS>(v, [](T a, T b) { return fmax(a, b); });
}
template <int GS, typename T> __device__ __forceinline__ T grp_min(T v) {
    return grp_reduce<GS>(v, [](T a, T b) { return fmin(a, b); });
}

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

// Step (ii) for one cell (Section 3, state vector and equation of state):
//   rho = m/V, v = p/m, P = (g-1)(E - m v^2/2)/V.
// Fills the primitive record (W and s_i - r_i, whole; coff [D][n] the
// centroid offsets in double or, rounded once, in the records' float); in the mixed mode
// (T = float) the velocity stored is v_i - W0, rounded once from double, W0
// the reference velocity w0 [D] (device). Returns the cell's sound speed (0
// unless rho > 0 and P > 0) and sets v (lab frame), |v - w|^2, the radius R
// of the cell's volume and ok = (rho > 0 and P > 0). Cells with m <= 0 are
// vacuum: rho = P = 0, v = 0.
template <int D, typename T, typename C>
__device__ __forceinline__ double cell_prim(int64_t i, int64_t n, double gamma, const double *__restrict__ V,
                                            const double *__restrict__ Q, const double *__restrict__ mvel,
                                            const C *__restrict__ coff, const double *__restrict__ w0,
                                            T (&r)[Lay<D>::PREC], double (&v)[D], double &rel2, double &R, bool &ok) {
    using Y = Lay<D>;
    constexpr int NV = D + 2;
    constexpr bool rel = sizeof(T) == 4;
    for (int k = 0; k < Y::PREC; k++) r[k] = (T)0;
    for (int k = 0; k < D; k++) {
        r[Y::DL + k] = (T)coff[k * n + i];
        v[k] = 0.0;
        if (rel) r[Y::W + 1 + k] = (T)(0.0 - w0[k]);
    }
    rel2 = 0.0;
    R = 0.0;
    ok = false;
    const double m = Q[i];
    if (!(m > 0.0)) return 0.0;
    const double vol = V[i];
    const double inv_m = 1.0 / m;
    double ke = 0.0;
    for (int k = 0; k < D; k++) {
        v[k] = Q[(1 + k) * n + i] * inv_m;
        ke += v[k] * v[k];
        const double dv = v[k] - mvel[k * n + i];
        rel2 += dv * dv;
        r[Y::W + 1 + k] = rel ? (T)(v[k] - w0[k]) : (T)v[k];
    }
    const double rho = m / vol;
    const double P = (gamma - 1.0) * (Q[(NV - 1) * n + i] - 0.5 * m * ke) / vol;
    r[Y::W] = (T)rho;
    r[Y::W + NV - 1] = (T)P;
    ok = rho > 0.0 && P > 0.0;
    if (!ok) return 0.0;
    R = (D == 3) ? cbrt(vol * (3.0 / (4.0 * M_PI))) : sqrt(vol * (1.0 / M_PI));
    return sqrt(gamma * P / rho);
}

// Step (ii) and the timestep bound of step (v) (Section 7.1): the primitive
// record of every cell (cell_prim) and the per-block minimum of
//   dt_i = C R_i / (c_i + |v_i - w_i|), R_i the radius of the cell's volume;
// vacuum cells impose no limit. As the first kernel of a step it clears the
// step's non-finite flag (step_flag, may be null) and, given clear, the
// nclear counters of the face pass's hard-face list. w0: the mixed mode's
// reference velocity (null in double). coff: the centroid offsets in the
// records' precision (the mixed mode's float copy, made at upload).
template <int D, typename T>
__global__ void __launch_bounds__(kBlock) k_prim_cfl(int64_t n, double gamma, double cfl, const double *__restrict__ V,
                                                     const double *__restrict__ Q, const double *__restrict__ mvel,
                                                     const T *__restrict__ coff, T *__restrict__ prim,
                                                     const double *__restrict__ w0, double *__restrict__ dt_part,
                                                     int32_t *step_flag, int32_t *__restrict__ clear, int nclear) {
    using Y = Lay<D>;
    const int64_t i = xcd_global_id();
    if (step_flag && blockIdx.x == 0 && threadIdx.x == 0) *step_flag = 0;
    if (clear)
        for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < nclear; q += (int64_t)gridDim.x * kBlock)
            clear[q] = 0;
    double dti = INFINITY;
    if (i < n) {
        T r[Y::PREC];
        double v[D], rel2, R;
        bool ok;
        const double c = cell_prim<D, T>(i, n, gamma, V, Q, mvel, coff, w0, r, v, rel2, R, ok);
        if (ok) dti = cfl * R / (c + sqrt(rel2));
        store_rec<Y::PREC>(prim + i * Y::PREC, r);
    }
    dti = block_min(dti);
    if (threadIdx.x == 0) dt_part[xcd_tile()] = dti;
}

// The mixed mode's float copy of the centroid offsets s_i - r_i [D][n],
// rounded once per mesh as the primitive records hold them.
template <int D>
__global__ void __launch_bounds__(kBlock) k_coff32(int64_t n, const double *__restrict__ coff, float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < D; k++) out[k * n + i] = (float)coff[k * n + i];
}

// The reference velocity W0 of the mixed mode's records: per component the
// midrange (min + max)/2 of the generator velocities, which makes the
// largest |w_i - W0| (and so the float rounding of velocities relative to
// W0 on a mesh that follows the flow) as small as it can be. Per-block minima and maxima part [grid][2D], then one
// block for w0 [D]; both order-independent.
template <int D>
__global__ void __launch_bounds__(kBlock) k_w0_part(int64_t n, const double *__restrict__ mvel,
                                                    double *__restrict__ part) {
    __shared__ double red[2 * D][kBlock / 64];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (int k = 0; k < D; k++) {
        double lo = i < n ? mvel[k * n + i] : INFINITY;
        double hi = i < n ? mvel[k * n + i] : -INFINITY;
        for (int off = 32; off > 0; off >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, off, 64));
            hi = fmax(hi, __shfl_xor(hi, off, 64));
        }
        if ((threadIdx.x & 63) == 0) {
            red[2 * k][threadIdx.x / 64] = lo;
            red[2 * k + 1][threadIdx.x / 64] = hi;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * D) {
        const int q = threadIdx.x;
        double v = red[q][0];
        for (int w = 1; w < kBlock / 64; w++) v = (q & 1) ? fmax(v, red[q][w]) : fmin(v, red[q][w]);
        part[(int64_t)blockIdx.x * 2 * D + q] = v;
    }
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_w0_final(int64_t nparts, const double *__restrict__ part,
                                                     double *__restrict__ w0) {
    __shared__ double red[2 * D][kBlock / 64];
    for (int q = 0; q < 2 * D; q++) {
        double v = (q & 1) ? -INFINITY : INFINITY;
        for (int64_t b = threadIdx.x; b < nparts; b += kBlock)
            v = (q & 1) ? fmax(v, part[b * 2 * D + q]) : fmin(v, part[b * 2 * D + q]);
        for (int off = 32; off > 0; off >>= 1)
            v = (q & 1) ? fmax(v, __shfl_xor(v, off, 64)) : fmin(v, __shfl_xor(v, off, 64));
        if ((threadIdx.x & 63) == 0) red[q][threadIdx.x / 64] = v;
    }
    __syncthreads();
    if (threadIdx.x < D) {
        const int k = threadIdx.x;
        double lo = red[2 * k][0], hi = red[2 * k + 1][0];
        for (int w = 1; w < kBlock / 64; w++) {
            lo = fmin(lo, red[2 * k][w]);
            hi = fmax(hi, red[2 * k + 1][w]);
        }
        w0[k] = 0.5 * lo + 0.5 * hi;
    }
}

// Step (iii), Section 3.1, gradient and limiter of one cell per lane group.
// The Voronoi gradient estimate (exact to linear order)
//   V_i grad phi_i = sum_j A_ij ([phi_j - phi_i] c_ij - (phi_i + phi_j)/2 r_ij) / |r_ij|
// is evaluated in its difference form
//   V_i grad phi_i = sum_j (A_ij/|r_ij|) (phi_j - phi_i) (f_ij - r_i),
// equal to it because every Voronoi cell is closed (sum_j A_ij r_ij/|r_ij| = 0,
// checked at upload): the phi_i parts of the two sums cancel, and
// c_ij + (r_j - r_i)/2 = f_ij - r_i. Only differences of primitives enter,
// so a bulk velocity costs no precision.
// Limiter, per primitive: alpha = min(1, min_faces psi) with
//   psi = (phi_max - phi_i)/Dl if Dl > tol, (phi_min - phi_i)/Dl if Dl < -tol, 1 else,
// Dl = grad phi_i . (f - s_i) = grad phi_i . ((f - r_i) - (s_i - r_i)), the
// extremes over the face neighbours and i itself, and
// tol = eps_t max(|phi_i|, phi_max - phi_min) (a |Dl| at round-off level counts
// as zero). Since phi_max - phi_i >= 0 is fixed per cell and rounded
// division is monotone, the minimum over faces of (phi_max - phi_i)/Dl is
// (phi_max - phi_i)/max Dl, so two divisions per primitive suffice; and the
// sides with |Dl| <= tol never hold that maximum unless no side exceeds tol,
// so the lanes keep plain maxima and minima of Dl and the tolerance is
// applied once per cell.
// Mixed mode (T = float): the primitive records hold velocities relative to
// the reference velocity W0 (the midrange of the generator velocities), so
// the velocity difference across a side is
//   v_j - v_i = (v_j - W0) - (v_i - W0)
// and no lab-frame velocity is formed in float.
// Each lane keeps its first KR sides (A/|r|, f - r_i) in registers for the
// limiter pass and issues their loads together; sides beyond GS*KR (rare)
// are walked by a loop that re-reads them.
template <int D, typename T> struct SideAcc {
    static constexpr int NV = D + 2;
    T acc[NV][D], dmx[NV], dmn[NV];
};

// One side: s the side record, pj the neighbour's values and wi the cell's
// (W, velocities relative to W0 in the mixed mode).
template <int D, typename T>
__device__ __forceinline__ void grad_side(const T *s, const T *pj, const T *wi, SideAcc<D, T> &a) {
    constexpr int NV = D + 2;
    const T w = s[0];
    for (int c = 0; c < NV; c++) {
        const T dphi = pj[c] - wi[c];
        const T ad = w * dphi;
        for (int k = 0; k < D; k++) a.acc[c][k] += ad * s[1 + k];
        a.dmx[c] = fmax(a.dmx[c], dphi);
        a.dmn[c] = fmin(a.dmn[c], dphi);
    }
}

template <int D, typename T>
__device__ __forceinline__ void limit_side(const T *g, const T *dl, const T (&grad)[D + 2][D], T *up, T *dn) {
    constexpr int NV = D + 2;
    T dx[D];
    for (int k = 0; k < D; k++) dx[k] = g[k] - dl[k];
    for (int c = 0; c < NV; c++) {
        T dphi = (T)0;
        for (int k = 0; k < D; k++) dphi += grad[c][k] * dx[k];
        up[c] = fmax(up[c], dphi);
        dn[c] = fmin(dn[c], dphi);
    }
}

// The energy switch's term (Section 3.5, eq. eqnScrit1): the kinetic
// energy of neighbour j (or of cell i itself) in the frame of cell i's generator,
// M_j |v_j - w_i|^2 / 2 with M_j = rho_j V_j (0 for a vacuum neighbour), from
// j's values pj as the gradient pass reads them: the primitive records hold
// v_j (double) or v_j - W0 (float), and wg is w_i in the same frame, so
// v_j - w_i = pj's velocity - wg. In the records' precision: the float
// form's velocities carry float rounding already, and the switch compares
// this with the cell's thermal energy at a threshold alpha far above it.
template <int D, typename T>
__device__ __forceinline__ T ekin_in_frame(const T *pj, T Mj, const double (&wg)[D]) {
    T e = (T)0;
    for (int k = 0; k < D; k++) {
        const T dv = pj[1 + k] - (T)wg[k];
        e += dv * dv;
    }
    return pj[0] > (T)0 ? (T)0.5 * Mj * e : (T)0;
}

// The gradient kernel's window (mixed mode): the primitive records of the
// kGWin cells centred on its block's 64 cells, staged in LDS once per block.
// Cells are in Morton order, so most neighbours of a block's cells fall
// inside it (about 60% on a Poisson mesh); the rest are gathered from HBM.
constexpr int kGWin = 128;
// W of neighbour j (its primitive record's first D + 2 values): from the
// window when it holds j, else from the records prim.
template <int D, typename T>
__device__ __forceinline__ void load_nb(const T *__restrict__ prim, int64_t j, const float *win, int64_t c0,
                                        T (&o)[D + 2]) {
    constexpr int NJ = D + 2, PREC = Lay<D>::PREC;
    if constexpr (sizeof(T) == 4) {
        const int64_t k = j - c0;
        if (win && k >= 0 && k < kGWin) {
            load_rec_lds<NJ>((lds_cfloat *)win + k * PREC, o);
            return;
        }
    }
    load_rec<NJ>(prim + j * PREC + Lay<D>::W, o);
}

// The mass rho_j V_j of neighbour j in the records' precision (energy
// switch), rho_j its record's density: from the window's masses mwin (the
// same product, formed once per window cell) when it holds j, else formed here.
template <typename T>
__device__ __forceinline__ T nb_mass(const double *__restrict__ V, int64_t j, T rho, const float *mwin, int64_t c0) {
    const int64_t k = j - c0;
    if constexpr (sizeof(T) == 4)
        if (mwin && k >= 0 && k < kGWin) return ((lds_cfloat *)mwin)[k];
    return rho * (T)V[j];
}

// The gradient and limiter of cell i by its lane group (lane = index in
// the group); every lane of the group calls it with the same i. The
// neighbours' W come from their primitive records. With ESW, also the
// energy switch's largest kinetic energy of the cell and its neighbours in
// the frame of the cell's generator, into ekmax[i] (the states are the step's start states,
// those the gradient is taken from; mvel the generator velocities, w0 the
// mixed mode's reference velocity). win: the block's window of primitive
// records, starting at cell c0 (null: every record from HBM); vwin the
// window's volumes.
template <int D, typename T, bool ESW = false>
__device__ __forceinline__ void grad_cell(int64_t i, int lane, const int32_t *__restrict__ off,
                                          const int32_t *__restrict__ nbr, const T *__restrict__ srec,
                                          const double *__restrict__ V, const T *__restrict__ prim,
                                          T *__restrict__ grad_out, const double *__restrict__ mvel = nullptr,
                                          const double *__restrict__ w0 = nullptr, int64_t n = 0,
                                          T *__restrict__ ekmax = nullptr, const float *win = nullptr,
                                          int64_t c0 = 0, const float *mwin = nullptr) {
    using Y = Lay<D>;
    constexpr int NV = D + 2;
    constexpr int GS = Group<D>::GS;
    constexpr bool mixed = sizeof(T) == 4;
    constexpr int KR = mixed ? (ESW ? 3 : 5) : 3;   // sides per lane held in registers
    constexpr int SR = mixed ? Y::SREC32 : Y::SREC64;
    constexpr int NJ = NV;   // values read of a neighbour: its W
    const T eps_t = mixed ? (T)1e-6 : (T)1e-13;
    const int32_t b = off[i], e = off[i + 1];
    // the lane's first KR sides: side records and neighbour indices, then
    // the neighbours' records, all in flight together (an absent side reads
    // record 0 of the arrays and is skipped)
    T sr[KR][SR], pj[KR][NJ];
    T vj[KR];
    bool has[KR];
    for (int r = 0; r < KR; r++) {
        const int32_t q = b + lane + r * GS;
        has[r] = q < e;
        const int32_t qq = has[r] ? q : 0;
        load_rec<SR>(srec + (int64_t)qq * SR, sr[r]);
        const int32_t jn = nbr[qq];
        load_nb<D, T>(prim, jn, win, c0, pj[r]);
        if constexpr (ESW) vj[r] = nb_mass<T>(V, jn, pj[r][0], mwin, c0);
    }
    T pi[Y::PREC];
    load_rec<Y::PREC>(prim + i * Y::PREC, pi);
    const T *wi = pi + Y::W;
    const T *dl = pi + Y::DL;
    SideAcc<D, T> a;
    for (int c = 0; c < NV; c++) {
        a.dmx[c] = (T)0;
        a.dmn[c] = (T)0;
        for (int k = 0; k < D; k++) a.acc[c][k] = (T)0;
    }
    double wlab[D];
    T ek = (T)0;
    if constexpr (ESW)   // the cell's generator velocity, in the records' frame
        for (int k = 0; k < D; k++) wlab[k] = mixed ? mvel[k * n + i] - w0[k] : mvel[k * n + i];
    for (int r = 0; r < KR; r++)
        if (has[r]) {
            grad_side<D, T>(sr[r], pj[r], wi, a);
            if constexpr (ESW) ek = fmax(ek, ekin_in_frame<D, T>(pj[r], vj[r], wlab));
        }
    for (int32_t q = b + lane + KR * GS; q < e; q += GS) {
        T s2[SR], p2[NJ];
        load_rec<SR>(srec + (int64_t)q * SR, s2);
        const int32_t j = nbr[q];
        load_nb<D, T>(prim, j, win, c0, p2);
        grad_side<D, T>(s2, p2, wi, a);
        if constexpr (ESW) ek = fmax(ek, ekin_in_frame<D, T>(p2, nb_mass<T>(V, j, p2[0], mwin, c0), wlab));
    }
    if constexpr (ESW) {   // with the cell's own, in the same frame and precision
        ek = grp_max<GS>(ek);
        if (lane == 0) ekmax[i] = fmax(ek, ekin_in_frame<D, T>(wi, wi[0] * (T)V[i], wlab));
    }
    const T inv_v = (T)(1.0 / V[i]);
    T grad[NV][D], dmx[NV], dmn[NV];
    for (int c = 0; c < NV; c++) {
        for (int k = 0; k < D; k++) grad[c][k] = grp_sum<GS>(a.acc[c][k]) * inv_v;
        dmx[c] = grp_max<GS>(a.dmx[c]);
        dmn[c] = grp_min<GS>(a.dmn[c]);
    }
    T up[NV], dn[NV], tol[NV];
    for (int c = 0; c < NV; c++) {
        up[c] = (T)0;
        dn[c] = (T)0;
        const T av = wi[c] < (T)0 ? -wi[c] : wi[c];
        const T range = dmx[c] - dmn[c];
        tol[c] = eps_t * (av > range ? av : range);
    }
    for (int r = 0; r < KR; r++)
        if (has[r]) limit_side<D, T>(sr[r] + 1, dl, grad, up, dn);
    for (int32_t q = b + lane + KR * GS; q < e; q += GS) {
        T s2[SR];
        load_rec<SR>(srec + (int64_t)q * SR, s2);
        limit_side<D, T>(s2 + 1, dl, grad, up, dn);
    }
    T alpha[NV];
    for (int c = 0; c < NV; c++) {
        up[c] = grp_max<GS>(up[c]);   // max Dl (>= 0)
        dn[c] = grp_min<GS>(dn[c]);   // min Dl (<= 0)
        T al = (T)1;
        if (up[c] > tol[c]) { T p = dmx[c] / up[c]; al = p < al ? p : al; }
        if (dn[c] < -tol[c]) { T p = dmn[c] / dn[c]; al = p < al ? p : al; }
        alpha[c] = al;
    }
    if (lane == 0) {
        T go[Y::GREC];
        for (int k = 0; k < Y::GREC; k++) go[k] = (T)0;
        for (int c = 0; c < NV; c++)
            for (int k = 0; k < D; k++) go[c * D + k] = alpha[c] * grad[c][k];
        store_rec<Y::GREC>(grad_out + i * Y::GREC, go);
    }
}

// The gather-bound gradient kernels gain from one more wavefront per SIMD
// than the register count the compiler picks on its own (5 float / 4 double,
// about 7-9% faster; the 3D double kernel spills a few bytes per lane). The
// float kernels hold 5 sides per lane in registers, 3 with the energy
// switch's neighbour energies, without spills at 5 and (with the switch) 7
// wavefronts per SIMD (a spill of 32 bytes per lane once cost the float
// kernel about 20%; the switch's kernel at 7 is 1% faster per step than at
// 6); the double kernel with the switch runs at 3.
// With dt_out, block 0 also reduces the Courant pass's nparts block minima
// dt_part to the global timestep (the face pass after it reads it).
template <int D, typename T, bool ESW>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? (ESW ? 7 : 5) : (ESW ? 3 : 4))))
k_grad_limit(int64_t n, const int32_t *__restrict__ off, const int32_t *__restrict__ nbr, const T *__restrict__ srec,
             const double *__restrict__ V, const T *__restrict__ prim, T *__restrict__ grad_out,
             const double *__restrict__ mvel, const double *__restrict__ w0, T *__restrict__ ekmax,
             const double *__restrict__ dt_part, int64_t nparts, double *__restrict__ dt_out) {
    constexpr int GS = Group<D>::GS;
    if (dt_out && blockIdx.x == 0) {   // the whole block, before any group leaves
        double v = INFINITY;
        for (int64_t k = threadIdx.x; k < nparts; k += kBlock) v = fmin(v, dt_part[k]);
        v = block_min(v);
        if (threadIdx.x == 0) *dt_out = v;
    }
    const int64_t i = xcd_tile() * (kBlock / GS) + threadIdx.x / GS;
    // mixed mode: stage the window (every lane takes part in the copy and the
    // barrier before any group leaves)
    const float *win = nullptr;
    const float *mwin = nullptr;
    int64_t c0 = 0;
    if constexpr (sizeof(T) == 4) {
        constexpr int PREC = Lay<D>::PREC;
        __shared__ float wbuf[kGWin * PREC];
        c0 = xcd_tile() * (kBlock / GS) - (kGWin - kBlock / GS) / 2;
        for (int e = threadIdx.x; e < kGWin * PREC / 4; e += kBlock) {
            const int64_t j = c0 + e / (PREC / 4);
            f32x4u v = {0.0f, 0.0f, 0.0f, 0.0f};
            if (j >= 0 && j < n) v = *reinterpret_cast<const f32x4u *>((const float *)prim + j * PREC + (e % (PREC / 4)) * 4);
            *reinterpret_cast<f32x4u *>(wbuf + e * 4) = v;
        }
        if constexpr (ESW) {   // and the window's masses rho_j V_j
            __shared__ float mbuf[kGWin];
            for (int e = threadIdx.x; e < kGWin; e += kBlock) {
                const int64_t j = c0 + e;
                mbuf[e] = (j >= 0 && j < n) ? ((const float *)prim)[j * PREC + Lay<D>::W] * (float)V[j] : 0.0f;
            }
            mwin = mbuf;
        }
        __syncthreads();
        win = wbuf;
    }
    if (i >= n) return;  // whole groups leave together
    grad_cell<D, T, ESW>(i, threadIdx.x % GS, off, nbr, srec, V, prim, grad_out, mvel, w0, n, ekmax, win, c0, mwin);
}

// The total entropy of every cell from its conserved state (Section 3.5):
// S = M P / rho^gamma with P = (gamma-1)(E - |p|^2/(2M))/V; 0 for M <= 0.
// Q is [D+3][N], row D+2 written.
template <int D>
__global__ void __launch_bounds__(kBlock) k_entropy_init(int64_t n, const double *__restrict__ V, double gamma,
                                                         double *__restrict__ Q) {
    constexpr int NV = D + 2;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double m = Q[i];
    double S = 0.0;
    if (m > 0.0) {
        double p2 = 0.0;
        for (int k = 0; k < D; k++) p2 += Q[(1 + k) * n + i] * Q[(1 + k) * n + i];
        const double vol = V[i], rho = m / vol;
        const double P = (gamma - 1.0) * (Q[(NV - 1) * n + i] - 0.5 * p2 / m) / vol;
        S = m * P / mm_pow(rho, gamma);
    }
    Q[NV * n + i] = S;
}

// Mesh motion (Section 3.2, eq. eqnvelmesh, and Section 4.1, eq.
// EqnShapeCorrVel): each generator moves with its cell's fluid velocity,
// w_i = v_i (0 in a vacuum cell), plus chi times a pull towards the cell's
// centre of mass: with d = |s_i - r_i|, R_i the radius of a sphere (3D) or
// disc (2D) of the cell's volume and x = d / (eta R_i), none for x < 0.9,
// c_i (s_i - r_i)/d scaled by (d - 0.9 eta R_i)/(0.2 eta R_i) for
// 0.9 <= x < 1.1, and c_i (s_i - r_i)/d above, c_i the sound speed (0 in a
// vacuum cell); with dt_lloyd > 0, (s_i - r_i)/dt_lloyd replaces
// c_i (s_i - r_i)/d. w_out [D][N].
template <int D>
__global__ void __launch_bounds__(kBlock) k_mesh_velocity(int64_t n, const double *__restrict__ Q,
                                                          const double *__restrict__ V,
                                                          const double *__restrict__ coff, double gamma, double eta,
                                                          double chi, double dt_lloyd, double *__restrict__ w_out) {
    constexpr int NV = D + 2;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double m = Q[i], vol = V[i];
    double v[D], sr[D], d2 = 0.0, c = 0.0;
    for (int k = 0; k < D; k++) {
        sr[k] = coff[k * n + i];
        d2 += sr[k] * sr[k];
        v[k] = 0.0;
    }
    if (m > 0.0) {
        double p2 = 0.0;
        for (int k = 0; k < D; k++) {
            v[k] = Q[(1 + k) * n + i] / m;
            p2 += v[k] * v[k];
        }
        const double rho = m / vol;
        const double P = (gamma - 1.0) * (Q[(NV - 1) * n + i] - 0.5 * m * p2) / vol;
        if (rho > 0.0 && P > 0.0) c = sqrt(gamma * P / rho);
    }
    const double d = sqrt(d2);
    const double R = (D == 3) ? cbrt(3.0 * vol / (4.0 * M_PI)) : sqrt(vol / M_PI);
    const double x = d / (eta * R);
    const double frac = x >= 1.1 ? 1.0 : (x >= 0.9 ? (d - 0.9 * eta * R) / (0.2 * eta * R) : 0.0);
    for (int k = 0; k < D; k++) {
        double corr = 0.0;
        if (frac > 0.0) corr = dt_lloyd > 0.0 ? sr[k] / dt_lloyd : c * sr[k] / d;
        w_out[k * n + i] = v[k] + chi * frac * corr;
    }
}

// Volume rate of every cell from the face velocities of the uploaded mesh
// (Section 3.3, eq. eqnvolchange): dV_i/dt = sum over the cell's faces of
// +- A_f w_f . n_f, + where the cell is the face's left cell (the normal
// points out of it). One lane group per cell, a fixed summation order.
template <int D>
__global__ void __launch_bounds__(kBlock) k_volume_rate(int64_t n, const int32_t *__restrict__ off,
                                                        const int32_t *__restrict__ ent,
                                                        const double *__restrict__ frec,
                                                        const double *__restrict__ wf64, double *__restrict__ rate) {
    using Y = Lay<D>;
    constexpr int GS = Group<D>::GS;
    const int lane = threadIdx.x % GS;
    const int64_t i = xcd_tile() * (kBlock / GS) + threadIdx.x / GS;
    if (i >= n) return;
    double acc = 0.0;
    for (int32_t q = off[i] + lane; q < off[i + 1]; q += GS) {
        const int32_t en = ent[q];
        double fr[Y::FREC], w[D];
        load_rec<Y::FREC>(frec + (int64_t)(en >> 1) * Y::FREC, fr);
        load_rec<Y::WSTRIDE>(wf64 + (int64_t)(en >> 1) * Y::WSTRIDE, w);
        double wn = 0.0;
        for (int k = 0; k < D; k++) wn += w[k] * fr[Y::FN + k];
        acc += ((en & 1) ? -1.0 : 1.0) * fr[Y::FA] * wn;
    }
    acc = grp_sum<GS>(acc);
    if (lane == 0) rate[i] = acc;
}

}  // namespace mm
