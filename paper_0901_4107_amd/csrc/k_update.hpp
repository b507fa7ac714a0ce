// k_update.hpp -- step (vii), the conservative update (Section 3, eq.
// eqnupdate): each cell loses the fluxes of the faces where it is the left
// cell and gains those where it is the right cell.
//
// Faces are sorted by their left cell, so the faces of which cell i is the
// left cell form the contiguous range [lOff_i, lOff_{i+1}) of the face
// records: a wavefront's cells read one contiguous stretch of records for
// their left sides. The right sides are the faces rFace[rOff_i ...], in
// ascending face order, gathered. Lane l of the cell's group of GS lanes
// sums, from 0, minus the left faces lOff_i + l, + GS, ... and then plus
// the right faces of slots rOff_i + l, + GS, ...; the group's butterfly sum
// is added to Q_i. Every path (the step, the split entry points, the
// individual timesteps) uses this order, so they give the same bits.
//
// Records (face-major, written by the face kernels). EM is the entropy
// mode (0 off, 1 Mach switch, 2 energy switch). A face's values: the D + 2
// fluxes, then (EM >= 1) the entropy flux, then (EM == 1) the face's shock
// Mach number. The energy switch's neighbour energies come from the
// gradient pass (ekmax, one per cell).
#pragma once

#include "common.hpp"
#include "k_cell.hpp"
#include "layout.hpp"

namespace mm {

template <int D, int EM> struct Rec {
    static constexpr int NV = D + 2;
    static constexpr int NS = NV + (EM ? 1 : 0);                      // summed values
    static constexpr int MACH = NV + 1;                               // a maximum (EM == 1)
    static constexpr int FM = NV + (EM == 1 ? 2 : (EM == 2 ? 1 : 0)); // record stride
};

// What the end of a cell's update needs besides the sums.
struct UpdateArgs {
    int32_t *flags;            // [0] since the diagnostics' reset, [1] this step
    const double *V;
    double gamma, mach_thresh;
    DiagDev *diag;
    const double *accel;       // static field [D][n] or null
    const double *dt_ptr;      // timestep of the flux pass (device) or null
    double dt_val;             // ... or its value
    double alpha_s, beta_s;    // energy switch
    const double *ekmax;       // energy switch: the gradient pass's largest kinetic energy per cell,
    const float *ekmax32;      // ... or, in the mixed mode, the same in float
};

// The end of cell i's update, by lane 0 of its group: Q_i <- Q_i + acc,
// then the static field's sources (Section 5.2, a static field g = accel
// [D][n]: p += (dt/2)(M^n + M^(n+1)) g and E += (dt/2)(p^n + p^(n+1)).g, dt
// of the flux pass) and the entropy treatment (Section 3.5: a cell keeps
// its advected entropy, P = (S/M) rho^gamma and E = P V/(gamma-1) +
// |p|^2/(2M), when it is cold -- its largest face Mach number below
// mach_thresh (EM == 1), or its new thermal energy E - |p|^2/(2M) below
// alpha_s times the largest neighbour kinetic energy in its generator's
// frame, or with a field below beta_s M |g| R (EM == 2) -- and its new mass
// and entropy are positive; every other cell takes S = M P / rho^gamma of
// its updated state, 0 for M <= 0).
// mx: the largest face Mach number; the largest kinetic energy of the cell
// and its neighbours in the cell's generator frame is the gradient pass's
// ekmax. Returns whether the cell kept its entropy.
template <int D, int EM, bool GRAV>
__device__ __forceinline__ bool finish_cell(int64_t i, int64_t n, const double *acc, double mx,
                                            double *__restrict__ Q, const UpdateArgs &u) {
    constexpr int NV = D + 2;
    constexpr int NS = Rec<D, EM>::NS;
    double q[NS];
    for (int c = 0; c < NS; c++) q[c] = Q[c * n + i] + acc[c];
    double ek = 0.0;
    if constexpr (EM == 2) ek = u.ekmax32 ? (double)u.ekmax32[i] : u.ekmax[i];
    if constexpr (GRAV) {
        const double hdt = 0.5 * (u.dt_ptr ? *u.dt_ptr : u.dt_val), m0 = Q[i];
        double work = 0.0;
        for (int k = 0; k < D; k++) {
            const double gk = u.accel[k * n + i], p0 = Q[(1 + k) * n + i];
            q[1 + k] += hdt * (m0 + q[0]) * gk;
            work += (p0 + q[1 + k]) * gk;
        }
        q[NV - 1] += hdt * work;
    }
    bool keep = false;
    if constexpr (EM != 0) {
        const double m = q[0], S = q[NV];
        double p2 = 0.0;
        for (int k = 0; k < D; k++) p2 += q[1 + k] * q[1 + k];
        bool cold = mx < u.mach_thresh;
        if constexpr (EM == 2) {
            const double eth = m > 0.0 ? q[NV - 1] - 0.5 * p2 / m : 0.0;
            cold = u.alpha_s > 0.0 && eth < u.alpha_s * ek;
            if constexpr (GRAV) {
                if (!cold && u.beta_s > 0.0) {
                    double g2 = 0.0;
                    for (int k = 0; k < D; k++) g2 += u.accel[k * n + i] * u.accel[k * n + i];
                    const double vol = u.V[i];
                    const double R = (D == 3) ? cbrt(vol * (3.0 / (4.0 * M_PI))) : sqrt(vol * (1.0 / M_PI));
                    cold = eth < u.beta_s * m * sqrt(g2) * R;
                }
            }
        }
        keep = cold && m > 0.0 && S > 0.0;
        if (!(m > 0.0)) {
            q[NV] = 0.0;
        } else {
            const double vol = u.V[i], rho = m / vol, ke = 0.5 * p2 / m;
            if (keep) {
                const double P = (S / m) * mm_pow(rho, u.gamma);
                q[NV - 1] = P * vol / (u.gamma - 1.0) + ke;
            } else {
                const double P = (u.gamma - 1.0) * (q[NV - 1] - ke) / vol;
                q[NV] = m * P / mm_pow(rho, u.gamma);
            }
        }
    }
    bool fin = true;
    for (int c = 0; c < NS; c++) {
        Q[c * n + i] = q[c];
        fin = fin && isfinite(q[c]);
    }
    if (!fin) {
        atomicOr(u.flags, 1);       // since the last diagnostics reset
        atomicOr(u.flags + 1, 1);   // this step
    }
    return keep;
}

// The cells that kept their entropy, one atomic per wavefront. Every lane of
// the wavefront whose group is live takes part; lane 0 of the wavefront
// holds the lowest cell index, so it is live too.
__device__ __forceinline__ void count_kept(bool keep, DiagDev *diag) {
    const unsigned long long kb = __ballot(keep);
    if (diag && (threadIdx.x & 63) == 0 && kb)
        atomicAdd(&diag[blockIdx.x & (kDiagSlots - 1)].entropy_kept, (unsigned long long)__popcll(kb));
}

// The sums of cell i by lane `lane` of its group (the individual
// timesteps' update; k_update below sums in the same order): acc = the
// lane's share (minus its left faces, plus its right faces, in that order),
// butterfly summed over the group; mx the group's largest face Mach number.
// live(f): whether face f takes part; the rest contribute nothing. Each lane keeps up to KL left and KR right records in flight
// together (3 and 3; 2 and 2 for the Mach switch's 56-byte records), the
// rest in loops; the order of the sums does not depend on KL and KR.
template <int D, int EM, typename Live>
__device__ __forceinline__ void cell_sums(int64_t i, int lane, const int32_t *__restrict__ lOff,
                                          const int32_t *__restrict__ rOff, const int32_t *__restrict__ rFace,
                                          const double *__restrict__ flux, Live live,
                                          double (&acc)[Rec<D, EM>::NS], double &mx) {
    using RC = Rec<D, EM>;
    constexpr int NS = RC::NS, FM = RC::FM;
    constexpr int GS = Group<D>::GS;
    constexpr int KL = EM == 1 ? 2 : 3, KR = EM == 1 ? 2 : 3;
    for (int c = 0; c < NS; c++) acc[c] = 0.0;
    mx = 0.0;
    const int32_t l0 = lOff[i], l1 = lOff[i + 1], r0 = rOff[i], r1 = rOff[i + 1];
    double FLr[KL][FM], FRr[KR][FM];
    bool hl[KL], hr[KR];
    int32_t fr[KR];
    for (int r = 0; r < KR; r++) {
        const int32_t q = r0 + lane + r * GS;
        fr[r] = q < r1 ? rFace[q] : 0;
    }
    for (int r = 0; r < KL; r++) {
        const int32_t f = l0 + lane + r * GS;
        hl[r] = f < l1 && live(f);
        load_rec<FM>(flux + (int64_t)(hl[r] ? f : 0) * FM, FLr[r]);
    }
    for (int r = 0; r < KR; r++) {
        hr[r] = r0 + lane + r * GS < r1 && live(fr[r]);
        load_rec<FM>(flux + (int64_t)(hr[r] ? fr[r] : 0) * FM, FRr[r]);
    }
    auto take = [&](const double *F, double sign) {
        for (int c = 0; c < NS; c++) acc[c] += sign * F[c];
        if constexpr (EM == 1) mx = fmax(mx, F[RC::MACH]);
    };
    for (int r = 0; r < KL; r++)
        if (hl[r]) take(FLr[r], -1.0);
    for (int32_t f = l0 + lane + KL * GS; f < l1; f += GS) {
        if (!live(f)) continue;
        double F[FM];
        load_rec<FM>(flux + (int64_t)f * FM, F);
        take(F, -1.0);
    }
    for (int r = 0; r < KR; r++)
        if (hr[r]) take(FRr[r], 1.0);
    for (int32_t q = r0 + lane + KR * GS; q < r1; q += GS) {
        const int32_t f = rFace[q];
        if (!live(f)) continue;
        double F[FM];
        load_rec<FM>(flux + (int64_t)f * FM, F);
        take(F, 1.0);
    }
    for (int c = 0; c < NS; c++) acc[c] = grp_sum<GS>(acc[c]);
    if constexpr (EM == 1) mx = grp_max<GS>(mx);
}

// The update (the step, mm_apply_update): one lane group per cell. A
// block's cells c0 .. c1-1 are the left cells of one contiguous stretch of
// faces, [lOff_c0, lOff_c1): the block copies up to CAP of its records into
// LDS with coalesced 16-byte loads, while each lane's first KR right
// records are already being gathered, and the left sums read them there (a
// longer stretch reads the rest from global memory); so do the right sums
// for the faces whose left cell is in the block (about half on a Poisson
// mesh whose faces all run from the lower cell index to the higher; the
// share, not the result, depends on the orientation). The
// sums keep cell_sums' order, so the bits are those of every other path.
// Measured at 128^3 against cell_sums' 3 + 3 records in flight from HBM:
// the plain step 1.013 -> 0.967 ms, the Mach switch's 1.243 -> 1.163, the
// energy switch's 1.162 -> 1.102.
// Per entropy mode: the stage's records, the right records each lane keeps
// in flight, and the wavefronts per SIMD the kernel is held to (20, 28 and
// 24 KB of LDS a block).
template <int EM> struct UpdStage;
template <> struct UpdStage<0> { static constexpr int CAP = 512, KR = 3, W = 7; };
template <> struct UpdStage<1> { static constexpr int CAP = 512, KR = 3, W = 5; };
template <> struct UpdStage<2> { static constexpr int CAP = 512, KR = 3, W = 5; };

template <int D, int EM, bool GRAV>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(UpdStage<EM>::W)))
k_update(int64_t n, const int32_t *__restrict__ lOff, const int32_t *__restrict__ rOff,
         const int32_t *__restrict__ rFace, const double *__restrict__ flux, double *__restrict__ Q, UpdateArgs u) {
    using RC = Rec<D, EM>;
    constexpr int NS = RC::NS, FM = RC::FM;
    constexpr int GS = Group<D>::GS;
    const int lane = threadIdx.x % GS;
    constexpr int KR = UpdStage<EM>::KR, CAP = UpdStage<EM>::CAP;
    constexpr int PIECES = (CAP * FM + 1) / 2;   // 16-byte pieces of a full stage
    constexpr int IT = (PIECES + kBlock - 1) / kBlock;
    __shared__ __align__(16) double stage[2 * PIECES];
    const int64_t c0 = xcd_tile() * (kBlock / GS);
    if (c0 >= n) return;   // the whole block
    const int64_t i = c0 + threadIdx.x / GS;
    const bool live = i < n;
    const int64_t c1 = (c0 + kBlock / GS < n) ? c0 + kBlock / GS : n;
    const int64_t ic = live ? i : c0;
    const int32_t s0 = lOff[c0], s1 = lOff[c1];
    const int32_t l0 = lOff[ic], l1 = live ? lOff[ic + 1] : l0;
    const int32_t r0 = rOff[ic], r1 = live ? rOff[ic + 1] : r0;
    const int32_t ns = (s1 - s0 < CAP) ? s1 - s0 : CAP;
    int32_t fr[KR];
    for (int r = 0; r < KR; r++) {
        const int32_t q = r0 + lane + r * GS;
        fr[r] = q < r1 ? rFace[q] : 0;
    }
    const int tot = ns * FM;
    const double *src = flux + (int64_t)s0 * FM;
    f64x2u piece[IT];
    for (int k = 0; k < IT; k++) {
        const int e = 2 * (k * kBlock + (int)threadIdx.x);
        if (e + 1 < tot) piece[k] = *reinterpret_cast<const f64x2u *>(src + e);
        else if (e < tot) piece[k] = f64x2u{src[e], 0.0};
    }
    // a right face whose left cell is in the block (about half of them)
    // has its record in the stage too: read there after the barrier
    double FRr[KR][FM];
    bool hr[KR], inst[KR];
    for (int r = 0; r < KR; r++) {
        hr[r] = r0 + lane + r * GS < r1;
        inst[r] = hr[r] && (uint32_t)(fr[r] - s0) < (uint32_t)ns;
        if (hr[r] && !inst[r]) load_rec<FM>(flux + (int64_t)fr[r] * FM, FRr[r]);
    }
    typedef double f64x2a __attribute__((ext_vector_type(2)));
    for (int k = 0; k < IT; k++) {
        const int e = 2 * (k * kBlock + (int)threadIdx.x);
        if (e < tot) *reinterpret_cast<f64x2a *>(stage + e) = f64x2a{piece[k][0], piece[k][1]};
    }
    __syncthreads();
    if (!live) return;
    for (int r = 0; r < KR; r++)
        if (inst[r])
            for (int c = 0; c < FM; c++) FRr[r][c] = stage[(fr[r] - s0) * FM + c];
    double acc[NS], mx = 0.0;
    for (int c = 0; c < NS; c++) acc[c] = 0.0;
    auto take = [&](const double *F, double sign) {
        for (int c = 0; c < NS; c++) acc[c] += sign * F[c];
        if constexpr (EM == 1) mx = fmax(mx, F[RC::MACH]);
    };
    for (int32_t f = l0 + lane; f < l1; f += GS) {
        double F[FM];
        const int32_t q = f - s0;
        if (q < ns) {
            for (int c = 0; c < FM; c++) F[c] = stage[q * FM + c];
        } else {
            load_rec<FM>(flux + (int64_t)f * FM, F);
        }
        take(F, -1.0);
    }
    for (int r = 0; r < KR; r++)
        if (hr[r]) take(FRr[r], 1.0);
    for (int32_t q = r0 + lane + KR * GS; q < r1; q += GS) {
        const int32_t f = rFace[q];
        double F[FM];
        if ((uint32_t)(f - s0) < (uint32_t)ns) {
            for (int c = 0; c < FM; c++) F[c] = stage[(f - s0) * FM + c];
        } else {
            load_rec<FM>(flux + (int64_t)f * FM, F);
        }
        take(F, 1.0);
    }
    for (int c = 0; c < NS; c++) acc[c] = grp_sum<GS>(acc[c]);
    if constexpr (EM == 1) mx = grp_max<GS>(mx);
    bool keep = false;
    if (lane == 0) keep = finish_cell<D, EM, GRAV>(i, n, acc, mx, Q, u);
    if constexpr (EM != 0) count_kept(keep, u.diag);
}

}  // namespace mm
