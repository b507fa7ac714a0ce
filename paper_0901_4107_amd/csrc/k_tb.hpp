// k_tb.hpp -- individual power-of-two timesteps (Section 7.2): the kernels
// of one synchronisation point besides the flux passes, which run the
// shared face bodies over lists (k_face_flux*_list).
//
// Time is counted in ticks of dt_max / 2^levels. A cell in bin b takes
// steps of 2^b ticks that start at multiples of 2^b. The timeline's state
// lives on the device (the info block: current tick, path of the next
// point, counts per bin, the stop tick of the current batch), so the kernels
// of a point take the same arguments at every point and a batch of points
// runs without the host: a point whose tick has reached the stop tick, or
// follows a failed criterion, does nothing. At tick ti:
//   k_tb_open    per cell     the cells whose step ends now become active:
//                             primitive and signal records, trec = ti, and
//                             a split list of them
//   k_tb_active  lane group   neighbour signal-speed criterion and the bin
//                per active   rules (occupancy counts per bin), the
//                cell         gradient, and on sparse points the active faces
//                             from the cell's side list (every face of an
//                             active cell is active) and the touched cells
//   k_tb_faces   per face     (dense points) a face is active when the
//                             smaller step of its cells starts now: split
//                             list, and both cells stamped as touched
//   (fluxes of the active faces, each over its own step)
//   k_tb_update  lane group   touched cells add the signed, time-integrated
//                per cell     fluxes of their active faces (all cells with
//                             a stamp check, or the touched list)
//   k_tb_finish  one block    list sizes and totals for the host, the next
//                             tick and the next point's path; clears the
//                             lists for the next point
#pragma once

#include "common.hpp"
#include "k_cell.hpp"
#include "k_update.hpp"
#include "layout.hpp"

namespace mm {

constexpr int kTbMaxLevels = 30;
__device__ __forceinline__ bool tb_starts(int64_t ti, int b) { return (ti & ((int64_t(1) << b) - 1)) == 0; }
// Start of a timeline: the counters of up to four split lists (null ones
// skipped), the error slot and the non-finite flag.
__global__ void __launch_bounds__(kBlock) k_tb_reset(int32_t *l0, int32_t *l1, int32_t *l2, int32_t *l3,
                                                     int32_t *info, int32_t *step_flag) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < kLists) {
        if (l0) l0[t * kListPad] = 0;
        if (l1) l1[t * kListPad] = 0;
        if (l2) l2[t * kListPad] = 0;
        if (l3) l3[t * kListPad] = 0;
    }
    if (t == 0) {
        info[TB_ERR] = 0;
        *step_flag = 0;
    }
}

// Per residue class of the per-cell grid (the cells whose k_tb_open block
// appends to active sub-list c), the sum of the cells' side counts and the
// number of cells: bounds on what the sparse path appends to face and
// touched sub-list c. A block here covers one tile of the per-cell grid,
// whose cells share a class: one block sum, one atomic pair.
__global__ void __launch_bounds__(kBlock) k_tb_bound(int64_t n, unsigned grid, const int32_t *__restrict__ off,
                                                     int32_t *__restrict__ sides, int32_t *__restrict__ cells) {
    __shared__ int32_t red[2][kBlock / 64];
    const int64_t t = blockIdx.x, i = t * kBlock + threadIdx.x;
    int32_t d = i < n ? off[i + 1] - off[i] : 0, one = i < n ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) {
        d += __shfl_xor(d, o, 64);
        one += __shfl_xor(one, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x / 64] = d;
        red[1][threadIdx.x / 64] = one;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; w++) {
            d += red[0][w];
            one += red[1][w];
        }
        // the block b of a grid of `grid` blocks whose xcd_tile() is tile t
        const int64_t per = grid / kXcd;
        const int64_t b = (t % per) * kXcd + t / per;
        const int c = (int)(b % kLists);
        atomicAdd(sides + c, d);
        atomicAdd(cells + c, one);
    }
}

// A fresh timeline: every cell in the top bin with its step starting at
// tick 0 (so every cell is active at the first point, a dense one), no cell
// touched, no stop tick.
__global__ void __launch_bounds__(kBlock) k_tb_init(int64_t n, int32_t levels, int8_t *__restrict__ bin,
                                                    int64_t *__restrict__ trec, int32_t *__restrict__ touch,
                                                    int32_t *__restrict__ info) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        bin[i] = (int8_t)levels;
        trec[i] = 0;
        touch[i] = -1;
    }
    if (i < TB_INFO_INTS) info[i] = (i == TB_COUNTS + levels) ? (int32_t)n : 0;
}

// Start of a batch: its stop tick and cleared totals.
__global__ void k_tb_batch(int32_t *info, int64_t until) {
    tb64(info, TB_UNTIL) = until;
    tb64(info, TB_SUMC) = 0;
    tb64(info, TB_SUMF) = 0;
    info[TB_NPTS] = 0;
    info[TB_NSPARSE] = 0;
    info[TB_NONFIN] = 0;
}

// Opens the step of every cell whose step ends at ti: its primitive record
// (as in the global step), its signal record (c, lab velocity, and the local
// bound R / (c + |v - w|), infinite for vacuum), trec = ti, and a place in
// the split list of active cells.
// The point runs (info[TB_LIVE], for the later kernels of the point) when
// the timeline has not halted and its tick is below the batch's stop tick.
template <int D, typename T>
__global__ void __launch_bounds__(kBlock) k_tb_open(int64_t n, int32_t *__restrict__ info,
                                                    const int8_t *__restrict__ bin, int64_t *__restrict__ trec,
                                                    double gamma, const double *__restrict__ V,
                                                    const double *__restrict__ Q, const double *__restrict__ mvel,
                                                    const double *__restrict__ coff, T *__restrict__ prim,
                                                    const double *__restrict__ w0, double *__restrict__ sig, int32_t *__restrict__ list,
                                                    int64_t cap) {
    using Y = Lay<D>;
    constexpr int SG = D + 2;
    const int64_t ti = tb64(info, TB_TI);
    const bool live = info[TB_ERR] == 0 && ti < tb64(info, TB_UNTIL);
    if (blockIdx.x == 0 && threadIdx.x == 0) info[TB_LIVE] = live;
    if (!live) return;   // the whole grid
    const int64_t i = xcd_global_id();
    bool act = false;
    if (i < n) {
        act = tb_starts(ti, bin[i]);
        if (act) {
            T r[Y::PREC];
            double v[D], rel2, R;
            bool ok;
            const double c = cell_prim<D, T>(i, n, gamma, V, Q, mvel, coff, w0, r, v, rel2, R, ok);
            store_rec<Y::PREC>(prim + i * Y::PREC, r);
            double s[SG];
            s[0] = c;
            for (int k = 0; k < D; k++) s[1 + k] = v[k];
            s[D + 1] = ok ? R / (c + sqrt(rel2)) : INFINITY;
            store_rec<SG>(sig + i * SG, s);
            trec[i] = ti;
        }
    }
    list_append(list, cap, act, (int32_t)i);
}

// The work of each active cell, by a lane group walking the cell's sides:
//  1. its criterion and bin (eq. EqnTiStepIndividual over the Voronoi
//     neighbours):
//       dt_i = C min(tau_i, R_i / (c_i + |v_i - w_i|)),
//       tau_i = min over faces of |d| / v_sig,
//       v_sig = c_L + c_R - (v_R - v_L).n
//     (a face with v_sig <= 0 sets no bound). The bin is the largest
//     b <= levels with dt_max 2^(b - levels) <= dt_i; the cell takes it if it
//     is not above its old bin, else moves up one bin where that bin starts
//     a step at ti, else keeps its bin. A criterion below one tick raises
//     info[TB_ERR] (the flux and update passes then do nothing) and leaves
//     the bin. Occupancy changes are gathered per block in LDS and added to
//     the counts once per block and bin;
//  2. its gradient and limiter (grad_cell, from the primitive records of
//     all cells: fresh for the active ones, of their last active step for
//     the rest);
//  3. on sparse points, its share of the active faces: every face
//     of an active cell is active, since its smaller step divides the active
//     cell's; a face is listed by its active cell if the other cell is
//     inactive, else by its left cell. The cell itself and its inactive
//     neighbours (once each, by the touch stamp exchanged to cur) go to the
//     touched list. Whether a neighbour is active does not depend on the bin
//     updates of step 1 racing with the read: an active cell's old and new
//     bins both start a step at ti.
template <int D, typename T>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 3)))
k_tb_active(const int32_t *__restrict__ list, int64_t cap, double dt_max, int32_t levels, double cfl,
            const int32_t *__restrict__ off, const int32_t *__restrict__ ent, const int32_t *__restrict__ nbr,
            const double *__restrict__ frec, const double *__restrict__ sig, int8_t *__restrict__ bin,
            int32_t *__restrict__ info, const T *__restrict__ srec, const double *__restrict__ V,
            const T *__restrict__ prim, T *__restrict__ grad_out,
            int32_t *__restrict__ touch,
            int32_t *__restrict__ faces, int64_t fcap, int32_t *__restrict__ touched, int64_t tcap) {
    using Y = Lay<D>;
    constexpr int SG = D + 2;
    constexpr int GS = Group<D>::GS, G = kBlock / GS;
    const int64_t ti = tb64(info, TB_TI);
    const int32_t cur = info[TB_CUR];
    const bool claim_faces = info[TB_SPARSE] != 0;
    __shared__ int32_t delta[kTbMaxLevels + 2];
    if (threadIdx.x < kTbMaxLevels + 2) delta[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x % GS;
    const int c = blockIdx.x % kLists;
    const int32_t *items = list + (int64_t)kLists * kListPad + c * cap;
    const int64_t count = list[c * kListPad];
    const int64_t stride = (int64_t)(gridDim.x / kLists) * G;
    const double tick = ldexp(dt_max, -levels);
    for (int64_t q = (int64_t)(blockIdx.x / kLists) * G + threadIdx.x / GS; q < count; q += stride) {
        const int64_t i = items[q];
        const int32_t e0 = off[i], e1 = off[i + 1];
        // 1
        double si[SG];
        load_rec<SG>(sig + i * SG, si);
        double tau = INFINITY;
        for (int32_t e = e0 + lane; e < e1; e += GS) {
            const int32_t en = ent[e];
            const int64_t f = en >> 1, j = nbr[e];
            const bool i_right = en & 1;
            double sj[SG], fr[1 + D];
            load_rec<SG>(sig + j * SG, sj);
            load_rec<1 + D>(frec + f * Y::FREC + Y::FELL, fr);   // |d|, n
            double du = 0.0;
            for (int k = 0; k < D; k++) {
                const double vR = i_right ? si[1 + k] : sj[1 + k], vL = i_right ? sj[1 + k] : si[1 + k];
                du += (vR - vL) * fr[1 + k];
            }
            const double vsig = (si[0] + sj[0]) - du;
            if (vsig > 0.0) tau = fmin(tau, fr[0] / vsig);
        }
        tau = grp_min<GS>(tau);
        if (lane == 0) {
            const double dti = cfl * fmin(tau, si[D + 1]);
            if (!(dti >= tick)) {
                atomicOr(info + TB_ERR, 1);
            } else {
                int b = levels;
                while (b > 0 && ldexp(dt_max, b - levels) > dti) b--;
                const int old = bin[i];
                int nb = old;
                if (b <= old) nb = b;
                else if (tb_starts(ti, old + 1)) nb = old + 1;
                if (nb != old) {
                    bin[i] = (int8_t)nb;
                    atomicAdd(&delta[old], -1);
                    atomicAdd(&delta[nb], 1);
                }
            }
        }
        // 2
        grad_cell<D, T>(i, lane, off, nbr, srec, V, prim, grad_out);
        // 3
        if (claim_faces) {   // the same for the whole grid
            list_append(touched, tcap, lane == 0, (int32_t)i);
            for (int32_t e = e0 + lane; __any(e < e1); e += GS) {
                bool claim = false, fresh = false;
                int32_t f = 0, j = 0;
                if (e < e1) {
                    const int32_t en = ent[e];
                    f = en >> 1;
                    j = nbr[e];
                    const bool j_active = tb_starts(ti, bin[j]);
                    claim = !j_active || !(en & 1);
                    if (!j_active && touch[j] != cur) fresh = atomicExch(touch + j, cur) != cur;
                }
                list_append(faces, fcap, claim, f);
                list_append(touched, tcap, fresh, j);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x <= (unsigned)levels && delta[threadIdx.x] != 0)
        atomicAdd(info + TB_COUNTS + threadIdx.x, delta[threadIdx.x]);
}

// Dense points: active faces are those whose smaller step starts at ti
// (then one of their cells is active). Lists them and stamps both cells as
// touched at this point. A fixed grid strides over the faces, so that on
// sparse points (and halted or finished ones) it leaves at once.
__global__ void __launch_bounds__(kBlock) k_tb_faces(int64_t nf, const int32_t *__restrict__ fL,
                                                     const int32_t *__restrict__ fR, const int8_t *__restrict__ bin,
                                                     const int32_t *__restrict__ info, int32_t *__restrict__ touch,
                                                     int32_t *__restrict__ list, int64_t cap) {
    if (!info[TB_LIVE] || info[TB_SPARSE] || info[TB_ERR]) return;
    const int64_t ti = tb64(info, TB_TI);
    const int32_t cur = info[TB_CUR];
    for (int64_t base = (int64_t)blockIdx.x * kBlock; base < nf; base += (int64_t)gridDim.x * kBlock) {
        const int64_t f = base + threadIdx.x;
        bool act = false;
        if (f < nf) {
            const int32_t l = fL[f], r = fR[f];
            const int bl = bin[l], br = bin[r];
            act = tb_starts(ti, bl < br ? bl : br);
            if (act) {
                touch[l] = cur;
                touch[r] = cur;
            }
        }
        list_append(list, cap, act, (int32_t)f);
    }
}

// Where a cell's faces are, for the update (k_update.hpp): its left range,
// its right-cell slots and their faces, and every face's two cells.
struct TbSides {
    const int32_t *lOff, *rOff, *rFace, *fL, *fR;
};

// The update of a touched cell i by its lane group: Q_i changes by the
// time-integrated fluxes of its active faces (a face is active when the
// smaller step of its two cells starts at ti), in the global update's
// order (k_update.hpp), inactive faces adding nothing; so that a point at
// which every cell is active is the global step bit for bit. A non-finite
// result raises flags[0] and flags[1] like the global update.
template <int D>
__device__ __forceinline__ void tb_update_cell(int64_t i, int lane, int64_t n, const TbSides &sd,
                                               const int8_t *__restrict__ bin, int64_t ti,
                                               const double *__restrict__ flux, double *__restrict__ Q,
                                               int32_t *__restrict__ flags) {
    constexpr int NV = D + 2;
    auto live = [&](int32_t f) {
        const int bl = bin[sd.fL[f]], br = bin[sd.fR[f]];
        return tb_starts(ti, bl < br ? bl : br);
    };
    double acc[NV], mx;
    cell_sums<D, 0>(i, lane, sd.lOff, sd.rOff, sd.rFace, flux, live, acc, mx);
    if (lane == 0) {
        UpdateArgs u{};
        u.flags = flags;
        finish_cell<D, 0, false>(i, n, acc, 0.0, Q, u);
    }
}

// Dense points: every cell, those not stamped at this point leaving at
// once; a fixed grid of lane groups strides over the cells.
template <int D>
__global__ void __launch_bounds__(kBlock) k_tb_update(int64_t n, TbSides sd, const int8_t *__restrict__ bin,
                                                      const int32_t *__restrict__ info,
                                                      const int32_t *__restrict__ touch,
                                                      const double *__restrict__ flux, double *__restrict__ Q,
                                                      int32_t *__restrict__ flags) {
    constexpr int GS = Group<D>::GS, G = kBlock / GS;
    if (!info[TB_LIVE] || info[TB_SPARSE] || info[TB_ERR]) return;
    const int64_t ti = tb64(info, TB_TI);
    const int32_t cur = info[TB_CUR];
    for (int64_t i = (int64_t)blockIdx.x * G + threadIdx.x / GS; i < n; i += (int64_t)gridDim.x * G)
        if (touch[i] == cur) tb_update_cell<D>(i, threadIdx.x % GS, n, sd, bin, ti, flux, Q, flags);
}

// Sparse points: the cells of the touched list.
template <int D>
__global__ void __launch_bounds__(kBlock) k_tb_update_list(const int32_t *__restrict__ list, int64_t cap, int64_t n,
                                                           TbSides sd, const int8_t *__restrict__ bin,
                                                           const double *__restrict__ flux, double *__restrict__ Q,
                                                           int32_t *__restrict__ flags,
                                                           const int32_t *__restrict__ info) {
    constexpr int GS = Group<D>::GS, G = kBlock / GS;
    if (!info[TB_LIVE] || !info[TB_SPARSE] || info[TB_ERR]) return;
    const int64_t ti = tb64(info, TB_TI);
    const int c = blockIdx.x % kLists;
    const int32_t *items = list + (int64_t)kLists * kListPad + c * cap;
    const int64_t count = list[c * kListPad];
    const int64_t stride = (int64_t)(gridDim.x / kLists) * G;
    for (int64_t q = (int64_t)(blockIdx.x / kLists) * G + threadIdx.x / GS; q < count; q += stride)
        tb_update_cell<D>(items[q], threadIdx.x % GS, n, sd, bin, ti, flux, Q, flags);
}

// End of a point: on a point that ran and did not halt, the sizes of its
// active-cell and active-face lists, the batch totals, the occupied bins,
// the next tick (the next multiple of the smallest occupied bin's step),
// the next point's path (sparse when sparse_ok and at most 1/8 of the cells
// are due then) and the next touch stamp. Always: the point's non-finite
// flag into the batch's, and the counters of the point's lists (hard may be
// null) and the flag cleared for the next point.
__global__ void __launch_bounds__(kBlock) k_tb_finish(int64_t n, int32_t levels, int32_t sparse_ok,
                                                      int32_t *__restrict__ cells, int32_t *__restrict__ faces,
                                                      int32_t *__restrict__ touched, int32_t *__restrict__ hard,
                                                      int32_t *__restrict__ step_flag, int32_t *__restrict__ info) {
    __shared__ int32_t red[2][kBlock / 64];
    int32_t a = 0, b = 0;
    for (int c = threadIdx.x; c < kLists; c += kBlock) {
        a += cells[c * kListPad];
        b += faces[c * kListPad];
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x / 64] = a;
        red[1][threadIdx.x / 64] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; w++) {
            a += red[0][w];
            b += red[1][w];
        }
        info[TB_NONFIN] |= *step_flag;
        if (info[TB_LIVE] && !info[TB_ERR]) {
            const int64_t ti = tb64(info, TB_TI);
            int lo = -1, hi = -1;
            for (int k = 0; k <= levels; k++)
                if (info[TB_COUNTS + k] > 0) {
                    if (lo < 0) lo = k;
                    hi = k;
                }
            if (lo < 0) lo = 0;   // the counts always hold every cell; never shift by a negative bin
            const int64_t next = ((ti >> lo) + 1) << lo;
            int64_t due = 0;
            for (int k = 0; k <= levels; k++)
                if (tb_starts(next, k)) due += info[TB_COUNTS + k];
            info[TB_CELLS] = a;
            info[TB_FACES] = b;
            info[TB_LO] = lo;
            info[TB_HI] = hi;
            info[TB_LASTSPARSE] = info[TB_SPARSE];
            info[TB_NSPARSE] += info[TB_SPARSE];
            info[TB_SPARSE] = sparse_ok && 8 * due <= n;
            tb64(info, TB_SUMC) += a;
            tb64(info, TB_SUMF) += b;
            tb64(info, TB_LAST) = ti;
            tb64(info, TB_TI) = next;
            info[TB_NPTS] += 1;
            info[TB_CUR] += 1;
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < kLists; c += kBlock) {
        cells[c * kListPad] = 0;
        faces[c * kListPad] = 0;
        touched[c * kListPad] = 0;
        if (hard) hard[c * kListPad] = 0;
    }
    if (threadIdx.x == 0) *step_flag = 0;
}

}  // namespace mm
