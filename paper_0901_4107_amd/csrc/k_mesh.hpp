// k_mesh.hpp -- device side of mm_mesh_upload: validation, each cell's left
// face range and sorted right faces, the face geometry and face velocities
// with the per-cell side lists of the gradient pass (left faces then right
// faces) written face by face, and the cells' closure test.
#pragma once

#include "common.hpp"
#include "k_cell.hpp"
#include "layout.hpp"

namespace mm {

enum MeshFlag : int {
    MF_INDEX = 1, MF_SELF = 2, MF_VOLUME = 4, MF_AREA = 8, MF_SEP = 16, MF_CTR = 32,
    MF_CENTROID = 64, MF_MESHVEL = 128, MF_OPEN = 256, MF_ORDER = 512
};

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_copy_i32(int32_t *dst, const int32_t *src, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_validate_faces(int64_t n, int64_t nf, const int32_t *L, const int32_t *R,
                                                           const double *area, const double *ctr, const double *sep,
                                                           int32_t *flags) {
    int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int bad = 0;
    if (f < nf) {
        int32_t l = L[f], r = R[f];
        if (l < 0 || l >= n || r < 0 || r >= n) bad |= MF_INDEX;
        if (l == r) bad |= MF_SELF;
        if (f > 0 && l < L[f - 1]) bad |= MF_ORDER;   // faces sorted by left cell
        double a = area[f];
        if (!(a >= 0.0) || !isfinite(a)) bad |= MF_AREA;
        double s2 = 0.0;
        bool fin = true, cfin = true;
        for (int k = 0; k < D; k++) {
            double d = sep[k * nf + f];
            fin = fin && isfinite(d);
            s2 += d * d;
            cfin = cfin && isfinite(ctr[k * nf + f]);
        }
        if (!fin || !(s2 > 0.0)) bad |= MF_SEP;
        if (!cfin) bad |= MF_CTR;
    }
    if (bad) atomicOr(flags, bad);
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_validate_cells(int64_t n, const double *volume, const double *coff,
                                                           const double *mvel, int32_t *flags) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int bad = 0;
    if (i < n) {
        double v = volume[i];
        if (!(v > 0.0) || !isfinite(v)) bad |= MF_VOLUME;
        for (int k = 0; k < D; k++) {
            if (!isfinite(coff[k * n + i])) bad |= MF_CENTROID;
            if (!isfinite(mvel[k * n + i])) bad |= MF_MESHVEL;
        }
    }
    if (bad) atomicOr(flags, bad);
}

// In-place inclusive scan of 1024-element tiles; tile totals go to bsum.
__global__ void __launch_bounds__(kBlock) k_scan_tiles(int32_t *data, int64_t n, int32_t *bsum) {
    __shared__ int32_t part[kBlock];
    const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
    int32_t v[4];
    int32_t run = 0;
    for (int q = 0; q < 4; q++) {
        int64_t i = base + q;
        run += (i < n) ? data[i] : 0;
        v[q] = run;
    }
    part[threadIdx.x] = run;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        int32_t t = (threadIdx.x >= (unsigned)off) ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += t;
        __syncthreads();
    }
    int32_t excl = part[threadIdx.x] - run;
    for (int q = 0; q < 4; q++) {
        int64_t i = base + q;
        if (i < n) data[i] = v[q] + excl;
    }
    if (threadIdx.x == kBlock - 1) bsum[blockIdx.x] = part[kBlock - 1];
}

__global__ void k_scan_add(int32_t *data, int64_t n, const int32_t *bsum_incl) {
    if (blockIdx.x == 0) return;
    const int32_t add = bsum_incl[blockIdx.x - 1];
    const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
    for (int q = 0; q < 4; q++) {
        int64_t i = base + q;
        if (i < n) data[i] += add;
    }
}

// Faces sorted by left cell: the first face of every cell's left range by
// binary search over face_L (loff [n + 1]; cells without left faces get the
// next range's start, loff[n] = nf).
__global__ void __launch_bounds__(kBlock) k_left_offsets(int64_t n, int64_t nf, const int32_t *__restrict__ L,
                                                         int32_t *__restrict__ loff) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i > n) return;
    int64_t lo = 0, hi = nf;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (L[mid] < i) lo = mid + 1;
        else hi = mid;
    }
    loff[i] = (int32_t)lo;
}

// rcnt[c] = number of faces whose right cell is c (rcnt points at roff + 1).
__global__ void k_count_right(int64_t nf, const int32_t *__restrict__ R, int32_t *__restrict__ rcnt) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f < nf) atomicAdd(&rcnt[R[f]], 1);
}

// Every face into its right cell's slots (any order; k_sort_right fixes it).
__global__ void k_place_right(int64_t nf, const int32_t *__restrict__ R, int32_t *__restrict__ cursor,
                              int32_t *__restrict__ rface) {
    const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f < nf) rface[atomicAdd(&cursor[R[f]], 1)] = (int32_t)f;
}

// Each cell's right faces in ascending face order, one thread per cell: up
// to 16 in registers through a bitonic sorting network, longer lists
// (rare) by insertion in memory. pos[f] = the slot of face f in rface.
__global__ void __launch_bounds__(kBlock) k_sort_right(int64_t n, const int32_t *__restrict__ roff,
                                                       int32_t *__restrict__ rface, int32_t *__restrict__ pos) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t b = roff[i], m = roff[i + 1] - b;
    if (m <= 16) {
        int32_t k[16];
#pragma unroll
        for (int j = 0; j < 16; j++) k[j] = j < m ? rface[b + j] : INT32_MAX;
#pragma unroll
        for (int size = 2; size <= 16; size <<= 1)
#pragma unroll
            for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
                for (int j = 0; j < 16; j++) {
                    const int p = j ^ stride;
                    if (p > j) {
                        const bool up = (j & size) == 0;
                        const int32_t x = k[j], y = k[p];
                        if ((x > y) == up) { k[j] = y; k[p] = x; }
                    }
                }
#pragma unroll
        for (int j = 0; j < 16; j++)
            if (j < m) {
                rface[b + j] = k[j];
                pos[k[j]] = b + j;
            }
    } else {
        for (int32_t a = b + 1; a < b + m; a++) {
            const int32_t key = rface[a];
            int32_t j = a - 1;
            while (j >= b && rface[j] > key) {
                rface[j + 1] = rface[j];
                j--;
            }
            rface[j + 1] = key;
        }
        for (int32_t a = b; a < b + m; a++) pos[rface[a]] = a;
    }
}

// Where the gradient pass's side lists put a face (each cell's left faces
// in face order, then its right faces in face order): its left side at
// f + roff[L], its right side at loff[R + 1] + pos[f] (pos from
// k_sort_right); per side ent = face << 1 | is_right, the neighbour, and
// the side record A/|d|, f - r_i = c +- (|d|/2) n (double or float).
struct SideOut {
    const int32_t *loff, *roff, *pos;
    int32_t *ent, *nbr;
    double *srec;    // double path, or
    float *srec32;   // mixed path
};

// Face records (Section 3.3 geometry and face velocity):
//   n = d/|d|, c = f - (r_L + r_R)/2 = g - d/2,
//   w_f = (w_L + w_R)/2 + [(w_L - w_R) . c / |d|] n.
// The double geometry record and the face velocity always; the float
// record and w_f - W0 (W0 at w0, into wrel) when mrec is given; with so.ent (the
// upload, not a change of velocities) also the face's two side records.
template <int D>
__global__ void __launch_bounds__(kBlock) k_face_records(int64_t n, int64_t nf, const int32_t *L, const int32_t *R,
                                                         const double *area, const double *ctr, const double *sep,
                                                         const double *mvel, double *frec, const double *w0,
                                                         float *mrec, float *wrel, double *wf64, SideOut so) {
    using Y = Lay<D>;
    int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f >= nf) return;
    int32_t l = L[f], r = R[f];
    double d[D], c[D], wl[D], wr[D], s2 = 0.0, proj = 0.0;
    for (int k = 0; k < D; k++) {
        d[k] = sep[k * nf + f];
        c[k] = ctr[k * nf + f] - 0.5 * d[k];
        s2 += d[k] * d[k];
        wl[k] = mvel[k * n + l];
        wr[k] = mvel[k * n + r];
    }
    for (int k = 0; k < D; k++) proj += (wl[k] - wr[k]) * c[k];
    const double ell = sqrt(s2);
    const double inv = 1.0 / ell;
    const double A = area[f];
    double o[Y::FREC];
    o[Y::FA] = A;
    o[Y::FELL] = ell;
    double w[D];
    for (int k = 0; k < D; k++) {
        o[Y::FN + k] = d[k] * inv;
        o[Y::FC + k] = c[k];
        w[k] = 0.5 * (wl[k] + wr[k]) + proj * d[k] / s2;
    }
    store_rec<Y::FREC>(frec + f * Y::FREC, o);
    store_rec<Y::WSTRIDE>(wf64 + f * Y::WSTRIDE, w);
    if (mrec) {
        float m[Y::MREC], wr[D];
        m[Y::FA] = (float)A;
        m[Y::FELL] = (float)ell;
        for (int k = 0; k < D; k++) {
            m[Y::FN + k] = (float)o[Y::FN + k];
            m[Y::FC + k] = (float)c[k];
            wr[k] = (float)(w[k] - w0[k]);
        }
        store_rec<Y::MREC>(mrec + f * Y::MREC, m);
        store_rec<D>(wrel + f * D, wr);
    }
    if (so.ent) {
        const int64_t q[2] = {f + so.roff[l], (int64_t)so.loff[r + 1] + so.pos[f]};
        const double hl = 0.5 * ell;
        for (int side = 0; side < 2; side++) {
            const double sg = side ? -1.0 : 1.0;
            double rec[Y::SREC64];
            rec[0] = A / ell;
            for (int k = 0; k < D; k++) rec[1 + k] = c[k] + sg * hl * o[Y::FN + k];
            for (int k = 1 + D; k < Y::SREC64; k++) rec[k] = 0.0;
            so.ent[q[side]] = (int32_t)(2 * f + side);
            so.nbr[q[side]] = side ? l : r;
            if (so.srec) store_rec<Y::SREC64>(so.srec + q[side] * Y::SREC64, rec);
            else {
                float m[Y::SREC32];
                for (int k = 0; k < Y::SREC32; k++) m[k] = (float)rec[k];
                store_rec<Y::SREC32>(so.srec32 + q[side] * Y::SREC32, m);
            }
        }
    }
}

// The gradient pass's list offsets off[i] = loff[i] + roff[i] and the
// closure test |sum_faces A n_out| <= 1e-9 sum_faces A of every cell (a
// closed surface is a property of every Voronoi cell; the gradient relies
// on it), one lane group per cell over its left range and right faces,
// A and n from the face records.
template <int D>
__global__ void __launch_bounds__(kBlock) k_closure(int64_t n, const double *__restrict__ frec,
                                                    const int32_t *__restrict__ loff, const int32_t *__restrict__ roff,
                                                    const int32_t *__restrict__ rface, int32_t *__restrict__ off,
                                                    int32_t *flags) {
    using Y = Lay<D>;
    constexpr int GS = Group<D>::GS;
    constexpr int NH = 2 + D;   // A, |d|, n
    static_assert(Y::FA == 0 && Y::FELL == 1 && Y::FN == 2, "face record head");
    const int lane = threadIdx.x % GS;
    const int64_t i = (int64_t)blockIdx.x * (kBlock / GS) + threadIdx.x / GS;
    if (i >= n) return;
    const int32_t l0 = loff[i], nl = loff[i + 1] - l0, r0 = roff[i], nr = roff[i + 1] - r0;
    if (lane == 0) {
        off[i] = l0 + r0;
        if (i == n - 1) off[n] = loff[n] + roff[n];
    }
    double clo[D], asum = 0.0;
    for (int k = 0; k < D; k++) clo[k] = 0.0;
    for (int32_t k = lane; k < nl + nr; k += GS) {
        const bool right = k >= nl;
        const int32_t f = right ? rface[r0 + k - nl] : l0 + k;
        double fr[NH];
        load_rec<NH>(frec + (int64_t)f * Y::FREC, fr);
        const double sa = right ? -fr[Y::FA] : fr[Y::FA];   // outward normal: n on the left, -n on the right
        for (int c = 0; c < D; c++) clo[c] += sa * fr[Y::FN + c];
        asum += fr[Y::FA];
    }
    double cl2 = 0.0;
    for (int c = 0; c < D; c++) {
        clo[c] = grp_sum<GS>(clo[c]);
        cl2 += clo[c] * clo[c];
    }
    asum = grp_sum<GS>(asum);
    if (lane == 0 && !(sqrt(cl2) <= 1e-9 * asum)) atomicOr(flags, MF_OPEN);
}

}  // namespace mm
