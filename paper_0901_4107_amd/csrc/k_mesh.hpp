// k_mesh.hpp -- device side of mm_mesh_upload: validation, the per-cell
// list of face sides (CSR, ascending face order inside each cell), the face
// geometry and the face velocities.
#pragma once

#include "common.hpp"
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

// cnt[c] = number of faces that cell c touches (cnt points at off + 1).
__global__ void k_count_sides(int64_t nf, const int32_t *L, const int32_t *R, int32_t *cnt) {
    int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f < nf) {
        atomicAdd(&cnt[L[f]], 1);
        atomicAdd(&cnt[R[f]], 1);
    }
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

// Place every face side into its cell's segment. The order inside a
// segment is fixed afterwards by k_sort_segments.
__global__ void k_fill_sides(int64_t nf, const int32_t *L, const int32_t *R, int32_t *cursor,
                             int32_t *ent, int32_t *nb) {
    int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (f < nf) {
        int32_t l = L[f], r = R[f];
        int32_t p = atomicAdd(&cursor[l], 1);
        ent[p] = (int32_t)(2 * f);
        nb[p] = r;
        int32_t q = atomicAdd(&cursor[r], 1);
        ent[q] = (int32_t)(2 * f + 1);
        nb[q] = l;
    }
}

// Sort each cell's face sides by face index (insertion sort: segments hold
// ~6 entries in 2D and ~15 in 3D), making every per-cell sum deterministic
// and equal in order to a loop over the face list.
__global__ void k_sort_segments(int64_t n, const int32_t *off, int32_t *ent, int32_t *nb) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int32_t b = off[i], e = off[i + 1];
    for (int32_t a = b + 1; a < e; a++) {
        int32_t ke = ent[a], kn = nb[a];
        int32_t j = a - 1;
        while (j >= b && ent[j] > ke) {
            ent[j + 1] = ent[j];
            nb[j + 1] = nb[j];
            j--;
        }
        ent[j + 1] = ke;
        nb[j + 1] = kn;
    }
}

// The update's view of each cell's faces (k_update.hpp), from its side list
// (ascending face order): the number of faces where it is the left and the
// right cell, into lcnt[i] and rcnt[i] (for the offset scans).
__global__ void k_lr_count(int64_t n, const int32_t *__restrict__ off, const int32_t *__restrict__ ent,
                           int32_t *__restrict__ lcnt, int32_t *__restrict__ rcnt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int32_t nl = 0, nr = 0;
    for (int32_t q = off[i]; q < off[i + 1]; q++) {
        if (ent[q] & 1) nr++;
        else nl++;
    }
    lcnt[i] = nl;
    rcnt[i] = nr;
}

// After the scans: each cell's right faces in ascending face order
// (rface[roff[i] ...]), and the check that the faces are sorted by left
// cell (the k-th left face of cell i must be face loff[i] + k, else
// MF_ORDER).
__global__ void k_lr_fill(int64_t n, const int32_t *__restrict__ off, const int32_t *__restrict__ ent,
                          const int32_t *__restrict__ loff, const int32_t *__restrict__ roff,
                          int32_t *__restrict__ rface, int32_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int32_t kl = loff[i], kr = roff[i];
    bool bad = false;
    for (int32_t q = off[i]; q < off[i + 1]; q++) {
        const int32_t en = ent[q], f = en >> 1;
        if (en & 1) {
            rface[kr++] = f;
        } else {
            bad = bad || f != kl;
            kl++;
        }
    }
    if (bad) atomicOr(flags, MF_ORDER);
}

// Face records (Section 3.3 geometry and face velocity):
//   n = d/|d|, c = f - (r_L + r_R)/2 = g - d/2,
//   w_f = (w_L + w_R)/2 + [(w_L - w_R) . c / |d|] n.
// The double record always; the mixed record (float geometry, the
// generators' velocities relative to the face) and the double face velocity
// when mixed != 0.
template <int D>
__global__ void __launch_bounds__(kBlock) k_face_records(int64_t n, int64_t nf, const int32_t *L, const int32_t *R,
                                                         const double *area, const double *ctr, const double *sep,
                                                         const double *mvel, double *frec, int mixed, float *mrec,
                                                         double *wf64) {
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
    double *o = frec + f * Y::FREC;
    o[Y::FA] = area[f];
    o[Y::FELL] = ell;
    double w[D];
    for (int k = 0; k < D; k++) {
        o[Y::FN + k] = d[k] * inv;
        o[Y::FC + k] = c[k];
        w[k] = 0.5 * (wl[k] + wr[k]) + proj * d[k] / s2;
        o[Y::FW + k] = w[k];
    }
    if (mixed) {
        float *m = mrec + f * Y::MREC;
        m[Y::FA] = (float)area[f];
        m[Y::FELL] = (float)ell;
        for (int k = 0; k < D; k++) {
            m[Y::FN + k] = (float)(d[k] * inv);
            m[Y::FC + k] = (float)c[k];
            m[Y::MDW + k] = (float)(wl[k] - wr[k]);
            wf64[f * Y::WSTRIDE + k] = w[k];
        }

    }
}

// Side records in CSR order, one lane per cell: A/|d| and f - r_i, in
// double for the double path and in float for the mixed path, and the
// closure test of each cell,
// |sum_faces A n_out| <= 1e-9 sum_faces A. A closed surface is a property of
// every Voronoi cell; the gradient kernels rely on it.
template <int D>
__global__ void __launch_bounds__(kBlock) k_side_records(int64_t n, int64_t nf, const int32_t *off,
                                                         const int32_t *ent, const double *area, const double *ctr,
                                                         const double *sep, double *srec, int mixed, float *srec32,
                                                         int32_t *flags) {
    using Y = Lay<D>;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double clo[D], asum = 0.0;
    for (int k = 0; k < D; k++) clo[k] = 0.0;
    for (int32_t q = off[i]; q < off[i + 1]; q++) {
        const int32_t en = ent[q];
        const int64_t f = en >> 1;
        const double sg = (en & 1) ? -1.0 : 1.0;  // outward separation e = sg * d
        double d[D], s2 = 0.0;
        for (int k = 0; k < D; k++) { d[k] = sep[k * nf + f]; s2 += d[k] * d[k]; }
        const double ell = sqrt(s2), A = area[f];
        double o[Y::SREC64];
        o[0] = A / ell;
        for (int k = 0; k < D; k++) {
            const double c = ctr[k * nf + f] - 0.5 * d[k];
            o[1 + k] = c + 0.5 * sg * d[k];
            clo[k] += A * sg * d[k] / ell;
        }
        for (int k = 1 + D; k < Y::SREC64; k++) o[k] = 0.0;
        if (!mixed)
            for (int k = 0; k < Y::SREC64; k++) srec[(int64_t)q * Y::SREC64 + k] = o[k];
        asum += A;
        if (mixed) {
            float m[Y::SREC32];
            for (int k = 0; k < Y::SREC32; k++) m[k] = (float)o[k];
            store_rec<Y::SREC32>(srec32 + (int64_t)q * Y::SREC32, m);
        }
    }
    double cl2 = 0.0;
    for (int k = 0; k < D; k++) cl2 += clo[k] * clo[k];
    if (!(sqrt(cl2) <= 1e-9 * asum)) atomicOr(flags, MF_OPEN);
}

}  // namespace mm
