// k_walls.hpp -- reflective walls by mirrored generators (the boundary of
// the Rayleigh-Taylor test of Section 8, by the mirroring of Section 3.6,
// boundary conditions): the generators next to a
// wall have mirror images across it, whose cells close the tessellation at
// the wall plane. Before each step every mirror cell takes the state of its
// source with the momentum component normal to the wall negated, so that
// the face on the wall carries a symmetric Riemann problem (no mass or
// energy crosses it; it exerts only a pressure).
#pragma once

#include "common.hpp"

namespace mm {

enum WallFlag : int { WF_INDEX = 1, WF_SELF = 2, WF_TWICE = 4, WF_CHAIN = 8 };

// Pass 1 of the validation of a wall list: indices in [0, n), no mirror
// cell its own source; counts every mirror cell in mark (zeroed before).
__global__ void k_walls_mark(int64_t n, int64_t ng, const int32_t *ghost, const int32_t *src, int32_t *mark,
                             int32_t *flags) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= ng) return;
    const int32_t g = ghost[k], s = src[k];
    int bad = 0;
    if (g < 0 || g >= n || s < 0 || s >= n) bad |= WF_INDEX;
    else if (g == s) bad |= WF_SELF;
    else atomicAdd(mark + g, 1);
    if (bad) atomicOr(flags, bad);
}

// Pass 2: every mirror cell listed once, and no source a mirror cell (the
// reflection is then one independent copy per entry, in any order).
__global__ void k_walls_check(int64_t n, int64_t ng, const int32_t *ghost, const int32_t *src, const int32_t *mark,
                              int32_t *flags) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= ng) return;
    const int32_t g = ghost[k], s = src[k];
    if (g < 0 || g >= n || s < 0 || s >= n) return;   // raised by pass 1
    int bad = 0;
    if (mark[g] != 1) bad |= WF_TWICE;
    if (mark[s] != 0) bad |= WF_CHAIN;
    if (bad) atomicOr(flags, bad);
}

// Q [nrow][n]: row r of mirror cell ghost[k] <- row r of src[k], the
// momentum row along the wall normal (1 + axis) negated. The lists are
// short (the cells along the walls) and scattered: one thread per entry.
__global__ void __launch_bounds__(kBlock) k_reflect(int64_t n, int64_t ng, int nrow, int axis, const int32_t *ghost,
                                                    const int32_t *src, double *Q) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= ng) return;
    const int64_t g = ghost[k], s = src[k];
    for (int r = 0; r < nrow; r++) {
        const double v = Q[r * n + s];
        Q[r * n + g] = r == 1 + axis ? -v : v;
    }
}

}  // namespace mm
