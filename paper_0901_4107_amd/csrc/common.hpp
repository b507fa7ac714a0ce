// common.hpp -- shared device helpers of libmm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mm {

constexpr int kBlock = 256;   // 4 wavefronts of 64 lanes
// Batched Riemann problems are solved in chunks of this many, the size of
// the hard-problem list of a mixed-precision context.
constexpr int64_t kBatchChunk = int64_t(1) << 22;
constexpr int kXcd = 8;       // MI355X: workgroups are dealt round-robin to 8 XCDs

// Grid size for n items, rounded up to a multiple of the XCD count so that
// xcd_tile() below is a bijection.
inline unsigned grid_for(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    b = (b + kXcd - 1) / kXcd * kXcd;
    return (unsigned)b;
}

// The hardware sends workgroup b to XCD b % 8. Remap so that each XCD works
// on one contiguous range of tiles: neighbouring cells and faces (in
// space-filling-curve order) then share one XCD's L2.
__device__ __forceinline__ int64_t xcd_tile() {
    const int64_t nb = gridDim.x;
    const int64_t b = blockIdx.x;
    const int64_t per = nb / kXcd;
    return (b % kXcd) * per + b / kXcd;
}

__device__ __forceinline__ int64_t xcd_global_id() {
    return xcd_tile() * kBlock + threadIdx.x;
}

// Records of N elements moved with 16-byte accesses (one memory instruction
// per 16 bytes, the remainder in single elements). The vector types carry
// the element's alignment only: the hardware takes 16-byte global accesses
// at any element-aligned address, so records need no padding to 16 bytes.
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));
typedef double f64x2u __attribute__((ext_vector_type(2), aligned(8)));
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef f32x4u type; static constexpr int n = 4; };
template <> struct Vec16<double> { typedef f64x2u type; static constexpr int n = 2; };

template <int N, typename T> __device__ __forceinline__ void load_rec(const T *__restrict__ p, T (&o)[N]) {
    using V = typename Vec16<T>::type;
    constexpr int per = Vec16<T>::n;
    for (int i = 0; i < N / per; i++) {
        const V v = *reinterpret_cast<const V *>(p + i * per);
        for (int j = 0; j < per; j++) o[i * per + j] = v[j];
    }
    for (int k = N / per * per; k < N; k++) o[k] = p[k];
}
// A record of N floats from LDS, through an LDS-typed pointer: a load that
// may come from LDS or from global memory behind one generic pointer would
// compile to a flat load, which waits on both memory paths.
typedef __attribute__((address_space(3))) const float lds_cfloat;
template <int N> __device__ __forceinline__ void load_rec_lds(lds_cfloat *p, float (&o)[N]) {
    typedef __attribute__((address_space(3))) const f32x4u lds_cf32x4;
    for (int i = 0; i < N / 4; i++) {
        const f32x4u v = *reinterpret_cast<lds_cf32x4 *>(p + i * 4);
        for (int j = 0; j < 4; j++) o[i * 4 + j] = v[j];
    }
    for (int k = N / 4 * 4; k < N; k++) o[k] = p[k];
}
template <int N, typename T> __device__ __forceinline__ void store_rec(T *__restrict__ p, const T (&o)[N]) {
    using V = typename Vec16<T>::type;
    constexpr int per = Vec16<T>::n;
    for (int i = 0; i < N / per; i++) {
        V v;
        for (int j = 0; j < per; j++) v[j] = o[i * per + j];
        *reinterpret_cast<V *>(p + i * per) = v;
    }
    for (int k = N / per * per; k < N; k++) p[k] = o[k];
}

// Device-side diagnostic accumulators (mirrors mm_diag's counters). Each
// block adds into one of kDiagSlots copies (chosen by block index) so that
// the per-block atomics spread over many addresses instead of serialising
// on one; the host sums the slots.
constexpr int kDiagSlots = 256;
struct DiagDev {
    unsigned long long newton_iters, newton_max, unconverged, vacuum, positivity_fallback, fp64_fallback,
        guess_fallback, wave_iter_max_sum, entropy_kept;
};

// A list of flagged items (hard faces or problems) split into kLists
// sub-lists, one per residue of the producing block index, each with its
// own counter on its own 128-byte line: appends from different blocks
// rarely meet on one atomic. Sub-list c holds the items of the blocks with
// blockIdx % kLists == c, at most list_cap(grid) of them.
// Layout (int32): kLists counters kListPad apart, then kLists item arrays.
constexpr int kLists = 256;
constexpr int kListPad = 32;
__host__ __device__ inline int64_t list_cap(int64_t grid) { return (grid + kLists - 1) / kLists * kBlock; }
inline int64_t list_ints(int64_t grid) { return (int64_t)kLists * kListPad + kLists * list_cap(grid); }

// Wave-aggregated append of `item` where `flag` is set; every lane of the
// wavefront calls it.
__device__ __forceinline__ void list_append(int32_t *list, int64_t cap, bool flag, int32_t item) {
    const unsigned long long mask = __ballot(flag);
    if (!mask) return;
    const int c = blockIdx.x % kLists;
    const int lane = threadIdx.x & 63;
    const int first = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane == first) base = atomicAdd(list + c * kListPad, __popcll(mask));
    base = __shfl(base, first, 64);
    if (flag) list[(int64_t)kLists * kListPad + c * cap + base + __popcll(mask & ((1ull << lane) - 1ull))] = item;
}

// Consumer side: a grid of a multiple of kLists blocks; block b walks
// sub-list b % kLists together with the other blocks of that residue.
struct ListWalk {
    const int32_t *items;
    int64_t count, start, stride;
};
__device__ __forceinline__ ListWalk list_walk(const int32_t *list, int64_t cap) {
    const int c = blockIdx.x % kLists;
    ListWalk w;
    w.items = list + (int64_t)kLists * kListPad + c * cap;
    w.count = list[c * kListPad];
    w.start = (int64_t)(blockIdx.x / kLists) * kBlock + threadIdx.x;
    w.stride = (int64_t)(gridDim.x / kLists) * kBlock;
    return w;
}

// Individual timesteps: the slots of a timeline's info block in device
// memory.
enum : int {
    TB_ERR = 0,         // a criterion fell below one tick: the timeline halts
    TB_CELLS = 1,       // active cells of the last point performed
    TB_FACES = 2,       // active faces of the last point performed
    TB_NONFIN = 3,      // a non-finite state since the batch began
    TB_SPARSE = 4,      // path of the next point (1: from the active cells' sides)
    TB_LIVE = 5,        // the current point runs (not halted, tick below the stop tick)
    TB_LO = 6,          // smallest and largest occupied bins
    TB_HI = 7,
    TB_COUNTS = 8,      // cells per bin, TB_COUNTS + b for b <= kTbMaxLevels
    TB_TI = 40,         // int64: the current tick
    TB_LAST = 42,       // int64: tick of the last point performed
    TB_SUMC = 44,       // int64: active cells over the batch
    TB_SUMF = 46,       // int64: active faces over the batch
    TB_UNTIL = 48,      // int64: the batch's stop tick
    TB_NPTS = 50,       // points performed in the batch
    TB_CUR = 51,        // touch stamp of the current point (points since begin)
    TB_NSPARSE = 52,    // sparse points in the batch
    TB_LASTSPARSE = 53, // path of the last point performed
    TB_INFO_INTS = 64
};

__device__ __forceinline__ int64_t &tb64(int32_t *info, int slot) { return *reinterpret_cast<int64_t *>(info + slot); }
__device__ __forceinline__ int64_t tb64(const int32_t *info, int slot) {
    return *reinterpret_cast<const int64_t *>(info + slot);
}

}  // namespace mm
