// common.hpp -- shared device helpers of libmm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mm {

constexpr int kBlock = 256;   // 4 wavefronts of 64 lanes
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

}  // namespace mm
