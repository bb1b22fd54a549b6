// Wavefront (64-lane) helpers for gfx950.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spc5 {

constexpr int kWave = 64;
constexpr int kXcds = 8;   // MI355X: 8 accelerator complex dies, one L2 each

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Inclusive prefix sum of an int over the 64 lanes of the wavefront.
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int t = __shfl_up(v, d);
        if (lane >= d) v += t;
    }
    return v;
}

// Workgroups are dispatched round-robin over the XCDs (workgroup w goes to
// XCD w % 8).  Remap the workgroup index so that each XCD walks one contiguous
// range of tiles: neighbouring tiles share x segments, which then stay in
// that XCD's L2.  Exact bijection on [0, n).
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t n) {
    const int64_t q = n / kXcds, rem = n % kXcds;
    const int64_t xcd = bid % kXcds, idx = bid / kXcds;
    return xcd * q + (xcd < rem ? xcd : rem) + idx;
}

template <int C> struct MaskOf { using type = uint8_t; };
template <> struct MaskOf<16> { using type = uint16_t; };

}  // namespace spc5
