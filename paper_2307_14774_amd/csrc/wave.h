// Wavefront (64-lane) helpers for gfx950.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spc5 {

constexpr int kWave = 64;
constexpr int kXcds = 8;   // MI355X: 8 accelerator complex dies, one L2 each

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Inclusive prefix sum of an int over the 64 lanes of the wavefront, built
// from DPP lane moves so that it costs VALU operations only (a shuffle-based
// scan waits on six LDS-unit round trips in a row).  Steps: shifts by 1, 2,
// 4 and 8 lanes inside each 16-lane row (lanes shifted in from outside the
// row read 0) give every row its own inclusive scan; then the last lane of
// row 0 is added into row 1 and the last lane of row 2 into row 3 (row
// broadcast of lane 15 with rows 1 and 3 enabled), and the last lane of row
// 1 -- by then the total of rows 0-1 -- into rows 2 and 3 (broadcast of lane
// 31 with rows 2 and 3 enabled).  Every lane of the wavefront must be active.
__device__ __forceinline__ int wave_incl_scan(int v) {
    constexpr int kRowShr = 0x110, kBcast15 = 0x142, kBcast31 = 0x143;
    v += __builtin_amdgcn_update_dpp(0, v, kRowShr + 1, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kRowShr + 2, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kRowShr + 4, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kRowShr + 8, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kBcast15, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kBcast31, 0xc, 0xf, false);
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

// Runs of g consecutive work items per XCD, the runs dealt round robin:
// neighbouring items still share one XCD's L2, and every XCD gets items from
// the whole range, so a range whose cost changes along it (a graph transpose:
// dense hub rows first, scattered tail rows after) stays balanced.  Items past
// the last full round keep their own index.
__device__ __forceinline__ int64_t xcd_chunks(int64_t bid, int64_t n, int g) {
    const int64_t full = (n / (kXcds * (int64_t)g)) * kXcds * g;
    if (bid >= full) return bid;
    const int64_t xcd = bid % kXcds, idx = bid / kXcds;
    return ((idx / g) * kXcds + xcd) * g + idx % g;
}

// Raw buffer loads.  A load whose byte offset lies at or beyond the
// descriptor's record count returns 0 and moves no data, which gives
// predicated gathers without branches: the lanes whose mask bit is clear pass
// kOOB.  Record counts are kept below 2^31 so kOOB is always out of range.
constexpr uint32_t kOOB = 0x80000000u;
constexpr int64_t kMaxBufBytes = 0x7FFFFFF0;

struct Buf {
    __amdgpu_buffer_rsrc_t r;
};

__device__ __forceinline__ Buf make_buf(const void *p, int64_t bytes) {
    Buf b;
    const int nrec = (int)(bytes < kMaxBufBytes ? bytes : kMaxBufBytes);
    // word 3: 32-bit data format, raw (unswizzled) addressing
    b.r = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, nrec, 0x00020000);
    return b;
}

template <typename T> __device__ __forceinline__ T buf_load(const Buf &b, uint32_t off);
template <> __device__ __forceinline__ double buf_load<double>(const Buf &b, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(b.r, (int)off, 0, 0));
}
template <> __device__ __forceinline__ float buf_load<float>(const Buf &b, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.r, (int)off, 0, 0));
}

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// 16-byte raw buffer load (zeros when out of the descriptor's range).
__device__ __forceinline__ v4u buf_load16(const Buf &b, uint32_t off) {
    return __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(b.r, (int)off, 0, 0));
}

template <int C> struct MaskOf { using type = uint8_t; };
template <> struct MaskOf<16> { using type = uint16_t; };

}  // namespace spc5
