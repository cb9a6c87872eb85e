// Wave-level building blocks for gfx950 shared by the streaming kernels:
// bounds-checked buffer loads and stores, and neighbour exchange between the
// lanes of a wave.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace stk {

// Buffer resources over one row (or any extent) of an array.  A lane that
// passes an offset at or past the extent reads 0 and its write is dropped, so
// bounds and walls need no branch; OOB is such an offset for any extent.
constexpr unsigned OOB = 0xFFFFFFF0u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, size_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

// Neighbour exchange inside a wave whose lane is a grid column: lane i gets
// the value of lane i + 1 (DPP wave_shl:1) or of lane i - 1 (wave_shr:1); a
// lane whose source is outside the wave gets 0.
constexpr int DPP_FROM_NEXT = 0x130, DPP_FROM_PREV = 0x138;
template <int CTRL>
__device__ __forceinline__ double wave_shift(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, (long long)(unsigned)lo | ((long long)hi << 32));
}
template <int CTRL>
__device__ __forceinline__ float wave_shift(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

// A value that is the same in every lane, moved to scalar registers (FP64
// arithmetic leaves its results in vector registers even when they are
// uniform; kernels that are short of vector registers keep them scalar).
__device__ __forceinline__ double wave_uniform(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readfirstlane((int)b);
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, (long long)(unsigned)lo | ((long long)hi << 32));
}
__device__ __forceinline__ float wave_uniform(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// Workgroups are dealt to the XCDs round-robin (workgroup w to XCD w mod 8),
// and each XCD has its own L2.  This renumbering gives each XCD one contiguous
// run of the workgroup index space, so that workgroups with neighbouring
// indices run on one XCD at the same time and share their halos in L2.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_tile(int w, int nwg) {
    const int q = nwg / NXCD, r = nwg % NXCD, x = w % NXCD;
    return x * q + (x < r ? x : r) + w / NXCD;
}

}  // namespace stk
