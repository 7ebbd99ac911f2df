// Device helpers shared by the kernel translation units.
#pragma once

#include <math.h>

#include "sc_internal.h"

namespace sc {

// Raw voxel i of the cube in the run's storage (FP32, or 16-bit noise-scaled).
__device__ __forceinline__ float f16_bits_to_float(uint16_t q) {
    return (float)__builtin_bit_cast(_Float16, q);
}
__device__ __forceinline__ float bf16_bits_to_float(uint16_t q) {
    return __uint_as_float((uint32_t)q << 16);
}
__device__ __forceinline__ float load_raw(const float *x, const uint16_t *xq, int type,
                                          int64_t i) {
    if (type == ST_F32) return x[i];
    const uint16_t q = xq[i];
    return type == ST_F16 ? f16_bits_to_float(q) : bf16_bits_to_float(q);
}

// Buffer access: the resource (a uniform base pointer) lives in scalar
// registers, a uniform byte offset goes in the scalar offset and the lane's
// byte offset in the vector offset, so no lane computes a 64-bit address.
// Offsets from one base stay below 2^32 (callers rebase per plane).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)0xffffffff,
                                             0x00020000);
}
__device__ __forceinline__ float buf_f32(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ uint16_t buf_u16(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void buf_st_f32(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                           uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ uint8_t buf_u8(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return (uint8_t)__builtin_amdgcn_raw_buffer_load_b8(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void buf_st_u8(uint8_t v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                          uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b8(v, r, (int)voff, (int)soff, 0);
}

// Lane masks of a wave: bit l of wave_mask(b) is lane l's b; lane_bit(m) is
// this lane's bit of a wave-uniform mask (the mask itself serves as the
// predicate, no per-lane arithmetic).
__device__ __forceinline__ uint64_t wave_mask(bool b) { return __builtin_amdgcn_ballot_w64(b); }
__device__ __forceinline__ bool lane_bit(uint64_t m) {
    return __builtin_amdgcn_inverse_ballot_w64(m);
}
// The 64-bit value that lane j (a wave-uniform index) holds, in every lane.
__device__ __forceinline__ uint64_t lane_word(uint64_t v, int j) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}
// The hardware's lane write (v_writelane_b32): lane `lane` of `old` set to
// the wave-uniform `val`, every other lane unchanged. HIP has no builtin for
// it, so the LLVM intrinsic is named directly.
extern "C" __device__ int sc_writelane_i32(int val, int lane, int old)
    __asm("llvm.amdgcn.writelane.i32");
// v with lane j (a wave-uniform index) replaced by the wave-uniform w.
__device__ __forceinline__ uint64_t with_lane_word(uint64_t v, int j, uint64_t w) {
    const uint32_t lo = (uint32_t)sc_writelane_i32((int)(uint32_t)w, j, (int)(uint32_t)v);
    const uint32_t hi =
        (uint32_t)sc_writelane_i32((int)(uint32_t)(w >> 32), j, (int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
// Number of lanes below this one whose bit is set in the mask m.
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Workgroups are handed to the 8 XCDs round-robin (block b runs on XCD
// b % 8). Remap so that each XCD works through one contiguous range of
// workgroups: neighbouring row chunks then share their halo rows through the
// same L2 instead of fetching them from HBM once per XCD.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
    const int64_t q = nb / 8, r = nb % 8, x = b % 8;
    return x * q + (x < r ? x : r) + b / 8;
}

__device__ __forceinline__ bool in_flux_range(double s, int range) {
    return range < 0 ? (s < 0.0) : (range > 0 ? (s > 0.0) : true);
}

}  // namespace sc
