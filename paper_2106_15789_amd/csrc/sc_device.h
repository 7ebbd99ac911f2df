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

__device__ __forceinline__ bool in_flux_range(double s, int range) {
    return range < 0 ? (s < 0.0) : (range > 0 ? (s > 0.0) : true);
}

}  // namespace sc
