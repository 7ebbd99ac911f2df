// Sampled-Gaussian spatial smoothing: the variant of the spatial kernel in
// which the Gaussian of the given FWHM (Fig. 9 caption; kernel sets of
// Sect. 5 and 6) is sampled at integer offsets |k| <= R, R = floor(4 sigma +
// 1/2), normalised to sum 1, and applied along x then along y with zero
// outside the cube.
//
// A workgroup of 256 threads smooths one strip of 256 output columns over
// one chunk of rows of one plane. It streams the input rows of the strip
// (256 + 2R columns) in steps of four:
//  * the x pass: wave j takes input row j of the step; each lane reads a
//    window of 2R + 4 staged values with 16-byte LDS loads and produces four
//    adjacent outputs (FP32 FMA, taps in scalar registers), written to a ring
//    of the last Q >= 2R + 4 x-filtered rows in LDS;
//  * the y pass: each thread owns one output column and produces four rows
//    from the 2R + 4 ring rows they share, accumulating in FP64 (the FP32
//    x-filtered values enter exactly), then rounds once to FP32.
// The global loads of the next step are in flight during both passes. On
// the input side replacement and blanking happen at load time, exactly as in
// the cascade kernel: a detected voxel becomes copysign(n sigma_0, x), a
// blanked one 0.
#pragma once

#include "sc_internal.h"
#include "sc_device.h"

namespace sc {

template <int R>
struct GaussShape {
    static constexpr int IN = kGaussCols + 2 * R;           // staged input columns
    static constexpr int WIN = 2 * R + 4;                   // x window of four outputs
    static constexpr int WIN4 = (WIN + 3) / 4;              // 16-byte loads per window
    static constexpr int RAW = ((IN + 3) / 4 + 1) * 4;      // staged row stride (floats)
    static constexpr int Q = ((2 * R + 4 + 3) / 4) * 4;     // ring rows
    static constexpr int EXTRA = IN - kGaussCols;           // threads loading a second column
};

template <int R, int XT, bool RP>
__global__ __launch_bounds__(kGaussCols) void k_gauss(GaussArgs a) {
    using S = GaussShape<R>;
    static_assert(S::EXTRA <= kGaussCols, "radius too large for the strip");
    __shared__ __align__(16) float raw[4][S::RAW];
    __shared__ __align__(16) float ring[S::Q][kGaussCols];

    const int tid = threadIdx.x;
    const int64_t nx = a.nx, ny = a.ny;
    const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t strip = tile % a.nstrips;
    const int64_t rest = tile / a.nstrips;
    const int64_t chunk = rest % a.nchunks;
    const int64_t z = rest / a.nchunks;
    if (z >= a.nz) return;

    const int64_t x0 = strip * kGaussCols;     // first output column
    const int64_t ya = chunk * a.rows;
    const int64_t yb = ya + a.rows < ny ? ya + a.rows : ny;
    const int64_t plane = z * nx * ny;

    const __amdgpu_buffer_rsrc_t xr = plane_rsrc(XT == ST_F32 ? (const void *)(a.x + plane)
                                                              : (const void *)(a.xq + plane));
    constexpr uint32_t XB = XT == ST_F32 ? 4u : 2u;
    const uint32_t *dp = RP ? reinterpret_cast<const uint32_t *>(a.det) + z * a.wpp * 2
                            : nullptr;
    const float rv = RP ? (float)(a.repl_n * a.st->sigma0) : 0.f;

    // input columns of this thread: c0 = tid, c1 = kGaussCols + tid (tid < EXTRA)
    const int64_t gx0 = x0 - R + tid, gx1 = x0 - R + kGaussCols + tid;
    const bool has1 = tid < S::EXTRA;
    const bool in0 = gx0 >= 0 && gx0 < nx, in1 = has1 && gx1 >= 0 && gx1 < nx;
    const uint32_t cx0 = (uint32_t)(in0 ? gx0 : 0), cx1 = (uint32_t)(in1 ? gx1 : 0);

    // Raw loads only: the conversions and bit tests happen in stage(), so
    // that no wait for these loads is needed before the barrier after them.
    auto ld = [&](uint32_t soff, uint32_t voff) -> uint32_t {
        if constexpr (XT == ST_F32) return __float_as_uint(buf_f32(xr, voff, soff));
        else return (uint32_t)buf_u16(xr, voff, soff);
    };
    auto to_float = [&](uint32_t q) -> float {
        if constexpr (XT == ST_F32) return __uint_as_float(q);
        else if constexpr (XT == ST_F16) return f16_bits_to_float((uint16_t)q);
        else return bf16_bits_to_float((uint16_t)q);
    };
    // value entering the smoothing: zero outside the cube and at blanked
    // voxels, copysign(n sigma_0, v) where the voxel's detection bit is set
    // (bit `pos` of the 32-bit word `word` of packed detection bits)
    auto value = [&](uint32_t q, bool inside, uint32_t word, uint32_t pos) -> float {
        const float v = to_float(q);
        if (!inside || !isfinite(v)) return 0.f;
        if (RP && ((word >> pos) & 1u)) return copysignf(rv, v);
        return v;
    };
    auto bit_of = [&](int64_t y, uint32_t cx) -> int64_t { return y * nx + (int64_t)cx; };

    // the next step's values (and detection words) are loaded one step ahead
    uint32_t pv0[4], pv1[4], pd0[4], pd1[4];
    auto fetch = [&](int64_t y0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t y = y0 + j;
            const bool yin = y >= 0 && y < ny;
            const int64_t yc = yin ? y : 0;
            const uint32_t roff = (uint32_t)yc * (uint32_t)nx * XB;
            pv0[j] = ld(roff, cx0 * XB);
            pv1[j] = has1 ? ld(roff, cx1 * XB) : 0u;
            if constexpr (RP) {
                pd0[j] = dp[bit_of(yc, cx0) >> 5];
                pd1[j] = has1 ? dp[bit_of(yc, cx1) >> 5] : 0u;
            } else {
                pd0[j] = pd1[j] = 0u;
            }
        }
    };
    auto stage = [&](int64_t y0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t y = y0 + j;
            const bool yin = y >= 0 && y < ny;
            const int64_t yc = yin ? y : 0;
            raw[j][tid] = value(pv0[j], in0 && yin, pd0[j], (uint32_t)(bit_of(yc, cx0) & 31));
            if (has1)
                raw[j][kGaussCols + tid] =
                    value(pv1[j], in1 && yin, pd1[j], (uint32_t)(bit_of(yc, cx1) & 31));
        }
    };

    const int wave = tid >> 6, lane = tid & 63;
    const int64_t y_first = ya - R;                 // first input row
    const int64_t n_in = (yb - ya) + 2 * R;
    const int64_t steps = (n_in + 3) / 4;

    fetch(y_first);
    for (int64_t s = 0; s < steps; ++s) {
        const int64_t yi0 = y_first + 4 * s;
        stage(yi0);
        __syncthreads();
        if (s + 1 < steps) fetch(yi0 + 4);

        // x pass: wave j filters input row yi0 + j, lane -> outputs 4 lane .. 4 lane + 3
        {
            float w[S::WIN4 * 4];
            const float4 *src = reinterpret_cast<const float4 *>(&raw[wave][4 * lane]);
#pragma unroll
            for (int q = 0; q < S::WIN4; ++q) {
                const float4 v = src[q];
                w[4 * q] = v.x; w[4 * q + 1] = v.y; w[4 * q + 2] = v.z; w[4 * q + 3] = v.w;
            }
            float o[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k <= 2 * R; ++k) {
                const float h = a.tf[k < R ? R - k : k - R];
#pragma unroll
                for (int p = 0; p < 4; ++p) o[p] = fmaf(h, w[p + k], o[p]);
            }
            int64_t slot = (yi0 + wave) % S::Q;
            if (slot < 0) slot += S::Q;
            *reinterpret_cast<float4 *>(&ring[slot][4 * lane]) = make_float4(o[0], o[1], o[2], o[3]);
        }
        __syncthreads();

        // y pass: output rows yi0 - R .. yi0 - R + 3 of column x0 + tid
        const int64_t yo0 = yi0 - R;
        if (yo0 + 3 >= ya && yo0 < yb) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            int64_t base = (yi0 - 2 * R) % S::Q;
            if (base < 0) base += S::Q;
#pragma unroll
            for (int m = 0; m < S::WIN; ++m) {
                int slot = (int)base + m;
                slot = slot >= S::Q ? slot - S::Q : slot;
                slot = slot >= S::Q ? slot - S::Q : slot;
                const double v = (double)ring[slot][tid];
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const int k = m - p;
                    if (k >= 0 && k <= 2 * R) acc[p] = fma(a.td[k < R ? R - k : k - R], v, acc[p]);
                }
            }
            const int64_t gx = x0 + tid;
            if (gx < nx) {
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const int64_t yo = yo0 + p;
                    if (yo >= ya && yo < yb) a.p[plane + yo * nx + gx] = (float)acc[p];
                }
            }
        }
    }
}

template <int R>
hipError_t launch_gauss_r(const GaussArgs &a, int xtype, bool repl, hipStream_t s) {
    const dim3 grid((unsigned)a.tiles), block(kGaussCols);
#define SC_GAUSS(XT, RP) hipLaunchKernelGGL((k_gauss<R, XT, RP>), grid, block, 0, s, a)
    if (xtype == ST_F16) {
        if (repl) SC_GAUSS(ST_F16, true); else SC_GAUSS(ST_F16, false);
    } else if (xtype == ST_BF16) {
        if (repl) SC_GAUSS(ST_BF16, true); else SC_GAUSS(ST_BF16, false);
    } else {
        if (repl) SC_GAUSS(ST_F32, true); else SC_GAUSS(ST_F32, false);
    }
#undef SC_GAUSS
    return hipGetLastError();
}

}  // namespace sc
