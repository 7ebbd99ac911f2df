// Spatial Gaussian as a cascade of NIT boxcars of width 2R+1 per axis,
// computed by streaming strips (one translation unit per NIT instantiates it).
//
// One wave owns a strip of 128 adjacent columns of one plane and streams a
// chunk of rows through it, top to bottom. Lane l holds the two columns
// x0 - H + 2l and x0 - H + 2l + 1 (H = R * NIT); after the cascade the
// columns H .. 127 - H of the strip are its 128 - 2H outputs.
//  - x passes run across lanes: a boxcar over the lane pairs is built from
//    the pair sums c0 + c1 of neighbouring lanes, reached through DPP wave
//    shifts, so a row never leaves the registers and two columns share most
//    of the work;
//  - y passes run down the rows: per pass a running sum over a ring of the
//    last 2R+1 inputs, so one new row advances all passes by one row and a
//    pass's output trails its input by R rows. Rings, sums and the values
//    handed from pass to pass are FP64, which holds these sums of FP32 data
//    exactly: the y passes add no rounding, and the result is rounded to
//    FP32 once.
// A workgroup holds the waves of adjacent strips of the same rows. It loads
// each row's span of columns once (every thread two columns, clamped into
// the plane, so loads are always in bounds) into a double-buffered LDS tile,
// a block of U rows ahead of use, together with the packed detection bits of
// those rows: strips that overlap by their halos never fetch a byte twice.
// Every pass sees zeros beyond the cube (per-pass zero padding): rows outside
// the plane are zeroed by a uniform test on the row index, columns outside
// it by a per-column select.
#pragma once

#include <type_traits>

#include "sc_device.h"

namespace sc {

// Lane i receives lane i-K's value (shr) or lane i+K's (shl); lanes without
// a source receive 0.
template <int K>
__device__ __forceinline__ float wave_shr(float v) {
#pragma unroll
    for (int k = 0; k < K; ++k)
        v = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
    return v;
}
template <int K>
__device__ __forceinline__ float wave_shl(float v) {
#pragma unroll
    for (int k = 0; k < K; ++k)
        v = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
    return v;
}

// Unnormalised boxcar of width 2R+1 along a row held as two columns per
// lane (c0 = column 2l, c1 = column 2l + 1). With p = c0 + c1 the pair sum,
// the window of column 2l or 2l+1 is a run of whole pairs plus one single
// column at one end:
//   R = 2m:   out0 = p[l-m] .. p[l+m-1] + c0[l+m],  out1 = p[l-m+1] .. p[l+m] + c1[l-m]
//   R = 2m+1: out0 = p[l-m] .. p[l+m]   + c1[l-m-1], out1 = p[l-m] .. p[l+m] + c0[l+m+1]
// Lanes within reach of either end of the wave get partial sums; they only
// ever feed columns that are themselves discarded.
template <int K>
struct PairSym {   // p[l-K] + .. + p[l+K]
    __device__ __forceinline__ static float sum(float p) {
        return PairSym<K - 1>::sum(p) + (wave_shr<K>(p) + wave_shl<K>(p));
    }
};
template <>
struct PairSym<0> {
    __device__ __forceinline__ static float sum(float p) { return p; }
};

template <int R>
__device__ __forceinline__ void box_pairs(float &c0, float &c1) {
    const float p = c0 + c1;
    constexpr int m = R / 2;
    if constexpr (R % 2 == 0) {
        const float core = PairSym<m - 1>::sum(p);            // p[l-m+1] .. p[l+m-1]
        const float o0 = (core + wave_shr<m>(p)) + wave_shl<m>(c0);
        const float o1 = (core + wave_shl<m>(p)) + wave_shr<m>(c1);
        c0 = o0;
        c1 = o1;
    } else {
        const float core = PairSym<m>::sum(p);                // p[l-m] .. p[l+m]
        const float o0 = core + wave_shr<m + 1>(c1);
        const float o1 = core + wave_shl<m + 1>(c0);
        c0 = o0;
        c1 = o1;
    }
}

template <int R, int NIT, int XT, bool RP>
__global__ __launch_bounds__(64 * kStripWaves) void k_strip(StripArgs a) {
    constexpr int H = R * NIT;
    constexpr int W = kStripCols - 2 * H;     // output columns per strip
    constexpr int Q = 2 * R + 1;              // ring slots: one boxcar window
    constexpr int U = Q * ((8 + Q - 1) / Q);  // rows per block (>= 8)
    constexpr int SPM = kStripWaves * W + 2 * H;   // widest staged span
    constexpr int DWM = SPM / 32 + 3;              // 32-bit detection words per staged row
    static_assert(W >= 2, "halo too large for a 128-column strip");
    static_assert(U <= 16, "detection-word staging assumes at most 16 rows per block");
    __shared__ float xs[2][U][SPM + 1];
    __shared__ uint32_t dws[2][U][RP ? DWM : 1];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nthr = blockDim.x;

    // strip group, row chunk and plane of this workgroup (groups fastest)
    const int64_t t = xcd_remap((int64_t)blockIdx.x, a.tiles);
    const int64_t per_plane = (int64_t)a.ngroups * a.nchunks;
    const int64_t z = t / per_plane;
    const int64_t rem = t - z * per_plane;
    const int chunk = (int)(rem / a.ngroups);
    const int grp = (int)(rem - (int64_t)chunk * a.ngroups);
    const int s0 = grp * a.wpb;                     // first strip of the group
    const int nw = min(a.wpb, a.nstrips - s0);      // strips of the group
    const bool active = wave < nw;                  // waves past them only stage

    const int64_t nx = a.nx;
    const int ny = (int)a.ny;
    const int64_t span0 = (int64_t)s0 * W - H;      // column of staged position 0
    const int span = nw * W + 2 * H;                // staged columns (<= 2 threads)
    const int64_t plane = z * nx * (int64_t)ny;
    const __amdgpu_buffer_rsrc_t xr = plane_rsrc(XT == ST_F32 ? (const void *)(a.x + plane)
                                                               : (const void *)(a.xq + plane));
    const __amdgpu_buffer_rsrc_t pr = plane_rsrc(a.p + plane);
    constexpr uint32_t XB = XT == ST_F32 ? 4u : 2u;  // bytes per stored voxel
    const uint32_t *dp = RP ? (const uint32_t *)(a.det + z * a.wpp) : nullptr;
    const int64_t ndw = 2 * a.wpp;                  // 32-bit detection words per plane
    auto clamp_col = [&](int64_t c) -> uint32_t {
        return (uint32_t)(c < 0 ? 0 : (c >= nx ? nx - 1 : c));
    };
    auto clamp_row = [&](int y) { return y < 0 ? 0 : (y >= ny ? ny - 1 : y); };

    // Staging role: thread tid loads staged positions tid and tid + nthr of
    // every row (clamped into the plane; positions past the span load a
    // duplicate and drop it), and detection word dcol of row drow.
    const bool st0 = tid < span, st1 = tid + nthr < span;
    const uint32_t sc0 = clamp_col(span0 + tid), sc1 = clamp_col(span0 + tid + nthr);
    // detection words a row needs: bit offsets reach 31 + span - 1, and a
    // lane reads the word of its offset and the next one
    const int dwn = (span + 31) / 32 + 2;
    // U * dwn <= 2 * nthr (span <= 2 nthr, U <= 16): two words per thread
    const int di0 = tid, di1 = tid + nthr;
    const int drow0 = min(di0 / dwn, U - 1), dcol0 = di0 - (di0 / dwn) * dwn;
    const int drow1 = min(di1 / dwn, U - 1), dcol1 = di1 - (di1 / dwn) * dwn;
    const bool dst0 = RP && di0 < U * dwn, dst1 = RP && di1 < U * dwn;
    // Detection bits of (clamped) row yy are staged from 32-bit word
    // floor((yy nx + span0) / 32) on; staged position x of that row is then
    // bit ((yy nx + span0) & 31) + x of the staged words (never negative).
    // Words before the plane (only where span0 < 0) read word 0 instead: they
    // only cover columns left of the cube.
    auto row_bit0 = [&](int yy) -> int64_t { return (int64_t)yy * nx + span0; };

    // Compute role: columns gx and gx + 1 of strip s0 + wave.
    const int lx = wave * W + 2 * lane;             // staged position of gx
    const int64_t gx = span0 + lx;
    const bool xin0 = gx >= 0 && gx < nx, xin1 = gx + 1 >= 0 && gx + 1 < nx;
    const uint32_t vo0 = clamp_col(gx) * 4u, vo1 = clamp_col(gx + 1) * 4u;   // P offsets
    // the whole strip (positions 0 .. kStripCols - 1) inside the plane in x
    const bool x_interior = span0 + wave * W >= 0 && span0 + wave * W + kStripCols - 1 < nx;
    const bool out0 = 2 * lane >= H && 2 * lane < kStripCols - H && xin0;
    const bool out1 = 2 * lane + 1 >= H && 2 * lane + 1 < kStripCols - H && xin1;
    const float rv = RP ? (float)(a.repl_n * a.st->sigma0) : 0.f;
    double norm = 1.0;
#pragma unroll
    for (int p = 0; p < 2 * NIT; ++p) norm *= (double)(2 * R + 1);
    const double scale = 1.0 / norm;

    const int ya = chunk * a.rows;
    const int yb = min(ny, ya + a.rows);
    const int y_first = ya - H;                     // first input row
    const int n_in = (yb - ya) + 2 * H;             // input rows streamed
    const int nblk = (n_in + U - 1) / U;

    float sv0[U], sv1[U];
    uint32_t sd0 = 0, sd1 = 0;
    const uint32_t so0 = sc0 * XB, so1 = sc1 * XB;   // staging column offsets
    auto ld = [&](uint32_t soff, uint32_t voff) -> float {
        if constexpr (XT == ST_F32) return buf_f32(xr, voff, soff);
        else if constexpr (XT == ST_F16) return f16_bits_to_float(buf_u16(xr, voff, soff));
        else return bf16_bits_to_float(buf_u16(xr, voff, soff));
    };
    auto stage_load = [&](int blk) {
        const int y0 = y_first + blk * U;
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint32_t roff = (uint32_t)clamp_row(y0 + j) * (uint32_t)nx * XB;
            sv0[j] = ld(roff, so0);
            sv1[j] = ld(roff, so1);
        }
        if (RP) {
            auto word = [&](int drow, int dcol) {
                int64_t w = (row_bit0(clamp_row(y0 + drow)) >> 5) + dcol;
                w = w < 0 ? 0 : (w >= ndw ? ndw - 1 : w);
                return dp[w];
            };
            sd0 = word(drow0, dcol0);
            sd1 = word(drow1, dcol1);
        }
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (st0) xs[buf][j][tid] = sv0[j];
            if (st1) xs[buf][j][tid + nthr] = sv1[j];
        }
        if (dst0) dws[buf][drow0][dcol0] = sd0;
        if (dst1) dws[buf][drow1][dcol1] = sd1;
    };

    double ring[2][NIT][Q];
    double S[2][NIT];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int p = 0; p < NIT; ++p) {
            S[c][p] = 0.0;
#pragma unroll
            for (int j = 0; j < Q; ++j) ring[c][p][j] = 0.0;
        }

    // EDGE = false: this wave's strip lies inside the plane in x and every
    // row and pass of the block inside it in y, so no zeroing is needed (the
    // selects and multiplies by 1 it skips are exact no-ops there).
    auto compute = [&](int buf, int blk, auto edge_c) {
        constexpr bool EDGE = decltype(edge_c)::value;
        const int base = blk * U;
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int yi = y_first + base + j;      // input row of this step
            const float vx = xs[buf][j][lx], vy = xs[buf][j][lx + 1];

            // pass-0 values: zero at blanked voxels, +-n sigma_0 (sign of the
            // datum) at detected ones (the packed bits mark only finite
            // voxels), zero outside the cube
            float c0 = isfinite(vx) ? vx : 0.f, c1 = isfinite(vy) ? vy : 0.f;
            if (RP) {
                const uint32_t t0 = (uint32_t)(row_bit0(clamp_row(yi)) & 31) + (uint32_t)lx;
                const uint32_t *wr = &dws[buf][j][t0 >> 5];
                const uint32_t bits = __builtin_amdgcn_alignbit(wr[1], wr[0], t0 & 31);
                if (bits & 1u) c0 = copysignf(rv, vx);
                if (bits & 2u) c1 = copysignf(rv, vy);
            }
            if (EDGE) {
                const bool yin = yi >= 0 && yi < ny;   // uniform
                c0 = (xin0 && yin) ? c0 : 0.f;
                c1 = (xin1 && yin) ? c1 : 0.f;
            }

#pragma unroll
            for (int p = 0; p < NIT; ++p) {
                box_pairs<R>(c0, c1);
                if (EDGE) {
                    c0 = xin0 ? c0 : 0.f;           // no-op away from the x edges
                    c1 = xin1 ? c1 : 0.f;
                }
            }

            // y passes; ring slot j % Q held the input of Q steps ago
            double d[2] = {(double)c0, (double)c1};
#pragma unroll
            for (int p = 0; p < NIT; ++p) {
                const int sl = j % Q;
                // zero outside the plane (a uniform 0/1: one multiply)
                const int q = yi - (p + 1) * R;     // row of this pass's output
                const double keep = (q >= 0 && q < ny) ? 1.0 : 0.0;
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const double old = ring[c][p][sl];
                    ring[c][p][sl] = d[c];
                    S[c][p] = (S[c][p] + d[c]) - old;
                    d[c] = (EDGE && p + 1 < NIT) ? S[c][p] * keep : S[c][p];
                }
            }
            const int yo = yi - H;
            if (yo >= ya && yo < yb) {
                const uint32_t roff = (uint32_t)yo * (uint32_t)nx * 4u;
                if (out0) buf_st_f32((float)(d[0] * scale), pr, vo0, roff);
                if (out1) buf_st_f32((float)(d[1] * scale), pr, vo1, roff);
            }
        }
        // the rings hold exactly the current windows: re-anchor the sums
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int p = 0; p < NIT; ++p) {
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < Q; ++j) acc += ring[c][p][j];
                S[c][p] = acc;
            }
    };

    // Block b is computed from LDS buffer b & 1 while block b + 1 waits in
    // the other buffer and block b + 2 is in flight in registers.
    stage_load(0);
    stage_store(0);
    __syncthreads();
    if (nblk > 1) stage_load(1);
    for (int blk = 0; blk < nblk; ++blk) {
        const int buf = blk & 1;
        if (active) {
            // The interior copy of the row loop costs registers: only the
            // narrow cascades (halo <= 6) keep their waves per SIMD with it.
            if constexpr (H <= 6) {
                const int yb0 = y_first + blk * U;
                if (x_interior && yb0 - (NIT - 1) * R >= 0 && yb0 + U - 1 < ny)
                    compute(buf, blk, std::integral_constant<bool, false>{});
                else
                    compute(buf, blk, std::integral_constant<bool, true>{});
            } else {
                compute(buf, blk, std::integral_constant<bool, true>{});
            }
        }
        if (blk + 1 < nblk) {
            stage_store(buf ^ 1);
            if (blk + 2 < nblk) stage_load(blk + 2);
        }
        __syncthreads();
    }
}

template <int R, int NIT>
hipError_t launch_strip(const StripArgs &a, int xtype, bool repl, hipStream_t s) {
    const dim3 grid((unsigned)a.tiles), block(64 * a.wpb);
#define SC_STRIP(XT, RP) \
    hipLaunchKernelGGL((k_strip<R, NIT, XT, RP>), grid, block, 0, s, a)
    if (xtype == ST_F16) {
        if (repl) SC_STRIP(ST_F16, true); else SC_STRIP(ST_F16, false);
    } else if (xtype == ST_BF16) {
        if (repl) SC_STRIP(ST_BF16, true); else SC_STRIP(ST_BF16, false);
    } else {
        if (repl) SC_STRIP(ST_F32, true); else SC_STRIP(ST_F32, false);
    }
#undef SC_STRIP
    return hipGetLastError();
}

}  // namespace sc
