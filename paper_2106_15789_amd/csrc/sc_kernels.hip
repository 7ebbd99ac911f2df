// gfx950 kernels of the smooth-and-clip finder.
//
// Method (Westmeier et al. 2021, Sect. 4.2 and 6.2.4): for each kernel, the
// cube with earlier detections replaced by +-n sigma_0 is smoothed with a
// spatial Gaussian (boxcar cascade along x then y) and a spectral boxcar
// (along z), its noise is measured over the finite voxels of the flux range,
// and |s| > t sigma_k is ORed into the mask.
//
// Work split, chosen for HBM streaming rather than for the paper's OpenMP
// loops:
//  * k_spatial: one wave per 64-column tile of one z-plane. The tile plus
//    its halo is staged in LDS; each lane then runs the x passes of the
//    cascade on one row held in registers, the block is transposed through
//    LDS, and each lane runs the y passes on one column. Output: the
//    spatially smoothed plane (float32) in a work buffer.
//  * k_column: one thread per (x, y) column streams z with a ring of the
//    last w inputs in LDS and an FP64 running sum (exact for FP32 inputs),
//    and performs one per-voxel operation: accumulate sum s^2 (std noise),
//    count level-1 or level-2 histogram digits of |s| (exact MAD), or clip
//    into the mask. Lanes cover consecutive x, so every plane access of a
//    wave is one contiguous run.
//  * tiny one-block kernels turn the partial sums / histograms into sigma_k
//    on the device, so a run never waits on the host between launches.
#include <math.h>

#include <type_traits>

#include "sc_device.h"

namespace sc {

// ----------------------------------------------------------------- helpers

// Write a noise value and the threshold derived from it into the state.
__device__ void put_sigma(DevState *st, int k, int also_sigma0, double sig,
                          double t) {
    if (k >= 0) st->sigma[k] = sig;
    if (also_sigma0 || k < 0) st->sigma0 = sig;
    st->thr = t * sig;
}

// ---------------------------------------------------------- mask / fill

__global__ void k_init_mask(const float *__restrict__ x,
                            const uint8_t *__restrict__ mask_in,
                            uint8_t *__restrict__ wm, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += stride) {
        uint8_t b = isfinite(x[i]) ? 0 : kBlank;
        if (mask_in && mask_in[i]) b |= kDet;
        wm[i] = b;
    }
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += stride)
        p[i] = 0ull;
}

// q = RN_T(RN_f32(x * RN_f64(1 / scale))); finite values saturate to the
// largest finite value of T; non-finite values stay non-finite.
template <int T>
__global__ void k_quantize(const float *__restrict__ x, const DevState *st, double scale,
                           uint16_t *__restrict__ out, int64_t n) {
    const double inv = 1.0 / (st ? st->sigma0 : scale);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float xv = x[i];
        float y = (float)((double)xv * inv);
        uint16_t q;
        if (T == ST_F16) {
            if (isfinite(xv) && !(fabsf(y) <= 65504.f)) y = copysignf(65504.f, y);
            q = __builtin_bit_cast(uint16_t, (_Float16)y);
        } else {
            const float bmax = __uint_as_float(0x7f7f0000u);
            if (isfinite(xv) && !(fabsf(y) <= bmax)) y = copysignf(bmax, y);
            const uint32_t u = __float_as_uint(y);
            if (isnan(y)) q = (uint16_t)((u >> 16) | 0x0040u);
            else q = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
        }
        out[i] = q;
    }
}

__global__ void k_enter_scaled(DevState *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->scale = st->sigma0;
        st->sigma0 = 1.0;
    }
}

__global__ void k_set_sigma0(DevState *st, double sigma0) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->sigma0 = sigma0;
        st->status = 0;
        st->thr = 0.0;
        st->m = 0;
        st->use_capture = 0;
        st->klo = 1u;
        st->khi = 0u;
        st->below = 0ull;
        st->fallback = 0ull;
        st->scale = 1.0;
        for (int k = 0; k < SOFIA_SC_MAX_KERNELS; ++k) st->sigma[k] = NAN;
    }
}

// ------------------------------------------------------ spatial cascade

// One boxcar pass over register array `in`, writing out[i] for i in
// [LO, HI): the unnormalised sum of in[i-R .. i+R]. The running sum is kept
// in FP64, which holds sums of FP32 values exactly, so each output carries a
// single FP32 rounding; it is recomputed directly every kAnchor outputs.
constexpr int kAnchor = 32;
template <int N, int R, int LO, int HI>
__device__ __forceinline__ void box_pass(const float (&in)[N], float (&out)[N]) {
    double s = 0.0;
#pragma unroll
    for (int i = LO; i < HI; ++i) {
        if ((i - LO) % kAnchor == 0) {
            s = 0.0;
#pragma unroll
            for (int j = -R; j <= R; ++j) s += (double)in[i + j];
        } else {
            s += (double)in[i + R] - (double)in[i - R - 1];
        }
        out[i] = (float)s;
    }
}

// Pass P of NIT. Input valid on [(P-1)R, N-(P-1)R); output on [PR, N-PR).
// With EDGE set, entries whose global coordinate lies outside the cube
// (local index outside [lo, hi), the same for every lane) are zeroed after
// each pass, so every pass sees zeros beyond the cube edge; the zeroing is a
// multiply by a uniform 0/1 so it stays branch-free.
template <int N, int R, int P, int NIT, bool EDGE>
struct Cascade {
    __device__ __forceinline__ static void run(float (&v)[N], int lo, int hi) {
        float o[N];
        box_pass<N, R, P * R, N - P * R>(v, o);
#pragma unroll
        for (int i = P * R; i < N - P * R; ++i) {
            if (EDGE) {
                const float keep = (i >= lo && i < hi) ? 1.f : 0.f;
                v[i] = o[i] * keep;
            } else {
                v[i] = o[i];
            }
        }
        Cascade<N, R, P + 1, NIT, EDGE>::run(v, lo, hi);
    }
};
template <int N, int R, int NIT, bool EDGE>
struct Cascade<N, R, NIT + 1, NIT, EDGE> {
    __device__ __forceinline__ static void run(float (&)[N], int, int) {}
};

// Workgroups are handed to the 8 XCDs round-robin (block b runs on XCD
// b % 8). Remap so that each XCD works through one contiguous range of
// tiles: neighbouring tiles then share their halo rows and columns through
// the same L2 instead of fetching them from HBM once per XCD.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
    const int64_t q = nb / 8, r = nb % 8, x = b % 8;
    return x * q + (x < r ? x : r) + b / 8;
}

// Tile of the launch: interior launches cover the rectangle of tiles whose
// region lies inside the cube; edge launches cover the ring of the others.
__device__ __forceinline__ void spatial_tile(const SpatialArgs &a, bool edge, int64_t t,
                                             int &tx, int &ty) {
    if (!edge) {
        ty = a.ty_begin + (int)(t / a.ntx);
        tx = a.tx_begin + (int)(t - (int64_t)(ty - a.ty_begin) * a.ntx);
        return;
    }
    const int64_t T = a.tiles_x;
    const int64_t above = a.ty_begin, below = a.tiles_y - a.ty_begin - a.nty;
    const int64_t left = a.tx_begin, right = a.tiles_x - a.tx_begin - a.ntx;
    if (t < above * T) {
        ty = (int)(t / T);
        tx = (int)(t - (int64_t)ty * T);
    } else if (t < (above + below) * T) {
        const int64_t j = t - above * T;
        ty = (int)(a.ty_begin + a.nty + j / T);
        tx = (int)(j % T);
    } else {
        const int64_t j = t - (above + below) * T, per = left + right;
        const int64_t row = j / per, k = j - row * per;
        ty = (int)(a.ty_begin + row);
        tx = (int)(k < left ? k : a.tx_begin + a.ntx + (k - left));
    }
}

template <int R, int NIT, bool EDGE>
__global__ __launch_bounds__(64) void k_spatial(SpatialArgs a) {
    constexpr int H = R * NIT;          // halo consumed by the cascade
    constexpr int RW = 64 + 2 * H;      // region width
    constexpr int P1 = RW + 1;          // odd LDS pitch: conflict-free rows
    constexpr int P2 = 65;
    constexpr int TY = 64 - 2 * H;      // output rows per tile
    static_assert(TY >= 1, "halo too large for a 64-row region");
    static_assert(2 * H <= 64, "second column strip must fit in one wave");
    __shared__ float lds[64 * P1];

    const int lane = threadIdx.x;
    const int64_t tiles = a.tiles_per_plane;
    const int64_t tile = xcd_remap((int64_t)blockIdx.x, tiles * a.nz);
    const int64_t z = tile / tiles;
    int tx, ty;
    spatial_tile(a, EDGE, tile - z * tiles, tx, ty);
    const int64_t nx = a.nx, ny = a.ny;
    const int64_t x0 = (int64_t)tx * 64, y0 = (int64_t)ty * TY;
    const float *xp = a.x ? a.x + z * nx * ny : nullptr;
    const uint16_t *xqp = a.xq ? a.xq + z * nx * ny : nullptr;
    const uint8_t *wp = a.wm ? a.wm + z * nx * ny : nullptr;
    const bool repl = a.repl_on && wp != nullptr;
    const float rv = repl ? (float)(a.repl_n * a.st->sigma0) : 0.f;
    const bool xedge = EDGE && ((x0 - H < 0) || (x0 + 64 + H > nx));
    const bool yedge = EDGE && ((y0 - H < 0) || (y0 - H + 64 > ny));

    // Stage the region (64 rows x RW columns): lanes take columns lane and
    // 64 + lane (the latter only for the 2H right-halo columns). Rows are
    // fetched in batches so many loads are in flight at once. Every lane
    // loads, from coordinates clamped into the cube, and what lies outside
    // is zeroed afterwards: a load under a divergent branch makes the
    // compiler merge or convert its result at once, which waits for it and
    // serialises the batch. The clamped duplicates hit in cache.
    constexpr int kRows = 8;
    const bool has2 = lane < 2 * H;
    const int64_t gx0 = x0 - H + lane, gx1 = gx0 + 64;
    const bool in0 = !xedge || (gx0 >= 0 && gx0 < nx);
    const bool in1 = has2 && (!xedge || gx1 < nx);
    const int64_t cx0 = xedge ? (gx0 < 0 ? 0 : (gx0 >= nx ? nx - 1 : gx0)) : gx0;
    const int64_t cx1 = in1 ? gx1 : cx0;
    // One batch of kRows region rows for a compile-time storage type XT and
    // replacement flag RP (a run-time flag would put the mask loads under a
    // branch, with the same effect).
    auto stage = [&](auto xt, auto rp, int r0) {
        constexpr int XT = decltype(xt)::value;
        constexpr bool RP = decltype(rp)::value;
        auto ld = [&](int64_t i) -> float {
            if (XT == ST_F16) return f16_bits_to_float(xqp[i]);
            if (XT == ST_BF16) return bf16_bits_to_float(xqp[i]);
            return xp[i];
        };
        float v0[kRows], v1[kRows];
        uint32_t m0[kRows], m1[kRows];
        bool yin[kRows];
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            const int64_t gy = y0 - H + r0 + k;
            yin[k] = !yedge || (gy >= 0 && gy < ny);
            const int64_t cy = yedge ? (gy < 0 ? 0 : (gy >= ny ? ny - 1 : gy)) : gy;
            const int64_t row = cy * nx;
            v0[k] = ld(row + cx0);
            v1[k] = ld(row + cx1);
            m0[k] = RP ? wp[row + cx0] : 0u;
            m1[k] = RP ? wp[row + cx1] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            float *dst = lds + (r0 + k) * P1;
            const bool f0 = yin[k] && in0 && isfinite(v0[k]);
            const bool f1 = yin[k] && in1 && isfinite(v1[k]);
            float y0v = f0 ? v0[k] : 0.f, y1v = f1 ? v1[k] : 0.f;
            if (RP && f0 && (m0[k] & kDet)) y0v = copysignf(rv, v0[k]);
            if (RP && f1 && (m1[k] & kDet)) y1v = copysignf(rv, v1[k]);
            dst[lane] = y0v;
            if (has2) dst[64 + lane] = y1v;
        }
    };
    auto stage_all = [&](auto xt) {
        for (int r0 = 0; r0 < 64; r0 += kRows) {
            if (repl) stage(xt, std::true_type{}, r0);
            else stage(xt, std::false_type{}, r0);
        }
    };
    if (a.xtype == ST_F16) stage_all(std::integral_constant<int, ST_F16>{});
    else if (a.xtype == ST_BF16) stage_all(std::integral_constant<int, ST_BF16>{});
    else stage_all(std::integral_constant<int, ST_F32>{});
    __syncthreads();

    // x passes: lane = region row.
    float r[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) r[i] = lds[lane * P1 + i];
    {
        const int lo = xedge ? (int)(H - x0) : 0;            // local index of gx = 0
        const int hi = xedge ? (int)(nx - x0 + H) : RW;      // local index of gx = nx
        Cascade<RW, R, 1, NIT, EDGE>::run(r, lo, hi);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 64; ++i) lds[lane * P2 + i] = r[H + i];
    __syncthreads();

    // y passes: lane = tile column.
    float c[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) c[j] = lds[j * P2 + lane];
    {
        const int lo = yedge ? (int)(H - y0) : 0;
        const int hi = yedge ? (int)(ny - y0 + H) : 64;
        Cascade<64, R, 1, NIT, EDGE>::run(c, lo, hi);
    }
    double norm = 1.0;
    for (int p = 0; p < 2 * NIT; ++p) norm *= (double)(2 * R + 1);
    const float scale = (float)(1.0 / norm);
    const int64_t gx = x0 + lane;
    if (!EDGE || gx < nx) {
        float *pp = a.p + z * nx * ny + gx;
#pragma unroll
        for (int j = 0; j < TY; ++j) {
            const int64_t gy = y0 + j;
            if (!EDGE || gy < ny) pp[gy * nx] = c[H + j] * scale;
        }
    }
}

// ------------------------------------------------------------ finalize

// Inclusive Hillis-Steele scan of one value per thread (blockDim.x values).
__device__ unsigned long long block_scan_incl(unsigned long long v,
                                              unsigned long long *buf) {
    const int tid = threadIdx.x, n = blockDim.x;
    buf[tid] = v;
    __syncthreads();
    for (int off = 1; off < n; off <<= 1) {
        const unsigned long long add = tid >= off ? buf[tid - off] : 0ull;
        __syncthreads();
        buf[tid] += add;
        __syncthreads();
    }
    return buf[tid];
}

__global__ __launch_bounds__(256) void k_finalize_std(
    DevState *st, const double *ps, const unsigned long long *pc, int n, int k,
    double t, int also0) {
    __shared__ double ss[256];
    __shared__ unsigned long long sc[256];
    const int tid = threadIdx.x;
    double a = 0.0;
    unsigned long long c = 0;
    for (int i = tid; i < n; i += 256) { a += ps[i]; c += pc[i]; }
    ss[tid] = a;
    sc[tid] = c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) { ss[tid] += ss[tid + off]; sc[tid] += sc[tid + off]; }
        __syncthreads();
    }
    if (tid == 0) {
        double sig = NAN;
        if (sc[0] > 0) sig = sqrt(ss[0] / (double)sc[0]);
        else st->status |= 1;
        put_sigma(st, k, also0, sig, t);
    }
}

// Level 1: locate the level-1 bins holding order statistics floor((m-1)/2)
// and floor(m/2) of the selected |s|, and the ranks left inside them. The
// histogram counts either every selected key (full pass; below = 0) or only
// the captured keys, which sit above `below` smaller ones.
__global__ __launch_bounds__(256) void k_finalize_mad1(
    DevState *st, const unsigned long long *hist1) {
    __shared__ unsigned long long buf[256];
    constexpr int PER = kL1Bins / 256;
    const int tid = threadIdx.x;
    const unsigned long long m = st->m;
    if (tid == 0) {
        st->bin[0] = st->bin[1] = 0xffffffffu;
        st->rank[0] = st->rank[1] = 0ull;
    }
    __syncthreads();
    if (m == 0) return;
    unsigned long long loc[PER];
    unsigned long long tot = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) { loc[j] = hist1[tid * PER + j]; tot += loc[j]; }
    const unsigned long long incl = block_scan_incl(tot, buf);
    const unsigned long long excl = incl - tot;
    const unsigned long long below = st->below;
    for (int q = 0; q < 2; ++q) {
        const unsigned long long r = (q ? m / 2 : (m - 1) / 2) - below;
        if (r >= excl && r < incl) {
            unsigned long long run = excl;
            for (int j = 0; j < PER; ++j) {
                if (r < run + loc[j]) {
                    st->bin[q] = (uint32_t)(tid * PER + j);
                    st->rank[q] = r - run;
                    break;
                }
                run += loc[j];
            }
        }
    }
}

// After the selection pass: the captured keys decide the order statistics
// when the count below the window and the captured count bracket both ranks
// (and nothing was dropped); otherwise the full level-1/level-2 passes run.
__global__ void k_finalize_select(DevState *st, const unsigned long long *sel_counts,
                                  const unsigned long long *cap_count,
                                  unsigned long long cap_capacity, int k) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const unsigned long long m = sel_counts[0], below = sel_counts[1], cin = *cap_count;
    st->m = m;
    st->below = 0ull;
    if (m == 0) {                 // no voxel in the flux range
        st->status |= 1;
        st->use_capture = 1;      // nothing to select: skip every later pass
        return;
    }
    const unsigned long long r_lo = (m - 1) / 2, r_hi = m / 2;
    const bool ok = cin <= cap_capacity && below <= r_lo && r_hi < below + cin;
    st->use_capture = ok ? 1 : 0;
    if (ok) st->below = below;
    else st->fallback |= 1ull << (k >= 0 ? k : 63);
}

// Predict the median of |s| from the level-1 histogram of a sample of
// columns (linear interpolation inside the bin that holds each central rank)
// and set the capture window to that estimate -/+ delta, with
// delta = 2 % + 3 / sqrt(sample size).
__global__ __launch_bounds__(256) void k_finalize_predict(
    DevState *st, const unsigned long long *hist_s) {
    __shared__ unsigned long long buf[256];
    __shared__ float est[2];
    constexpr int PER = kL1Bins / 256;
    const int tid = threadIdx.x;
    unsigned long long loc[PER];
    unsigned long long tot = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) { loc[j] = hist_s[tid * PER + j]; tot += loc[j]; }
    const unsigned long long incl = block_scan_incl(tot, buf);
    const unsigned long long excl = incl - tot;
    const unsigned long long m = buf[255];
    if (tid == 0) { est[0] = 0.f; est[1] = 0.f; }
    __syncthreads();
    if (m > 0) {
        for (int q = 0; q < 2; ++q) {
            const unsigned long long r = q ? m / 2 : (m - 1) / 2;
            if (r >= excl && r < incl) {
                unsigned long long run = excl;
                for (int j = 0; j < PER; ++j) {
                    if (r < run + loc[j]) {
                        const double f = ((double)(r - run) + 0.5) / (double)loc[j];
                        const uint32_t b = (uint32_t)(tid * PER + j);
                        const uint32_t key =
                            (b << kL1Shift) + (uint32_t)(f * (double)(1u << kL1Shift));
                        est[q] = __uint_as_float(key);
                        break;
                    }
                    run += loc[j];
                }
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        if (m == 0) {   // empty sample: capture nothing; the full passes decide
            st->klo = 1u;
            st->khi = 0u;
        } else {
            const double delta = 0.02 + 3.0 / sqrt((double)m);
            const double lo = (double)est[0] * (1.0 - delta);
            const double hi = (double)est[1] * (1.0 + delta);
            st->klo = lo > 0.0 ? __float_as_uint((float)lo) : 0u;
            st->khi = hi < 3.0e38 ? __float_as_uint((float)hi) : 0x7f800000u;
        }
    }
}

// Level-1 histogram of the captured keys (capture path only).
__global__ __launch_bounds__(256) void k_capture_l1(
    const DevState *st, const uint32_t *cap_buf, const unsigned long long *cap_count,
    unsigned long long *hist1) {
    if (!st->use_capture || st->m == 0) return;
    __shared__ unsigned hl[kL1Bins];
    const int tid = threadIdx.x;
    for (int i = tid; i < kL1Bins; i += 256) hl[i] = 0u;
    __syncthreads();
    const unsigned long long n = *cap_count;
    const unsigned long long stride = (unsigned long long)gridDim.x * 256;
    for (unsigned long long i = (unsigned long long)blockIdx.x * 256 + tid; i < n; i += stride)
        atomicAdd(&hl[cap_buf[i] >> kL1Shift], 1u);
    __syncthreads();
    for (int i = tid; i < kL1Bins; i += 256)
        if (hl[i]) atomicAdd(&hist1[i], (unsigned long long)hl[i]);
}

// Level 2 from the captured keys (instead of a second pass over the cube),
// when the median bins fell inside the captured window. Two short passes
// over the key list with LDS histograms: first the coarse digit (bits
// 18..9) of the keys in each wanted level-1 bin, then, once the coarse bin
// of each order statistic is known, the fine digit (bits 8..0) of the keys
// in that coarse bin. The counts land in the same arrays the full level-2
// pass fills, so the rank walk is shared.
__global__ __launch_bounds__(256) void k_capture_coarse(
    const DevState *st, const uint32_t *cap_buf, const unsigned long long *cap_count,
    unsigned long long *hist2c) {
    if (!st->use_capture || st->m == 0) return;
    __shared__ unsigned hc[2 * kL2Coarse];
    const int tid = threadIdx.x;
    for (int i = tid; i < 2 * kL2Coarse; i += 256) hc[i] = 0u;
    __syncthreads();
    const uint32_t b0 = st->bin[0], b1 = st->bin[1];
    const unsigned long long n = *cap_count;
    const unsigned long long stride = (unsigned long long)gridDim.x * 256;
    for (unsigned long long i = (unsigned long long)blockIdx.x * 256 + tid; i < n; i += stride) {
        const uint32_t key = cap_buf[i];
        const uint32_t k1 = key >> kL1Shift;
        const uint32_t cbin = (key & (kL2Bins - 1)) >> kL2CoarseShift;
        if (k1 == b0) atomicAdd(&hc[cbin], 1u);
        if (k1 == b1 && b1 != b0) atomicAdd(&hc[kL2Coarse + cbin], 1u);
    }
    __syncthreads();
    for (int i = tid; i < 2 * kL2Coarse; i += 256)
        if (hc[i]) atomicAdd(&hist2c[i], (unsigned long long)hc[i]);
}

__global__ __launch_bounds__(256) void k_capture_fine(
    const DevState *st, const uint32_t *cap_buf, const unsigned long long *cap_count,
    unsigned long long *hist2) {
    if (!st->use_capture || st->m == 0) return;
    __shared__ unsigned hf[2 * kL2Fine];
    const int tid = threadIdx.x;
    for (int i = tid; i < 2 * kL2Fine; i += 256) hf[i] = 0u;
    __syncthreads();
    // (level-1 bin, coarse bin) prefix of each order statistic
    const uint32_t p0 = (st->bin[0] << kL1Shift) | (st->cbin[0] << kL2CoarseShift);
    const uint32_t p1 = (st->bin[1] << kL1Shift) | (st->cbin[1] << kL2CoarseShift);
    const int arr1 = st->bin[1] != st->bin[0] ? 1 : 0;
    const bool second = p1 != p0;   // else both ranks share one fine histogram
    const unsigned long long n = *cap_count;
    const unsigned long long stride = (unsigned long long)gridDim.x * 256;
    for (unsigned long long i = (unsigned long long)blockIdx.x * 256 + tid; i < n; i += stride) {
        const uint32_t key = cap_buf[i];
        const uint32_t pre = key & ~(uint32_t)(kL2Fine - 1);
        const uint32_t f = key & (kL2Fine - 1);
        if (pre == p0) atomicAdd(&hf[f], 1u);
        if (second && pre == p1) atomicAdd(&hf[kL2Fine + f], 1u);
    }
    __syncthreads();
    // Fine counts go to the level-2 array at (arr, coarse bin, fine digit).
    for (int i = tid; i < 2 * kL2Fine; i += 256) {
        if (!hf[i]) continue;
        const int q = i / kL2Fine, f = i % kL2Fine;
        const int arr = q == 0 ? 0 : arr1;
        const uint32_t cb = st->cbin[q];
        atomicAdd(&hist2[(size_t)arr * kL2Bins + (size_t)cb * kL2Fine + f],
                  (unsigned long long)hf[i]);
    }
}

// Level 2, coarse walk: for each wanted order statistic find the coarse bin
// (bits 18..9) inside its level-1 bin and the rank left inside it.
__global__ __launch_bounds__(1024) void k_finalize_mad2a(
    DevState *st, const unsigned long long *hist2c) {
    __shared__ unsigned long long buf[1024];
    const int tid = threadIdx.x;
    if (st->m == 0) return;
    for (int q = 0; q < 2; ++q) {
        const int arr = (q == 1 && st->bin[1] != st->bin[0]) ? 1 : 0;
        const unsigned long long r = st->rank[q];
        if (tid == 0) { st->cbin[q] = 0u; st->crank[q] = 0ull; }
        __syncthreads();
        const unsigned long long v = hist2c[arr * kL2Coarse + tid];
        const unsigned long long incl = block_scan_incl(v, buf);
        if (r >= incl - v && r < incl) { st->cbin[q] = (uint32_t)tid; st->crank[q] = r - (incl - v); }
        __syncthreads();
    }
}

// Level 2, fine walk: the exact key of each order statistic, then
// sigma = 1.4826 x median (mean of the two central order statistics).
__global__ __launch_bounds__(512) void k_finalize_mad2b(
    DevState *st, const unsigned long long *hist2, int k, double t, int also0) {
    __shared__ unsigned long long buf[512];
    __shared__ uint32_t key[2];
    const int tid = threadIdx.x;
    if (st->m == 0) {
        if (tid == 0) put_sigma(st, k, also0, NAN, t);
        return;
    }
    for (int q = 0; q < 2; ++q) {
        const uint32_t bq = st->bin[q];
        const int arr = (q == 1 && bq != st->bin[0]) ? 1 : 0;
        const uint32_t cb = st->cbin[q] < (uint32_t)kL2Coarse ? st->cbin[q] : 0u;
        const unsigned long long rr = st->crank[q];
        if (tid == 0) key[q] = (bq << kL1Shift) | (cb << kL2CoarseShift);
        __syncthreads();
        const unsigned long long fv = hist2[(size_t)arr * kL2Bins + (size_t)cb * kL2Fine + tid];
        const unsigned long long fincl = block_scan_incl(fv, buf);
        if (rr >= fincl - fv && rr < fincl)
            key[q] = (bq << kL1Shift) | (cb << kL2CoarseShift) | (uint32_t)tid;
        __syncthreads();
    }
    if (tid == 0) {
        const double v0 = (double)__uint_as_float(key[0]);
        const double v1 = (double)__uint_as_float(key[1]);
        const double med = 0.5 * (v0 + v1);
        put_sigma(st, k, also0, kMadFactor * med, t);
    }
}

// ------------------------------------------------------------ launchers

static int grid_for(int64_t n, int threads, int cap) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_init_mask(const float *x, const uint8_t *mask_in, uint8_t *wm,
                            int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_init_mask, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s,
                       x, mask_in, wm, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_quantize(const float *x, const DevState *st, double scale, int type,
                           uint16_t *out, int64_t n, hipStream_t s) {
    const dim3 grid(grid_for(n, 256, 16384)), block(256);
    if (type == ST_F16)
        hipLaunchKernelGGL(k_quantize<ST_F16>, grid, block, 0, s, x, st, scale, out, n);
    else if (type == ST_BF16)
        hipLaunchKernelGGL(k_quantize<ST_BF16>, grid, block, 0, s, x, st, scale, out, n);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_enter_scaled(DevState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_enter_scaled, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_set_sigma0(DevState *st, double sigma0, hipStream_t s) {
    hipLaunchKernelGGL(k_set_sigma0, dim3(1), dim3(64), 0, s, st, sigma0);
    return hipGetLastError();
}

template <int R, int NIT>
static hipError_t spatial_inst(const SpatialArgs &a, hipStream_t s) {
    const int64_t n_int = (int64_t)a.ntx * a.nty;
    const int64_t n_edge = (int64_t)a.tiles_x * a.tiles_y - n_int;
    if (n_int > 0) {
        SpatialArgs b = a;
        b.tiles_per_plane = n_int;
        hipLaunchKernelGGL((k_spatial<R, NIT, false>), dim3((unsigned)(n_int * a.nz)),
                           dim3(64), 0, s, b);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_edge > 0) {
        SpatialArgs b = a;
        b.tiles_per_plane = n_edge;
        hipLaunchKernelGGL((k_spatial<R, NIT, true>), dim3((unsigned)(n_edge * a.nz)),
                           dim3(64), 0, s, b);
    }
    return hipGetLastError();
}

hipError_t launch_spatial(int n_iter, int radius, const SpatialArgs &a,
                          hipStream_t s) {
#define SC_SP(N, R) \
    if (n_iter == N && radius == R) return spatial_inst<R, N>(a, s);
    SC_SP(3, 1) SC_SP(3, 2) SC_SP(3, 3) SC_SP(3, 4) SC_SP(3, 5)
    SC_SP(4, 1) SC_SP(4, 2) SC_SP(4, 3) SC_SP(4, 4)
    SC_SP(5, 1) SC_SP(5, 2) SC_SP(5, 3)
    SC_SP(6, 1) SC_SP(6, 2)
#undef SC_SP
    return hipErrorInvalidValue;
}

template <int OP>
hipError_t launch_column_op(int src, bool spec, bool has_wm, const ColArgs &a, int nb,
                            hipStream_t s);

hipError_t launch_column(int src, int op, bool spectral, bool has_wm,
                         const ColArgs &a, int nblocks, hipStream_t s) {
    switch (op) {
        case OP_STD: return launch_column_op<OP_STD>(src, spectral, has_wm, a, nblocks, s);
        case OP_HIST1: return launch_column_op<OP_HIST1>(src, spectral, has_wm, a, nblocks, s);
        case OP_HIST2: return launch_column_op<OP_HIST2>(src, spectral, has_wm, a, nblocks, s);
        case OP_CLIP: return launch_column_op<OP_CLIP>(src, spectral, has_wm, a, nblocks, s);
        case OP_WRITE: return launch_column_op<OP_WRITE>(src, spectral, has_wm, a, nblocks, s);
        case OP_SELECT: return launch_column_op<OP_SELECT>(src, spectral, has_wm, a, nblocks, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_finalize_std(DevState *st, const double *part_sum,
                               const unsigned long long *part_cnt, int nparts,
                               int k, double t, int also_sigma0, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_std, dim3(1), dim3(256), 0, s, st, part_sum,
                       part_cnt, nparts, k, t, also_sigma0);
    return hipGetLastError();
}

hipError_t launch_finalize_mad1(DevState *st, const unsigned long long *hist1,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_mad1, dim3(1), dim3(256), 0, s, st, hist1);
    return hipGetLastError();
}

hipError_t launch_finalize_select(DevState *st, const unsigned long long *sel_counts,
                                  const unsigned long long *cap_count,
                                  unsigned long long cap_capacity, int k, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_select, dim3(1), dim3(64), 0, s, st, sel_counts,
                       cap_count, cap_capacity, k);
    return hipGetLastError();
}

hipError_t launch_capture_l1(const DevState *st, const uint32_t *cap_buf,
                             const unsigned long long *cap_count,
                             unsigned long long *hist1, hipStream_t s) {
    hipLaunchKernelGGL(k_capture_l1, dim3(512), dim3(256), 0, s, st, cap_buf, cap_count,
                       hist1);
    return hipGetLastError();
}

hipError_t launch_finalize_predict(DevState *st, const unsigned long long *hist_s,
                                   hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_predict, dim3(1), dim3(256), 0, s, st, hist_s);
    return hipGetLastError();
}

hipError_t launch_capture_coarse(const DevState *st, const uint32_t *cap_buf,
                                 const unsigned long long *cap_count,
                                 unsigned long long *hist2c, hipStream_t s) {
    hipLaunchKernelGGL(k_capture_coarse, dim3(1024), dim3(256), 0, s, st, cap_buf,
                       cap_count, hist2c);
    return hipGetLastError();
}

hipError_t launch_capture_fine(const DevState *st, const uint32_t *cap_buf,
                               const unsigned long long *cap_count,
                               unsigned long long *hist2, hipStream_t s) {
    hipLaunchKernelGGL(k_capture_fine, dim3(1024), dim3(256), 0, s, st, cap_buf,
                       cap_count, hist2);
    return hipGetLastError();
}

hipError_t launch_finalize_mad2a(DevState *st, const unsigned long long *hist2c,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_mad2a, dim3(1), dim3(1024), 0, s, st, hist2c);
    return hipGetLastError();
}

hipError_t launch_finalize_mad2b(DevState *st, const unsigned long long *hist2, int k,
                                 double t, int also_sigma0, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_mad2b, dim3(1), dim3(512), 0, s, st, hist2, k, t,
                       also_sigma0);
    return hipGetLastError();
}

}  // namespace sc
