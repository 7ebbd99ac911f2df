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

#include "sc_internal.h"

namespace sc {

// ----------------------------------------------------------------- helpers

__device__ __forceinline__ bool in_flux_range(double s, int range) {
    return range < 0 ? (s < 0.0) : (range > 0 ? (s > 0.0) : true);
}

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

__global__ void k_set_sigma0(DevState *st, double sigma0) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->sigma0 = sigma0;
        st->status = 0;
        st->thr = 0.0;
        st->m = 0;
        for (int k = 0; k < SOFIA_SC_MAX_KERNELS; ++k) st->sigma[k] = NAN;
    }
}

// ------------------------------------------------------ spatial cascade

// One boxcar pass over register array `in`, writing out[i] for i in
// [LO, HI): unnormalised sum of in[i-R .. i+R]. For R = 1 the three taps are
// summed directly (as cheap as a running sum); wider boxcars use a running
// sum recomputed directly every kAnchor outputs, which bounds the FP32
// rounding carried along a row by the terms that already left the window.
constexpr int kAnchor = 4;
template <int N, int R, int LO, int HI>
__device__ __forceinline__ void box_pass(const float (&in)[N], float (&out)[N]) {
    float s = 0.f;
#pragma unroll
    for (int i = LO; i < HI; ++i) {
        if (R == 1 || (i - LO) % kAnchor == 0) {
            s = 0.f;
#pragma unroll
            for (int j = -R; j <= R; ++j) s += in[i + j];
        } else {
            s += in[i + R] - in[i - R - 1];
        }
        out[i] = s;
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
    const float *xp = a.x + z * nx * ny;
    const uint8_t *wp = a.wm ? a.wm + z * nx * ny : nullptr;
    const bool repl = a.repl_on && wp != nullptr;
    const float rv = repl ? (float)(a.repl_n * a.st->sigma0) : 0.f;
    const bool xedge = EDGE && ((x0 - H < 0) || (x0 + 64 + H > nx));
    const bool yedge = EDGE && ((y0 - H < 0) || (y0 - H + 64 > ny));

    // Stage the region (64 rows x RW columns): lanes take columns lane and
    // 64 + lane (the latter only for the 2H right-halo columns). Rows are
    // fetched in batches so many loads are in flight at once.
    constexpr int kRows = 8;
    const bool has2 = lane < 2 * H;
    for (int r0 = 0; r0 < 64; r0 += kRows) {
        float v0[kRows], v1[kRows];
        uint8_t m0[kRows], m1[kRows];
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            const int64_t gy = y0 - H + r0 + k;
            const int64_t gx0 = x0 - H + lane, gx1 = gx0 + 64;
            v0[k] = v1[k] = 0.f;
            m0[k] = m1[k] = 0;
            const bool yin = !yedge || (gy >= 0 && gy < ny);
            if (yin) {
                const int64_t row = gy * nx;
                if (!xedge || (gx0 >= 0 && gx0 < nx)) {
                    v0[k] = xp[row + gx0];
                    if (repl) m0[k] = wp[row + gx0];
                }
                if (has2 && (!xedge || gx1 < nx)) {
                    v1[k] = xp[row + gx1];
                    if (repl) m1[k] = wp[row + gx1];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            float *dst = lds + (r0 + k) * P1;
            const bool f0 = isfinite(v0[k]), f1 = isfinite(v1[k]);
            float y0v = f0 ? v0[k] : 0.f, y1v = f1 ? v1[k] : 0.f;
            if (f0 && (m0[k] & kDet)) y0v = copysignf(rv, v0[k]);
            if (f1 && (m1[k] & kDet)) y1v = copysignf(rv, v1[k]);
            dst[lane] = y0v;
            if (has2) dst[64 + lane] = y1v;
        }
    }
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

// ------------------------------------------------------ column streaming

struct ColAcc {
    double sum;
    unsigned long long cnt;
};

// One thread per (x, y) column. The column is streamed as a sequence of
// input planes zi = z0 - h .. z1 - 1 + h (the leading edge of the spectral
// window); after input zi the window sum S covers planes zi - 2h .. zi, i.e.
// the output plane z = zi - h. Inputs are fetched in groups of U planes and
// the next group is requested before the current one is consumed, so every
// wave keeps up to 2U plane reads in flight.
//
// Ring buffers (LDS, one slot per thread per plane of the window): the FP32
// inputs of the window, for the running sum; with SRC_X also the working-mask
// byte read at the leading edge, reused when that plane becomes the output.
template <int SRC, int OP, bool SPEC, bool HASWM>
__global__ __launch_bounds__(kColThreads) void k_column(ColArgs a) {
    extern __shared__ float dyn_lds[];
    constexpr int B = kColThreads;
    constexpr int U = 8;
    const int tid = threadIdx.x;
    const int cb = (int)(blockIdx.x % (unsigned)a.ncb);
    const int zc = (int)(blockIdx.x / (unsigned)a.ncb);
    const int64_t c = (int64_t)cb * B + tid;
    const bool active = c < a.ncol;
    const int64_t ncol = a.ncol, nz = a.nz;
    const int64_t z0 = (int64_t)zc * a.zchunk;
    const int64_t z1 = min(nz, z0 + (int64_t)a.zchunk);
    const int w = SPEC ? a.w : 1;
    const int h = SPEC ? a.h : 0;

    // LDS layout: float ring [w][B] | byte ring [w][B] (SRC_X, SPEC) | histogram
    float *ring = dyn_lds;
    uint8_t *bring = (uint8_t *)(dyn_lds + (SPEC ? w * B : 0));
    unsigned *hist = (unsigned *)(bring + ((SPEC && SRC == SRC_X) ? ((w * B + 3) & ~3) : 0));
    constexpr int kHistWords = OP == OP_HIST1 ? kL1Bins : (OP == OP_HIST2 ? 2 * kL2Coarse : 0);
    if (kHistWords) {
        for (int i = tid; i < kHistWords; i += B) hist[i] = 0u;
    }
    if (SPEC) {
        for (int j = 0; j < w; ++j) {
            ring[j * B + tid] = 0.f;
            if (SRC == SRC_X) bring[j * B + tid] = 0;
        }
    }
    if (kHistWords) __syncthreads();

    const bool repl = SRC == SRC_X && HASWM && a.repl_on;
    const float rv = repl ? (float)(a.repl_n * a.st->sigma0) : 0.f;
    const double T = (OP == OP_CLIP) ? a.st->thr : 0.0;
    uint32_t b0 = 0xffffffffu, b1 = 0xffffffffu;
    if (OP == OP_HIST2) { b0 = a.st->bin[0]; b1 = a.st->bin[1]; }
    const int range = a.range;
    ColAcc acc{0.0, 0ull};
    const float *src = SRC == SRC_X ? a.x : a.p;

    auto consume = [&](int64_t i, double s, bool blank, uint8_t wb) {
        if (OP == OP_STD) {
            if (!blank && in_flux_range(s, range)) { acc.sum += s * s; acc.cnt += 1; }
        } else if (OP == OP_HIST1) {
            if (!blank && in_flux_range(s, range)) {
                const uint32_t key = __float_as_uint(fabsf((float)s));
                atomicAdd(&hist[key >> kL1Shift], 1u);
            }
        } else if (OP == OP_HIST2) {
            if (!blank && in_flux_range(s, range)) {
                const uint32_t key = __float_as_uint(fabsf((float)s));
                const uint32_t k1 = key >> kL1Shift;
                const uint32_t lo = key & (kL2Bins - 1);
                if (k1 == b0) {
                    atomicAdd(&a.hist2[lo], 1ull);
                    atomicAdd(&hist[lo >> kL2CoarseShift], 1u);
                }
                if (k1 == b1 && b1 != b0) {
                    atomicAdd(&a.hist2[kL2Bins + lo], 1ull);
                    atomicAdd(&hist[kL2Coarse + (lo >> kL2CoarseShift)], 1u);
                }
            }
        } else if (OP == OP_CLIP) {
            const uint8_t det = (!blank && fabs(s) > T) ? kDet : 0;
            uint8_t out;
            if (a.out_user) out = (uint8_t)((wb & kDet) | det);
            else out = (uint8_t)(wb | det | (blank ? kBlank : 0));
            a.mask_out[i] = out;
        } else {  // OP_WRITE
            a.s_out[i] = blank ? NAN : (float)s;
        }
    };

    // Spectral input of a raw voxel: blanked -> 0, detected -> +-n sigma_0.
    auto raw_value = [&](float xv, uint8_t wb) -> float {
        if (!isfinite(xv)) return 0.f;
        if (repl && (wb & kDet)) return copysignf(rv, xv);
        return xv;
    };

    struct Group {
        float v[U];
        uint8_t b[U];
    };
    // Input planes zi = zb .. zb + U - 1 (SPEC) or output planes (not SPEC).
    auto load_group = [&](int64_t zb, Group &g) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t zi = zb + u;
            g.v[u] = 0.f;
            g.b[u] = 0;
            if (!SPEC) {
                if (zi < z1) {
                    const int64_t i = zi * ncol + c;
                    g.v[u] = src[i];
                    if (HASWM) g.b[u] = a.wm_in[i];
                }
            } else {
                const bool in_run = zi < z1 + h;
                if (in_run && zi >= 0 && zi < nz) {
                    const int64_t i = zi * ncol + c;
                    g.v[u] = src[i];
                    if (SRC == SRC_X) g.b[u] = a.wm_in[i];
                }
                if (SRC == SRC_P) {
                    const int64_t zo = zi - h;
                    if (in_run && zo >= z0) g.b[u] = a.wm_in[zo * ncol + c];
                }
            }
        }
    };

    double S = 0.0;
    int slot = 0;
    const double inv_w = SPEC ? 1.0 / (double)w : 1.0;
    const int64_t zstart = SPEC ? z0 - h : z0;
    const int64_t zend = SPEC ? z1 + h : z1;   // exclusive
    int64_t step = 0;

    auto process_group = [&](int64_t zb, const Group &g) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t zi = zb + u;
            if (zi >= zend) break;
            if (!SPEC) {
                const int64_t i = zi * ncol + c;
                if (SRC == SRC_X) {
                    const bool blank = !isfinite(g.v[u]);
                    consume(i, (double)raw_value(g.v[u], g.b[u]), blank, g.b[u]);
                } else {
                    consume(i, (double)g.v[u], (g.b[u] & kBlank) != 0, g.b[u]);
                }
            } else {
                const float vn = SRC == SRC_X ? raw_value(g.v[u], g.b[u]) : g.v[u];
                const float vo = ring[slot * B + tid];
                ring[slot * B + tid] = vn;
                uint8_t wb_out;
                if (SRC == SRC_X) {
                    bring[slot * B + tid] = g.b[u];
                    int os = slot + h + 1;
                    if (os >= w) os -= w;
                    wb_out = bring[os * B + tid];
                } else {
                    wb_out = g.b[u];
                }
                S += (double)vn - (double)vo;
                if (++slot == w) slot = 0;
                if ((++step & 63) == 0) {   // re-anchor the running sum
                    S = 0.0;
                    for (int j = 0; j < w; ++j) S += (double)ring[j * B + tid];
                }
                const int64_t zo = zi - h;
                if (zo >= z0) consume(zo * ncol + c, S * inv_w, (wb_out & kBlank) != 0, wb_out);
            }
        }
    };

    if (active) {
        Group ga, gb;
        load_group(zstart, ga);
        for (int64_t zb = zstart; zb < zend; zb += 2 * U) {
            if (zb + U < zend) load_group(zb + U, gb);
            process_group(zb, ga);
            if (zb + U >= zend) break;
            if (zb + 2 * U < zend) load_group(zb + 2 * U, ga);
            process_group(zb + U, gb);
        }
    }

    if (OP == OP_STD) {
        // Block reduction in a fixed order: deterministic partials.
        __shared__ double rs[B];
        __shared__ unsigned long long rc[B];
        rs[tid] = acc.sum;
        rc[tid] = acc.cnt;
        __syncthreads();
        for (int off = B / 2; off > 0; off >>= 1) {
            if (tid < off) { rs[tid] += rs[tid + off]; rc[tid] += rc[tid + off]; }
            __syncthreads();
        }
        if (tid == 0) { a.part_sum[blockIdx.x] = rs[0]; a.part_cnt[blockIdx.x] = rc[0]; }
    } else if (OP == OP_HIST1) {
        __syncthreads();
        for (int i = tid; i < kL1Bins; i += B)
            if (hist[i]) atomicAdd(&a.hist1[i], (unsigned long long)hist[i]);
    } else if (OP == OP_HIST2) {
        __syncthreads();
        for (int i = tid; i < 2 * kL2Coarse; i += B)
            if (hist[i]) atomicAdd(&a.hist2c[i], (unsigned long long)hist[i]);
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

// Level 1: locate the bins holding order statistics floor((m-1)/2) and
// floor(m/2) of the selected |s| and the ranks left inside them.
__global__ __launch_bounds__(256) void k_finalize_mad1(
    DevState *st, const unsigned long long *hist1) {
    __shared__ unsigned long long buf[256];
    constexpr int PER = kL1Bins / 256;
    const int tid = threadIdx.x;
    unsigned long long loc[PER];
    unsigned long long tot = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) { loc[j] = hist1[tid * PER + j]; tot += loc[j]; }
    const unsigned long long incl = block_scan_incl(tot, buf);
    const unsigned long long excl = incl - tot;
    const unsigned long long m = buf[255];
    if (tid == 0) {
        st->m = m;
        st->bin[0] = st->bin[1] = 0xffffffffu;
        st->rank[0] = st->rank[1] = 0ull;
        if (m == 0) st->status |= 1;
    }
    __syncthreads();
    if (m == 0) return;
    for (int q = 0; q < 2; ++q) {
        const unsigned long long r = q ? m / 2 : (m - 1) / 2;
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

// Level 2: walk the coarse then the fine histogram of each wanted bin to the
// exact key, and turn the two order statistics into sigma = 1.4826 x median.
__global__ __launch_bounds__(1024) void k_finalize_mad2(
    DevState *st, const unsigned long long *hist2,
    const unsigned long long *hist2c, int k, double t, int also0) {
    __shared__ unsigned long long buf[1024];
    __shared__ uint32_t key[2];
    __shared__ uint32_t cbin;
    __shared__ unsigned long long crank;
    const int tid = threadIdx.x;
    const unsigned long long m = st->m;
    if (m == 0) {
        if (tid == 0) put_sigma(st, k, also0, NAN, t);
        return;
    }
    for (int q = 0; q < 2; ++q) {
        const uint32_t bq = st->bin[q];
        const int arr = (q == 1 && bq != st->bin[0]) ? 1 : 0;
        const unsigned long long r = st->rank[q];
        if (tid == 0) { cbin = 0; crank = 0; key[q] = bq << kL1Shift; }
        __syncthreads();
        const unsigned long long v = hist2c[arr * kL2Coarse + tid];
        const unsigned long long incl = block_scan_incl(v, buf);
        if (r >= incl - v && r < incl) { cbin = (uint32_t)tid; crank = r - (incl - v); }
        __syncthreads();
        const uint32_t cb = cbin < (uint32_t)kL2Coarse ? cbin : 0u;
        const unsigned long long rr = crank;
        const unsigned long long fv =
            tid < kL2Fine ? hist2[(size_t)arr * kL2Bins + (size_t)cb * kL2Fine + tid] : 0ull;
        const unsigned long long fincl = block_scan_incl(fv, buf);
        if (tid < kL2Fine && rr >= fincl - fv && rr < fincl)
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

size_t column_lds_bytes(int src, int op, bool spectral, int w) {
    size_t b = 0;
    if (spectral) b += (size_t)w * kColThreads * sizeof(float);
    if (spectral && src == SRC_X) b += ((size_t)w * kColThreads + 3) & ~(size_t)3;
    if (op == OP_HIST1) b += (size_t)kL1Bins * sizeof(unsigned);
    if (op == OP_HIST2) b += (size_t)2 * kL2Coarse * sizeof(unsigned);
    return b;
}

template <int SRC, int OP, bool SPEC, bool HASWM>
static hipError_t column_inst(const ColArgs &a, int nblocks, hipStream_t s) {
    const size_t lds = column_lds_bytes(SRC, OP, SPEC, a.w);
    hipLaunchKernelGGL((k_column<SRC, OP, SPEC, HASWM>), dim3(nblocks),
                       dim3(kColThreads), lds, s, a);
    return hipGetLastError();
}

template <int SRC, int OP>
static hipError_t column_op(bool spec, bool has_wm, const ColArgs &a, int nb,
                            hipStream_t s) {
    if (SRC == SRC_P || spec) {
        if (!has_wm) return hipErrorInvalidValue;
        return spec ? column_inst<SRC, OP, true, true>(a, nb, s)
                    : column_inst<SRC, OP, false, true>(a, nb, s);
    }
    return has_wm ? column_inst<SRC, OP, false, true>(a, nb, s)
                  : column_inst<SRC, OP, false, false>(a, nb, s);
}

template <int SRC>
static hipError_t column_src(int op, bool spec, bool has_wm, const ColArgs &a,
                             int nb, hipStream_t s) {
    switch (op) {
        case OP_STD: return column_op<SRC, OP_STD>(spec, has_wm, a, nb, s);
        case OP_HIST1: return column_op<SRC, OP_HIST1>(spec, has_wm, a, nb, s);
        case OP_HIST2: return column_op<SRC, OP_HIST2>(spec, has_wm, a, nb, s);
        case OP_CLIP: return column_op<SRC, OP_CLIP>(spec, has_wm, a, nb, s);
        case OP_WRITE: return column_op<SRC, OP_WRITE>(spec, has_wm, a, nb, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_column(int src, int op, bool spectral, bool has_wm,
                         const ColArgs &a, int nblocks, hipStream_t s) {
    return src == SRC_X ? column_src<SRC_X>(op, spectral, has_wm, a, nblocks, s)
                        : column_src<SRC_P>(op, spectral, has_wm, a, nblocks, s);
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

hipError_t launch_finalize_mad2(DevState *st, const unsigned long long *hist2,
                                const unsigned long long *hist2c, int k, double t,
                                int also_sigma0, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_mad2, dim3(1), dim3(1024), 0, s, st, hist2,
                       hist2c, k, t, also_sigma0);
    return hipGetLastError();
}

}  // namespace sc
