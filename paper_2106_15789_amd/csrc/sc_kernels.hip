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
// With edge set, entries whose global coordinate lies outside the cube
// (local index outside [lo, hi)) are zeroed after the pass, so every pass
// sees zeros beyond the cube edge.
template <int N, int R, int P, int NIT>
struct Cascade {
    __device__ __forceinline__ static void run(float (&v)[N], bool edge, int lo,
                                               int hi) {
        float o[N];
        box_pass<N, R, P * R, N - P * R>(v, o);
#pragma unroll
        for (int i = P * R; i < N - P * R; ++i)
            v[i] = (edge && (i < lo || i >= hi)) ? 0.f : o[i];
        Cascade<N, R, P + 1, NIT>::run(v, edge, lo, hi);
    }
};
template <int N, int R, int NIT>
struct Cascade<N, R, NIT + 1, NIT> {
    __device__ __forceinline__ static void run(float (&)[N], bool, int, int) {}
};

template <int R, int NIT>
__global__ __launch_bounds__(64) void k_spatial(SpatialArgs a) {
    constexpr int H = R * NIT;          // halo consumed by the cascade
    constexpr int RW = 64 + 2 * H;      // region width
    constexpr int P1 = RW + 1;          // odd LDS pitch: conflict-free rows
    constexpr int P2 = 65;
    constexpr int TY = 64 - 2 * H;      // output rows per tile
    static_assert(TY >= 1, "halo too large for a 64-row region");
    __shared__ float lds[64 * P1];

    const int lane = threadIdx.x;
    const int64_t tiles = (int64_t)a.tiles_x * a.tiles_y;
    const int64_t z = (int64_t)blockIdx.x / tiles;
    const int64_t t = (int64_t)blockIdx.x - z * tiles;
    const int ty = (int)(t / a.tiles_x);
    const int tx = (int)(t - (int64_t)ty * a.tiles_x);
    const int64_t nx = a.nx, ny = a.ny;
    const int64_t x0 = (int64_t)tx * 64, y0 = (int64_t)ty * TY;
    const float *xp = a.x + z * nx * ny;
    const uint8_t *wp = a.wm ? a.wm + z * nx * ny : nullptr;
    const bool repl = a.repl_on && wp != nullptr;
    const float rv = repl ? (float)(a.repl_n * a.st->sigma0) : 0.f;

    // Stage the region (64 rows x RW columns) with blanking and replacement.
    // The region is walked as one flat array so every load instruction of the
    // wave is (nearly) contiguous; loads are issued in batches of kBatch so
    // many are in flight before the first LDS store waits on them.
    constexpr int NE = 64 * RW;
    constexpr int kBatch = 16;
    for (int e0 = 0; e0 < NE; e0 += 64 * kBatch) {
        float v[kBatch];
        uint8_t m[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int e = e0 + b * 64 + lane;
            const int row = e / RW, col = e - row * RW;
            const int64_t gy = y0 - H + row, gx = x0 - H + col;
            v[b] = 0.f;
            m[b] = 0;
            if (e < NE && gy >= 0 && gy < ny && gx >= 0 && gx < nx) {
                const int64_t idx = gy * nx + gx;
                v[b] = xp[idx];
                if (repl) m[b] = wp[idx];
            }
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int e = e0 + b * 64 + lane;
            const int row = e / RW, col = e - row * RW;
            const bool fin = isfinite(v[b]);
            float y = fin ? v[b] : 0.f;
            if (fin && (m[b] & kDet)) y = copysignf(rv, v[b]);
            if (e < NE) lds[row * P1 + col] = y;
        }
    }
    __syncthreads();

    // x passes: lane = region row.
    float r[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) r[i] = lds[lane * P1 + i];
    {
        const bool edge = (x0 - H < 0) || (x0 + 64 + H > nx);
        const int lo = (int)(H - x0);        // local index of gx = 0
        const int hi = (int)(nx - x0 + H);   // local index of gx = nx
        Cascade<RW, R, 1, NIT>::run(r, edge, lo, hi);
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
        const bool edge = (y0 - H < 0) || (y0 - H + 64 > ny);
        const int lo = (int)(H - y0);
        const int hi = (int)(ny - y0 + H);
        Cascade<64, R, 1, NIT>::run(c, edge, lo, hi);
    }
    double norm = 1.0;
    for (int p = 0; p < 2 * NIT; ++p) norm *= (double)(2 * R + 1);
    const float scale = (float)(1.0 / norm);
    const int64_t gx = x0 + lane;
    if (gx < nx) {
        float *pp = a.p + z * nx * ny;
#pragma unroll
        for (int j = 0; j < TY; ++j) {
            const int64_t gy = y0 + j;
            if (gy < ny) pp[gy * nx + gx] = c[H + j] * scale;
        }
    }
}

// ------------------------------------------------------ column streaming

struct ColAcc {
    double sum;
    unsigned long long cnt;
};

template <int SRC, int OP, bool SPEC, bool HASWM>
__global__ __launch_bounds__(kColThreads) void k_column(ColArgs a) {
    extern __shared__ float dyn_lds[];
    constexpr int B = kColThreads;
    const int tid = threadIdx.x;
    const int cb = (int)(blockIdx.x % (unsigned)a.ncb);
    const int zc = (int)(blockIdx.x / (unsigned)a.ncb);
    const int64_t c = (int64_t)cb * B + tid;
    const bool active = c < a.ncol;
    const int64_t ncol = a.ncol, nz = a.nz;
    const int64_t z0 = (int64_t)zc * a.zchunk;
    const int64_t z1 = min(nz, z0 + (int64_t)a.zchunk);

    float *ring = dyn_lds;                                   // [w][B]
    unsigned *hist = (unsigned *)(dyn_lds + (SPEC ? a.w * B : 0));
    if (OP == OP_HIST1) {
        for (int i = tid; i < kL1Bins; i += B) hist[i] = 0u;
        __syncthreads();
    }

    const float rv = (SRC == SRC_X && HASWM && a.repl_on)
                         ? (float)(a.repl_n * a.st->sigma0) : 0.f;
    const double T = (OP == OP_CLIP) ? a.st->thr : 0.0;
    uint32_t b0 = 0xffffffffu, b1 = 0xffffffffu;
    if (OP == OP_HIST2) { b0 = a.st->bin[0]; b1 = a.st->bin[1]; }
    const int range = a.range;
    ColAcc acc{0.0, 0ull};

    // Input of the spectral boxcar at (c, zz): replaced/blanked raw voxel or
    // the spatially smoothed value.
    auto value = [&](int64_t zz) -> float {
        const int64_t i = zz * ncol + c;
        if (SRC == SRC_X) {
            const float xv = a.x[i];
            if (!isfinite(xv)) return 0.f;
            if (HASWM && a.repl_on && (a.wm_in[i] & kDet)) return copysignf(rv, xv);
            return xv;
        } else {
            return a.p[i];
        }
    };

    // Per-voxel operation on the smoothed value s at (c, z).
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
                    atomicAdd(&a.hist2c[lo >> kL2CoarseShift], 1ull);
                }
                if (k1 == b1 && b1 != b0) {
                    atomicAdd(&a.hist2[kL2Bins + lo], 1ull);
                    atomicAdd(&a.hist2c[kL2Coarse + (lo >> kL2CoarseShift)], 1ull);
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

    // Planes are processed in groups of U: all loads of a group are issued
    // before any of them is consumed, so a wave keeps U plane reads in flight.
    constexpr int U = 8;
    if (active) {
        if (!SPEC) {
            for (int64_t zb = z0; zb < z1; zb += U) {
                float xv[U];
                uint8_t wv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t z = zb + u;
                    xv[u] = 0.f;
                    wv[u] = 0;
                    if (z < z1) {
                        const int64_t i = z * ncol + c;
                        xv[u] = SRC == SRC_X ? a.x[i] : a.p[i];
                        if (HASWM) wv[u] = a.wm_in[i];
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t z = zb + u;
                    if (z >= z1) break;
                    const int64_t i = z * ncol + c;
                    float v;
                    bool blank;
                    if (SRC == SRC_X) {
                        blank = !isfinite(xv[u]);
                        v = blank ? 0.f
                                  : ((HASWM && a.repl_on && (wv[u] & kDet)) ? copysignf(rv, xv[u])
                                                                            : xv[u]);
                    } else {
                        v = xv[u];
                        blank = (wv[u] & kBlank) != 0;
                    }
                    consume(i, (double)v, blank, wv[u]);
                }
            }
        } else {
            const int w = a.w, h = a.h;
            const double inv_w = 1.0 / (double)w;
            // Ring slot j holds plane z0 - 1 - h + j: the window of z0 - 1.
            double S = 0.0;
            for (int j = 0; j < w; ++j) {
                const int64_t zz = z0 - 1 - h + j;
                const float v = (zz >= 0 && zz < nz) ? value(zz) : 0.f;
                ring[j * B + tid] = v;
                S += (double)v;
            }
            int slot = 0;
            for (int64_t zb = z0; zb < z1; zb += U) {
                float vn[U];
                uint8_t wo[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t z = zb + u, zn = z + h;
                    vn[u] = (z < z1 && zn < nz) ? value(zn) : 0.f;
                    wo[u] = z < z1 ? a.wm_in[z * ncol + c] : (uint8_t)0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t z = zb + u;
                    if (z >= z1) break;
                    const float vo = ring[slot * B + tid];
                    ring[slot * B + tid] = vn[u];
                    S += (double)vn[u] - (double)vo;
                    if (++slot == w) slot = 0;
                    if (((z - z0) & 63) == 63) {   // re-anchor the running sum
                        S = 0.0;
                        for (int j = 0; j < w; ++j) S += (double)ring[j * B + tid];
                    }
                    consume(z * ncol + c, S * inv_w, (wo[u] & kBlank) != 0, wo[u]);
                }
            }
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
    const int64_t blocks = (int64_t)a.tiles_x * a.tiles_y * a.nz;
    hipLaunchKernelGGL((k_spatial<R, NIT>), dim3((unsigned)blocks), dim3(64), 0, s, a);
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

size_t column_lds_bytes(int op, bool spectral, int w) {
    size_t b = 0;
    if (spectral) b += (size_t)w * kColThreads * sizeof(float);
    if (op == OP_HIST1) b += (size_t)kL1Bins * sizeof(unsigned);
    return b;
}

template <int SRC, int OP, bool SPEC, bool HASWM>
static hipError_t column_inst(const ColArgs &a, int nblocks, hipStream_t s) {
    const size_t lds = column_lds_bytes(OP, SPEC, a.w);
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
