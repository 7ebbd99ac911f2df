// Local noise normalisation (Westmeier et al. 2021, Sect. 4.1, last
// paragraph): where the noise level varies across the cube, the cube is
// divided by the noise measured in a running window before a constant
// threshold is applied; the speed test of Sect. 5 uses a 31-pixel,
// 31-channel window.
//
// The noise is measured on a grid: each axis is cut into blocks of g voxels
// (the last one may be shorter), the window of a block is the w voxels
// centred on the block's middle voxel (lower middle for an even length),
// clipped to the cube, and every voxel of the block is divided by the noise
// of that window. The estimators are those of the smooth-and-clip noise: RMS
// about zero, or 1.4826 x the median of |v| (mean of the two central order
// statistics for an even count), over finite voxels of the flux range.
//
//  * k_window_noise: one workgroup per block. Its waves stream the window's
//    rows (two 32-lane row slots per wave when the window is at most 32
//    voxels wide) straight from HBM. For the median, the keys (bit patterns
//    of |v|, which order like the values) of the selected voxels are staged
//    in LDS while a level-1 histogram of their top 11 bits is counted; three
//    histogram levels (11 + 10 + 10 bits) then find the lower central order
//    statistic exactly, and a min-reduction over the keys above it gives the
//    upper one when they differ. No key leaves the CU. For the RMS, FP64
//    partial sums are reduced in a fixed order.
//  * k_norm_divide: streams the cube row by row (4 B in, 4 B out per voxel);
//    the block indices of a row are uniform, and the division is done in
//    FP64 and rounded to FP32 once.
#include <math.h>

#include "sc_device.h"

namespace sc {

namespace {

// Block bi of an axis of n voxels cut into blocks of g: its window
// [lo, hi] of half-width r around the block's middle voxel, clipped.
__device__ __forceinline__ void window_bounds(int64_t bi, int64_t n, int g, int w,
                                              int64_t &lo, int64_t &hi) {
    const int64_t first = bi * g;
    const int64_t last = (first + g < n ? first + g : n) - 1;
    const int64_t mid = first + (last - first) / 2;
    const int64_t r = (w - 1) / 2;
    lo = mid - r < 0 ? 0 : mid - r;
    hi = mid + r > n - 1 ? n - 1 : mid + r;
}

// Bin of rank `rank` (0-based) in an LDS histogram of nbins counts: every
// thread sums a contiguous run of bins, a block scan of the run sums finds
// the run holding the rank, and its thread walks it. Writes the bin and the
// count of keys below it to out[0], out[1]. All threads call it.
__device__ void find_rank(const uint32_t *hist, int nbins, uint32_t rank, uint32_t *scan,
                          uint32_t *out) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int per = (nbins + nt - 1) / nt;
    const int b0 = tid * per, b1 = min(nbins, b0 + per);
    uint32_t run = 0;
    for (int b = b0; b < b1; ++b) run += hist[b];
    // inclusive scan of the run sums: wave scan, then the wave totals
    const int lane = tid & 63, wave = tid >> 6;
    uint32_t v = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    if (lane == 63) scan[wave] = v;
    __syncthreads();
    if (tid == 0) {
        uint32_t acc = 0;
        for (int w = 0; w < nt / 64; ++w) {
            const uint32_t t = scan[w];
            scan[w] = acc;
            acc += t;
        }
    }
    __syncthreads();
    const uint32_t incl = v + scan[wave];
    const uint32_t excl = incl - run;
    if (run && rank >= excl && rank < incl) {
        uint32_t below = excl;
        for (int b = b0; b < b1; ++b) {
            if (rank < below + hist[b]) {
                out[0] = (uint32_t)b;
                out[1] = below;
                break;
            }
            below += hist[b];
        }
    }
    __syncthreads();
}

}  // namespace

template <bool MAD>
__global__ __launch_bounds__(kNormThreads) void k_window_noise(NormArgs a) {
    extern __shared__ uint32_t lds[];
    // MAD: keys [wxy * wxy * wz] | histogram [2048]; RMS: nothing dynamic
    __shared__ uint32_t scan[kNormThreads / 64];
    __shared__ uint32_t res[8];
    __shared__ double psum[kNormThreads / 64];
    __shared__ unsigned long long pcnt[kNormThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nwaves = blockDim.x >> 6;

    const int64_t nb = (int64_t)a.nbx * a.nby * a.nbz;
    const int64_t b = xcd_remap((int64_t)blockIdx.x, nb);
    const int64_t bx = b % a.nbx, by = (b / a.nbx) % a.nby, bz = b / ((int64_t)a.nbx * a.nby);
    int64_t x0, x1, y0, y1, z0, z1;
    window_bounds(bx, a.nx, a.gxy, a.wxy, x0, x1);
    window_bounds(by, a.ny, a.gxy, a.wxy, y0, y1);
    window_bounds(bz, a.nz, a.gz, a.wz, z0, z1);
    const int wx = (int)(x1 - x0 + 1), wy = (int)(y1 - y0 + 1);
    const int nrows = wy * (int)(z1 - z0 + 1);
    // row slots: two 32-lane slots per wave for narrow windows
    const bool two = wx <= 32;
    const int slot = two ? lane >> 5 : 0, sl = two ? lane & 31 : lane;
    const int step_x = two ? 32 : 64, slots = nwaves * (two ? 2 : 1);

    uint32_t *keys = lds;
    uint32_t *hist = lds + (int64_t)a.wxy * a.wxy * a.wz;   // after the largest window's keys
    if (MAD) {
        for (int i = tid; i < 2048; i += blockDim.x) hist[i] = 0u;
        if (tid == 0) res[0] = 0u;   // keys staged
        __syncthreads();
    }
    const bool all_range = a.range == 0;
    const float rsgn = (float)a.range;
    double acc = 0.0;
    unsigned long long cnt = 0;
    // items: (row, 32- or 64-column piece of it); every slot takes every
    // slots-th item, four at a time so that four loads are in flight
    const int pieces = (wx + step_x - 1) / step_x;
    const int items = nrows * pieces;
    constexpr int UN = 4;
    for (int i0 = wave * (two ? 2 : 1) + slot; i0 < items; i0 += UN * slots) {
        float v[UN];
        bool sel[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const int it = i0 + u * slots;
            const int r = it / pieces, xx = (it - r * pieces) * step_x + sl;
            v[u] = 0.f;
            if (it < items && xx < wx) {
                const int64_t yy = y0 + r % wy, zz = z0 + r / wy;
                v[u] = a.x[(zz * a.ny + yy) * a.nx + x0 + xx];
                sel[u] = isfinite(v[u]) && (all_range || v[u] * rsgn > 0.f);
            } else {
                sel[u] = false;
            }
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            if (MAD) {
                // append the keys of this wave's selected voxels
                const unsigned long long bal = __ballot(sel[u]);
                const int nsel = __popcll(bal);
                uint32_t base = 0;
                const int leader = __ffsll((long long)(bal | 1ull)) - 1;
                if (nsel && lane == leader) base = atomicAdd(&res[0], (uint32_t)nsel);
                base = __shfl(base, leader);
                if (sel[u]) {
                    const int below = (int)__builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                    const uint32_t key = __float_as_uint(fabsf(v[u]));
                    keys[base + below] = key;
                    atomicAdd(&hist[key >> 20], 1u);
                }
            } else if (sel[u]) {
                acc += (double)v[u] * (double)v[u];
                cnt += 1;
            }
        }
    }

    double sigma;
    if (!MAD) {
        // fixed-order reduction: waves, then the wave totals
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            acc += __shfl_down(acc, off);
            cnt += __shfl_down(cnt, off);
        }
        if (lane == 0) { psum[wave] = acc; pcnt[wave] = cnt; }
        __syncthreads();
        if (tid != 0) return;
        double s = 0.0;
        unsigned long long m = 0;
        for (int w = 0; w < nwaves; ++w) { s += psum[w]; m += pcnt[w]; }
        sigma = m ? sqrt(s / (double)m) : (double)NAN;
        a.sigma[b] = sigma;
        return;
    }

    __syncthreads();
    const uint32_t m = res[0];
    if (m == 0) {
        if (tid == 0) a.sigma[b] = NAN;
        return;
    }
    const uint32_t r_lo = (m - 1) / 2, r_hi = m / 2;
    // level 1: bits 30..20
    find_rank(hist, 2048, r_lo, scan, res + 1);
    const uint32_t b1 = res[1], below1 = res[2];
    // level 2: bits 19..10 of the keys in bin b1
    for (int i = tid; i < 1024; i += blockDim.x) hist[i] = 0u;
    __syncthreads();
    for (uint32_t i = tid; i < m; i += blockDim.x) {
        const uint32_t k = keys[i];
        if ((k >> 20) == b1) atomicAdd(&hist[(k >> 10) & 1023u], 1u);
    }
    __syncthreads();
    find_rank(hist, 1024, r_lo - below1, scan, res + 1);
    const uint32_t b2 = res[1], below2 = res[2];
    // level 3: bits 9..0 of the keys with the prefix (b1, b2)
    for (int i = tid; i < 1024; i += blockDim.x) hist[i] = 0u;
    __syncthreads();
    const uint32_t pre = (b1 << 10) | b2;
    for (uint32_t i = tid; i < m; i += blockDim.x) {
        const uint32_t k = keys[i];
        if ((k >> 10) == pre) atomicAdd(&hist[k & 1023u], 1u);
    }
    __syncthreads();
    find_rank(hist, 1024, r_lo - below1 - below2, scan, res + 1);
    const uint32_t b3 = res[1], below3 = res[2];
    const uint32_t k_lo = (pre << 10) | b3;
    // keys at or below k_lo
    const uint32_t le = below1 + below2 + below3 + hist[b3];
    uint32_t k_hi = k_lo;
    if (r_hi >= le) {
        // the next larger key: a min-reduction over the keys above k_lo
        if (tid == 0) res[4] = 0xffffffffu;
        __syncthreads();
        uint32_t mn = 0xffffffffu;
        for (uint32_t i = tid; i < m; i += blockDim.x) {
            const uint32_t k = keys[i];
            if (k > k_lo && k < mn) mn = k;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const uint32_t t = __shfl_down(mn, off);
            mn = t < mn ? t : mn;
        }
        if (lane == 0) atomicMin(&res[4], mn);
        __syncthreads();
        k_hi = res[4];
    }
    if (tid == 0) {
        const double v_lo = (double)__uint_as_float(k_lo), v_hi = (double)__uint_as_float(k_hi);
        const double med = (r_lo == r_hi) ? v_lo : 0.5 * (v_lo + v_hi);
        a.sigma[b] = 1.4826 * med;
    }
}

// One block of 256 threads per (row, chunk of 1024 columns).
__global__ __launch_bounds__(256) void k_norm_divide(NormArgs a, int64_t chunks, int64_t items) {
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int64_t row = it / chunks, ch = it - row * chunks;
        const int64_t yy = row % a.ny, zz = row / a.ny;
        const double *srow =
            a.sigma + ((zz / a.gz) * a.nby + yy / a.gxy) * (int64_t)a.nbx;
        const int64_t base = row * a.nx;
        const uint32_t g = (uint32_t)a.gxy;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t xx = ch * 1024 + k * 256 + threadIdx.x;
            if (xx < a.nx) {
                const float v = a.x[base + xx];
                const double s = srow[(uint32_t)xx / g];   // nx < 2^32 (plane limit)
                const bool ok = isfinite(v) && isfinite(s) && s > 0.0;
                a.y[base + xx] = ok ? (float)((double)v / s) : NAN;
            }
        }
    }
}

hipError_t launch_window_noise(int mode, const NormArgs &a, hipStream_t s) {
    const int64_t nb = (int64_t)a.nbx * a.nby * a.nbz;
    if (nb < 1 || nb > 0x7fffffffLL) return hipErrorInvalidValue;
    if (mode == SOFIA_SC_NOISE_MAD) {
        const int64_t vol = (int64_t)a.wxy * a.wxy * a.wz;
        if (vol > kNormMaxWindow) return hipErrorInvalidValue;
        const size_t lds = (size_t)(vol + 2048) * sizeof(uint32_t);
        hipLaunchKernelGGL(k_window_noise<true>, dim3((unsigned)nb), dim3(kNormThreads), lds, s,
                           a);
    } else {
        hipLaunchKernelGGL(k_window_noise<false>, dim3((unsigned)nb), dim3(kNormThreads), 0, s,
                           a);
    }
    return hipGetLastError();
}

hipError_t launch_norm_divide(const NormArgs &a, hipStream_t s) {
    const int64_t chunks = (a.nx + 1023) / 1024;
    const int64_t items = chunks * a.ny * a.nz;
    const int64_t grid = items < 262144 ? items : 262144;
    hipLaunchKernelGGL(k_norm_divide, dim3((unsigned)grid), dim3(256), 0, s, a, chunks, items);
    return hipGetLastError();
}

}  // namespace sc
