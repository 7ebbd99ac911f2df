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
    __shared__ uint32_t hist[MAD ? 2048 : 1];
    __shared__ uint32_t stage[MAD ? kNormStage : 1];
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
    const bool all_range = a.range == 0;
    const float rsgn = (float)a.range;

    // Stream the window: row slot q (0 .. slots-1) takes the rows q,
    // q + slots, ..., UN of them at a time so that UN loads are in flight,
    // each row in pieces of step_x columns; a row's (y, z) offset inside the
    // window advances incrementally (no division per item). visit(v, sel) is
    // called for every item, selected (finite, in the flux range) or not.
    const int pieces = (wx + step_x - 1) / step_x;
    const int q = wave * (two ? 2 : 1) + slot;
    const int dz_step = slots / wy, dy_step = slots - dz_step * wy;
    auto stream = [&](auto &&visit) {
        constexpr int UN = 4;
        int cy = q % wy, cz = q / wy;
        for (int r0 = q; r0 < nrows; r0 += UN * slots) {
            int64_t rowoff[UN];
            bool rin[UN];
#pragma unroll
            for (int u = 0; u < UN; ++u) {
                rin[u] = r0 + u * slots < nrows;
                rowoff[u] = ((z0 + cz) * a.ny + y0 + cy) * a.nx + x0;
                cy += dy_step;
                cz += dz_step;
                if (cy >= wy) { cy -= wy; ++cz; }
            }
            for (int p = 0; p < pieces; ++p) {
                const int xx = p * step_x + sl;
                const bool xin = xx < wx;
                float v[UN];
                bool sel[UN];
#pragma unroll
                for (int u = 0; u < UN; ++u) {
                    v[u] = 0.f;
                    sel[u] = false;
                    if (rin[u] && xin) {
                        v[u] = a.x[rowoff[u] + xx];
                        sel[u] = isfinite(v[u]) && (all_range || v[u] * rsgn > 0.f);
                    }
                }
#pragma unroll
                for (int u = 0; u < UN; ++u) visit(v[u], sel[u]);
            }
        }
    };

    if (!MAD) {
        double acc = 0.0;
        unsigned long long cnt = 0;
        stream([&](float v, bool sel) {
            if (sel) {
                acc += (double)v * (double)v;
                cnt += 1;
            }
        });
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
        a.sigma[b] = m ? sqrt(s / (double)m) : (double)NAN;
        return;
    }

    // MAD. Keys are the bit patterns of |v| (they order like the values).
    // Pass 1: level-1 histogram of bits 30..20 and the number of keys m.
    for (int i = tid; i < 2048; i += blockDim.x) hist[i] = 0u;
    if (tid == 0) { res[0] = 0u; res[5] = 0u; res[6] = 0xffffffffu; }
    __syncthreads();
    uint32_t mine = 0;
    stream([&](float v, bool sel) {
        if (sel) {
            atomicAdd(&hist[__float_as_uint(fabsf(v)) >> 20], 1u);
            ++mine;
        }
    });
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mine += __shfl_down(mine, off);
    if (lane == 0) atomicAdd(&res[0], mine);
    __syncthreads();
    const uint32_t m = res[0];
    if (m == 0) {
        if (tid == 0) a.sigma[b] = NAN;
        return;
    }
    const uint32_t r_lo = (m - 1) / 2, r_hi = m / 2;
    find_rank(hist, 2048, r_lo, scan, res + 1);
    const uint32_t b1 = res[1], below1 = res[2];
    const uint32_t in_b1 = hist[b1];
    // the upper order statistic lies in a higher bin when the lower one is
    // the last key of bin b1: it is then the smallest key above bin b1
    const bool hi_above = r_hi >= below1 + in_b1;
    const bool staged = in_b1 <= (uint32_t)kNormStage;
    __syncthreads();

    // Pass 2: the keys of bin b1 into LDS (when they fit), and the smallest
    // key above bin b1.
    uint32_t above = 0xffffffffu;
    stream([&](float v, bool sel) {
        const uint32_t key = __float_as_uint(fabsf(v));
        const bool in = sel && (key >> 20) == b1;
        if (hi_above && sel && (key >> 20) > b1 && key < above) above = key;
        if (staged) {
            const unsigned long long bal = __ballot(in);
            const int nsel = __popcll(bal);
            uint32_t base = 0;
            const int leader = __ffsll((long long)(bal | 1ull)) - 1;
            if (nsel && lane == leader) base = atomicAdd(&res[5], (uint32_t)nsel);
            base = __shfl(base, leader);
            if (in) {
                const int below = (int)__builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                stage[base + below] = key;
            }
        }
    });
    if (hi_above) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const uint32_t t = __shfl_down(above, off);
            above = t < above ? t : above;
        }
        if (lane == 0) atomicMin(&res[6], above);
    }
    __syncthreads();
    const uint32_t k_above = res[6];

    // the keys of bin b1, from LDS or (when they did not fit) from HBM again
    auto for_bin_keys = [&](auto &&f) {
        if (staged) {
            for (uint32_t i = tid; i < in_b1; i += blockDim.x) f(stage[i]);
        } else {
            stream([&](float v, bool sel) {
                const uint32_t key = __float_as_uint(fabsf(v));
                if (sel && (key >> 20) == b1) f(key);
            });
        }
    };
    // level 2: bits 19..10 of the keys in bin b1
    for (int i = tid; i < 1024; i += blockDim.x) hist[i] = 0u;
    __syncthreads();
    for_bin_keys([&](uint32_t k) { atomicAdd(&hist[(k >> 10) & 1023u], 1u); });
    __syncthreads();
    find_rank(hist, 1024, r_lo - below1, scan, res + 1);
    const uint32_t b2 = res[1], below2 = res[2];
    // level 3: bits 9..0 of the keys with the prefix (b1, b2)
    for (int i = tid; i < 1024; i += blockDim.x) hist[i] = 0u;
    __syncthreads();
    const uint32_t pre = (b1 << 10) | b2;
    for_bin_keys([&](uint32_t k) {
        if ((k >> 10) == pre) atomicAdd(&hist[k & 1023u], 1u);
    });
    __syncthreads();
    find_rank(hist, 1024, r_lo - below1 - below2, scan, res + 1);
    const uint32_t b3 = res[1], below3 = res[2];
    const uint32_t k_lo = (pre << 10) | b3;
    // keys at or below k_lo
    const uint32_t le = below1 + below2 + below3 + hist[b3];
    uint32_t k_hi = k_lo;
    if (hi_above) {
        k_hi = k_above;
    } else if (r_hi >= le) {
        // the next larger key inside bin b1: a min-reduction
        if (tid == 0) res[4] = 0xffffffffu;
        __syncthreads();
        uint32_t mn = 0xffffffffu;
        for_bin_keys([&](uint32_t k) {
            if (k > k_lo && k < mn) mn = k;
        });
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
    if (mode == SOFIA_SC_NOISE_MAD)
        hipLaunchKernelGGL(k_window_noise<true>, dim3((unsigned)nb), dim3(kNormThreads), 0, s, a);
    else
        hipLaunchKernelGGL(k_window_noise<false>, dim3((unsigned)nb), dim3(kNormThreads), 0, s, a);
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
