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
//  * k_strip (sc_spatial.h): one wave per strip of 64 columns of one
//    z-plane streams a chunk of rows; x passes across the lanes (DPP wave
//    shifts), y passes as running sums down the rows. Output: the spatially
//    smoothed cube (float32) in a work buffer.
//  * k_column: one thread per (x, y) column streams z with a ring of the
//    last w inputs in LDS and an FP64 running sum (exact for FP32 inputs),
//    and performs one per-voxel operation: accumulate sum s^2 (std noise),
//    count level-1 or level-2 histogram digits of |s| (exact MAD), or clip
//    into the mask. Lanes cover consecutive x, so every plane access of a
//    wave is one contiguous run.
//  * tiny one-block kernels turn the partial sums / histograms into sigma_k
//    on the device, so a run never waits on the host between launches.
#include <math.h>

#include <cmath>

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

// One wave per (plane, word): lane l tests column 64w + l of the plane. A
// blank bit marks a non-finite voxel; with a caller's mask a detection bit
// marks each nonzero byte of a finite voxel (the loaders replace every
// detected voxel; a caller's marks on blanked voxels reach the output mask
// through k_write_mask's source mask instead).
__global__ void k_init_bits(const float *__restrict__ x, const uint8_t *__restrict__ mask_in,
                            uint64_t *__restrict__ blank, uint64_t *__restrict__ det,
                            int64_t ncol, int64_t nz, int64_t wpp) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = nz * wpp;
    const int64_t wstride = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < nw;
         w += wstride) {
        const int64_t z = w / wpp, col = (w - z * wpp) * 64 + lane;
        const bool in = col < ncol;
        const int64_t i = z * ncol + col;
        const uint64_t bb = __ballot(in && !isfinite(x[in ? i : 0]));
        if (lane == 0) blank[w] = bb;
        if (mask_in) {
            const uint64_t db =
                __ballot(in && mask_in[in ? i : 0] != 0 && isfinite(x[in ? i : 0]));
            if (lane == 0) det[w] = db;
        }
    }
}

// Thread t writes bytes 16t .. 16t+15 of the caller's mask (16-byte stores
// whenever the mask itself is 16-byte aligned, whatever the plane size):
// their 16 bits come from one or two words of the plane's detection bits;
// only the few runs that cross a plane boundary (or the cube's end) go
// byte by byte. mask = bit (keep = 0), mask |= bit (keep = 1), or, with a
// source mask src, mask = bit | (src != 0).
__global__ __launch_bounds__(256) void k_write_mask(const uint64_t *__restrict__ det,
                                                    uint8_t *__restrict__ mask, int keep,
                                                    const uint8_t *__restrict__ src,
                                                    int64_t ncol, int64_t nz, int64_t wpp) {
    const int64_t n = nz * ncol;
    const int64_t nt = (n + 15) / 16;
    const bool aligned = ((uintptr_t)mask & 15) == 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += stride) {
        const int64_t i0 = 16 * t;
        int64_t z = i0 / ncol, c = i0 - z * ncol;
        uint8_t *m = mask + i0;
        const uint8_t *sm = src ? src + i0 : nullptr;
        if (aligned && c + 16 <= ncol) {
            const uint64_t *dz = det + z * wpp;
            const int64_t w = c >> 6;
            const uint32_t sh = (uint32_t)(c & 63);
            uint64_t b = dz[w] >> sh;
            if (sh > 48) b |= dz[w + 1] << (64 - sh);
            const uint32_t bits = (uint32_t)b & 0xffffu;
            // nibble -> four 0/1 bytes
            auto expand = [](uint32_t q) {
                return (q & 1u) | ((q & 2u) << 7) | ((q & 4u) << 14) | ((q & 8u) << 21);
            };
            uint4 v = make_uint4(expand(bits & 15u), expand((bits >> 4) & 15u),
                                 expand((bits >> 8) & 15u), expand((bits >> 12) & 15u));
            if (keep) {
                const uint4 o = *reinterpret_cast<const uint4 *>(m);
                v.x |= o.x; v.y |= o.y; v.z |= o.z; v.w |= o.w;
            }
            if (sm) {
                for (int e = 0; e < 16; ++e)
                    if (sm[e]) reinterpret_cast<uint8_t *>(&v)[e] = 1;
            }
            *reinterpret_cast<uint4 *>(m) = v;
        } else {
            const int ne = (int)(n - i0 < 16 ? n - i0 : 16);
            for (int e = 0; e < ne; ++e) {
                uint8_t b = (uint8_t)((det[z * wpp + (c >> 6)] >> (c & 63)) & 1u);
                if (sm && sm[e]) b = 1;
                m[e] = keep ? (uint8_t)(m[e] | b) : b;
                if (++c == ncol) { c = 0; ++z; }
            }
        }
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
        st->clip_fallback = 0ull;
        st->fused_ok = 0;
        st->thr_lo = 0.0;
        st->thr_hi = 0.0;
        st->scale = 1.0;
        for (int k = 0; k < SOFIA_SC_MAX_KERNELS; ++k) st->sigma[k] = NAN;
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
// amb_count may be null: no fused clip in this pass (then fused_ok = 0 and
// the plain clip pass runs).
__global__ __launch_bounds__(256) void k_finalize_select(
    DevState *st, const unsigned long long *sel_part, int nparts,
    const unsigned long long *cap_count, unsigned long long cap_capacity, int k,
    const unsigned long long *amb_count, unsigned long long amb_capacity) {
    // sum the selection pass's per-block counts (fixed order)
    __shared__ unsigned long long rs[2][256];
    const int tid = threadIdx.x;
    unsigned long long c0 = 0, c1 = 0;
    for (int b = tid; b < nparts; b += 256) {
        c0 += sel_part[2 * b];
        c1 += sel_part[2 * b + 1];
    }
    rs[0][tid] = c0;
    rs[1][tid] = c1;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) {
            rs[0][tid] += rs[0][tid + off];
            rs[1][tid] += rs[1][tid + off];
        }
        __syncthreads();
    }
    if (tid != 0) return;
    const unsigned long long m = rs[0][0], below = rs[1][0], cin = *cap_count;
    const unsigned long long bit = 1ull << (k >= 0 ? k : 63);
    st->m = m;
    st->below = 0ull;
    st->fused_ok = 0;
    if (m == 0) {                 // no voxel in the flux range
        st->status |= 1;
        st->use_capture = 1;      // nothing to select: skip every later pass
        st->clip_fallback |= bit; // (the mask is undefined then)
        return;
    }
    const unsigned long long r_lo = (m - 1) / 2, r_hi = m / 2;
    const bool ok = cin <= cap_capacity && below <= r_lo && r_hi < below + cin;
    st->use_capture = ok ? 1 : 0;
    if (ok) st->below = below;
    else st->fallback |= bit;
    // The median lies in the captured window, so the threshold lies in
    // (thr_lo, thr_hi]: every voxel outside it was clipped exactly.
    const bool fused = ok && amb_count && *amb_count <= amb_capacity;
    st->fused_ok = fused ? 1 : 0;
    if (!fused) st->clip_fallback |= bit;
}

// Voxels with thr_lo < |s| <= thr_hi, decided with the exact threshold.
__global__ void k_clip_fixup(const DevState *st, const AmbEntry *amb,
                             const unsigned long long *amb_count,
                             unsigned long long amb_capacity, uint64_t *det_out, int64_t ncol,
                             int64_t wpp) {
    if (!st->fused_ok) return;
    const unsigned long long n = *amb_count < amb_capacity ? *amb_count : amb_capacity;
    const double T = st->thr;
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
         i < n; i += stride) {
        const AmbEntry e = amb[i];
        if (!(fabs(e.s) > T)) continue;
        const int64_t z = (int64_t)(e.idx / (uint64_t)ncol);
        const int64_t col = (int64_t)e.idx - z * ncol;
        atomicOr((unsigned long long *)&det_out[z * wpp + (col >> 6)], 1ull << (col & 63));
    }
}

// Predict the median of |s| from the level-1 histogram of a sample of
// columns (linear interpolation inside the bin that holds each central rank)
// and set the capture window to that estimate -/+ delta, with
// delta = 2 % + 3 / sqrt(sample size).
__global__ __launch_bounds__(256) void k_finalize_predict(
    DevState *st, const unsigned long long *hist_s, double t) {
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
        // If the two central order statistics v0 <= v1 fall in the window,
        // t * 1.4826 * (v0 + v1) / 2 lies between these bounds (widened far
        // beyond the three roundings of that product).
        st->thr_lo = t * (kMadFactor * (double)__uint_as_float(st->klo)) * (1.0 - 1e-12);
        st->thr_hi = t * (kMadFactor * (double)__uint_as_float(st->khi)) * (1.0 + 1e-12);
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

hipError_t launch_init_bits(const float *x, const uint8_t *mask_in, uint64_t *blank,
                            uint64_t *det, int64_t ncol, int64_t nz, int64_t wpp,
                            hipStream_t s) {
    const int64_t waves = nz * wpp;
    const int blocks = (int)(waves / 4 + 1 < 65536 ? waves / 4 + 1 : 65536);
    hipLaunchKernelGGL(k_init_bits, dim3(blocks), dim3(256), 0, s, x, mask_in, blank, det,
                       ncol, nz, wpp);
    return hipGetLastError();
}

hipError_t launch_write_mask(const uint64_t *det, uint8_t *mask, int keep, const uint8_t *src,
                             int64_t ncol, int64_t nz, int64_t wpp, hipStream_t s) {
    const int64_t n = (nz * ncol + 15) / 16;
    hipLaunchKernelGGL(k_write_mask, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, det, mask,
                       keep, src, ncol, nz, wpp);
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

hipError_t launch_spatial(int n_iter, int radius, int xtype, bool repl,
                          const StripArgs &a, hipStream_t s) {
#define SC_SP(N, R) \
    if (n_iter == N && radius == R) return launch_strip<R, N>(a, xtype, repl, s);
    SC_SP(3, 1) SC_SP(3, 2) SC_SP(3, 3) SC_SP(3, 4) SC_SP(3, 5)
    SC_SP(4, 1) SC_SP(4, 2) SC_SP(4, 3) SC_SP(4, 4)
    SC_SP(5, 1) SC_SP(5, 2) SC_SP(5, 3)
    SC_SP(6, 1) SC_SP(6, 2)
#undef SC_SP
    return hipErrorInvalidValue;
}

int gauss_radius(double fwhm) {
    const double sigma = fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    return (int)std::floor(4.0 * sigma + 0.5);
}

void gauss_setup(GaussArgs &a, double fwhm, int rows_max) {
    const double sigma = fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    const int R = gauss_radius(fwhm);
    double h[kGaussMaxR + 1] = {};
    double sum = 0.0;
    for (int k = 0; k <= R && k <= kGaussMaxR; ++k) {
        h[k] = std::exp(-(double)k * (double)k / (2.0 * sigma * sigma));
        sum += k == 0 ? h[k] : 2.0 * h[k];
    }
    for (int k = 0; k <= kGaussMaxR; ++k) {
        a.td[k] = k <= R ? h[k] / sum : 0.0;
        a.tf[k] = (float)a.td[k];
    }
    a.nstrips = (int32_t)((a.nx + kGaussCols - 1) / kGaussCols);
    int64_t rows = rows_max;
    while (rows > 32 && (int64_t)a.nstrips * ((a.ny + rows - 1) / rows) * a.nz < 16384) rows /= 2;
    if (rows > a.ny) rows = a.ny;
    a.rows = (int32_t)rows;
    a.nchunks = (int32_t)((a.ny + rows - 1) / rows);
    a.tiles = (int64_t)a.nstrips * a.nchunks * a.nz;
}

hipError_t launch_gauss(int radius, int xtype, bool repl, const GaussArgs &a, hipStream_t s) {
    switch (radius) {
#define SC_G(R) case R: return launch_gauss_r<R>(a, xtype, repl, s);
        SC_G(1) SC_G(2) SC_G(3) SC_G(4) SC_G(5) SC_G(6) SC_G(7) SC_G(8)
        SC_G(9) SC_G(10) SC_G(11) SC_G(12) SC_G(13) SC_G(14) SC_G(15) SC_G(16)
        SC_G(17) SC_G(18) SC_G(19) SC_G(20) SC_G(21) SC_G(22) SC_G(23) SC_G(24)
#undef SC_G
    }
    return hipErrorInvalidValue;
}

template <int OP>
hipError_t launch_column_op(int src, bool spec, const ColArgs &a, int nb, hipStream_t s);

hipError_t launch_column(int src, int op, bool spectral, const ColArgs &a, int nblocks,
                         hipStream_t s) {
    switch (op) {
        case OP_STD: return launch_column_op<OP_STD>(src, spectral, a, nblocks, s);
        case OP_HIST1: return launch_column_op<OP_HIST1>(src, spectral, a, nblocks, s);
        case OP_HIST2: return launch_column_op<OP_HIST2>(src, spectral, a, nblocks, s);
        case OP_CLIP: return launch_column_op<OP_CLIP>(src, spectral, a, nblocks, s);
        case OP_WRITE: return launch_column_op<OP_WRITE>(src, spectral, a, nblocks, s);
        case OP_SELECT: return launch_column_op<OP_SELECT>(src, spectral, a, nblocks, s);
        case OP_SELCLIP: return launch_column_op<OP_SELCLIP>(src, spectral, a, nblocks, s);
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

hipError_t launch_finalize_select(DevState *st, const unsigned long long *sel_part, int nparts,
                                  const unsigned long long *cap_count,
                                  unsigned long long cap_capacity, int k,
                                  const unsigned long long *amb_count,
                                  unsigned long long amb_capacity, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_select, dim3(1), dim3(256), 0, s, st, sel_part, nparts,
                       cap_count, cap_capacity, k, amb_count, amb_capacity);
    return hipGetLastError();
}

hipError_t launch_clip_fixup(const DevState *st, const AmbEntry *amb,
                             const unsigned long long *amb_count,
                             unsigned long long amb_capacity, uint64_t *det_out, int64_t ncol,
                             int64_t wpp, hipStream_t s) {
    hipLaunchKernelGGL(k_clip_fixup, dim3(512), dim3(256), 0, s, st, amb, amb_count,
                       amb_capacity, det_out, ncol, wpp);
    return hipGetLastError();
}

hipError_t launch_capture_l1(const DevState *st, const uint32_t *cap_buf,
                             const unsigned long long *cap_count,
                             unsigned long long *hist1, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_capture_l1, dim3(blocks), dim3(256), 0, s, st, cap_buf, cap_count,
                       hist1);
    return hipGetLastError();
}

hipError_t launch_finalize_predict(DevState *st, const unsigned long long *hist_s,
                                   double t, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_predict, dim3(1), dim3(256), 0, s, st, hist_s, t);
    return hipGetLastError();
}

hipError_t launch_capture_coarse(const DevState *st, const uint32_t *cap_buf,
                                 const unsigned long long *cap_count,
                                 unsigned long long *hist2c, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_capture_coarse, dim3(blocks), dim3(256), 0, s, st, cap_buf,
                       cap_count, hist2c);
    return hipGetLastError();
}

hipError_t launch_capture_fine(const DevState *st, const uint32_t *cap_buf,
                               const unsigned long long *cap_count,
                               unsigned long long *hist2, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_capture_fine, dim3(blocks), dim3(256), 0, s, st, cap_buf,
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
