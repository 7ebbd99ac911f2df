// Replacement off: the kernel pairs of a run no longer depend on each other
// (replacement of earlier detections, Sect. 6.2.4, is what chains them), so
// the pairs that share a spatial kernel can share their passes. For one
// spatial kernel (or none) and up to kMultiMax spectral widths:
//  * k_multi<SRC, STATS>: one stream over the columns computes every width's
//    smoothed value per voxel from one LDS ring of the last 2 hmax + 2 input
//    planes (hmax = the largest half-width) and accumulates each width's sum
//    of s^2 and count over the selected voxels (RMS noise about zero);
//  * k_multi_finalize: sigma of every width from the per-block partials in a
//    fixed order;
//  * k_multi<SRC, CLIP>: the same stream, every voxel detected when any
//    width's |s| exceeds t sigma of that width, ORed into the run's packed
//    detection bits (one word per wave and plane, read and written by the
//    same wave, so the bits may be updated in place).
// Every width's running sum is an FP64 sum of the same float inputs as the
// per-pair column pass, re-anchored from the ring every 32 planes; the
// windows of all widths are centred on the same output plane.
#include <math.h>

#include "sc_device.h"

namespace sc {

template <int SRC, int MOP, int NW>
__global__ __launch_bounds__(kColThreads) void k_multi(MultiArgs a) {
    extern __shared__ float mring[];
    constexpr int B = kColThreads;
    const int tid = threadIdx.x;
    // XCD-aware tile order, as in the column kernel
    const int tile = (int)xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x);
    const int cb = tile % a.ncb;
    const int zc = tile / a.ncb;
    const int64_t ncol = a.ncol;
    const int64_t col0 = (int64_t)cb * B;
    const bool active = col0 + tid < ncol;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int64_t wcol = (col0 >> 6) + wave;      // the wave's word of each bit plane
    const bool live = col0 + 64 * wave < ncol;    // the wave has a column in the plane
    const int nz = (int)a.nz;
    const int z0 = zc * a.zchunk;
    const int z1 = min(nz, z0 + a.zchunk);
    constexpr int nw = NW;
    const int hm = a.hmax, RW = 2 * a.hmax + 2;
    const bool all_range = a.range == 0;
    const double rsgn = (double)a.range;

    double S[NW], inv_w[NW], T[NW], acc[NW];
    unsigned cnt[NW];
    int hw[NW];
    // MOP_SELECT: key windows, counts, and per-wave staging of captured keys
    uint32_t klo[NW], khi[NW];
    unsigned nbelow[NW];
    int fill[NW];
    uint32_t *stagew = reinterpret_cast<uint32_t *>(mring + (size_t)RW * B) +
                       (size_t)(tid >> 6) * NW * kMultiStage;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        S[i] = 0.0;
        acc[i] = 0.0;
        cnt[i] = 0u;
        hw[i] = a.h[i];
        inv_w[i] = 1.0 / (double)a.w[i];
        T[i] = MOP == MOP_CLIP ? a.t * a.st->sigma[a.k[i]] : 0.0;
        klo[i] = MOP == MOP_SELECT ? a.sti[i]->klo : 1u;
        khi[i] = MOP == MOP_SELECT ? a.sti[i]->khi : 0u;
        nbelow[i] = 0u;
        fill[i] = 0;
    }
    const int wlane = tid & 63;
    // this wave's staged keys of width i go to the width's capture list (one
    // atomic per flush; entries past the capacity are dropped, the count
    // still grows and sends the width to the full histogram passes)
    auto flush = [&](int i) {
        __builtin_amdgcn_wave_barrier();
        unsigned long long base = 0;
        if (wlane == 0) base = atomicAdd(a.cap_count[i], (unsigned long long)fill[i]);
        const uint32_t lo32 = __shfl((uint32_t)base, 0);
        const uint32_t hi32 = __shfl((uint32_t)(base >> 32), 0);
        base = ((unsigned long long)hi32 << 32) | lo32;
        const uint32_t *sw = stagew + (size_t)i * kMultiStage;
        for (int e = wlane; e < fill[i]; e += 64)
            if (base + e < a.cap_capacity) a.cap[i][base + e] = sw[e];
        __builtin_amdgcn_wave_barrier();
        fill[i] = 0;
    };
    auto fin = [](float v) { return isfinite(v) ? v : 0.f; };
    // ring slot of the plane d planes before the newest one (0 <= d < RW)
    int si = RW - 1;     // slot of the newest plane
    auto back = [&](int d) -> float & {
        const int r = si - d;
        return mring[(r < 0 ? r + RW : r) * B + tid];
    };

    // planes z0 - hm .. z1 + hm - 1 stream through; outputs z0 .. z1 - 1
    const int zs = z0 - hm, ze = z1 + hm;
    constexpr int G = 8;
    float cur[G], nxt[G];
    // packed bits of the group's output planes: lane j holds the wave's word
    // of output plane j (blank bits for SRC_P; detection bits so far, CLIP)
    uint64_t bcur = 0, bnxt = 0, dcur = 0, dnxt = 0;
    // lanes past the plane's end load their block's first column (in bounds;
    // they count as blanked); a group inside the stream and the cube loads
    // its planes through one buffer descriptor with per-plane scalar offsets
    const uint32_t vo = (uint32_t)(active ? tid : 0) * 4u;
    const int zhi = min(ze, nz);
    const bool one_rsrc = (int64_t)(G - 1) * ncol * 4 + (int64_t)B * 4 < (1ll << 32);
    const uint32_t pbytes = (uint32_t)(ncol * 4);
    auto load_group = [&](int zb, float *v, uint64_t &bw, uint64_t &dw) {
        if (one_rsrc && zb >= 0 && zb + G <= zhi) {
            const __amdgpu_buffer_rsrc_t r = plane_rsrc(a.src + (int64_t)zb * ncol + col0);
#pragma unroll
            for (int j = 0; j < G; ++j) v[j] = buf_f32(r, vo, (uint32_t)j * pbytes);
        } else {
#pragma unroll
            for (int j = 0; j < G; ++j) {
                const int zi = zb + j;
                v[j] = 0.f;
                if (zi < ze && zi >= 0 && zi < nz)
                    v[j] = buf_f32(plane_rsrc(a.src + (int64_t)zi * ncol + col0), vo, 0u);
            }
        }
        bw = 0;
        dw = 0;
        const int zo = zb + lane - hm;
        if (lane < G && zb + lane < ze && zo >= z0) {
            const int64_t wi = (int64_t)zo * a.wpp + wcol;
            if (SRC == SRC_P) bw = a.blank[wi];
            if (MOP == MOP_CLIP && a.det_in) dw = a.det_in[wi];
        }
    };
    int steps = 0;
    if (live) load_group(zs, cur, bcur, dcur);
    for (int zb = zs; live && zb < ze; zb += G) {
        if (zb + G < ze) load_group(zb + G, nxt, bnxt, dnxt);
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int zi = zb + j;
            if (zi >= ze) break;
            si = si + 1 == RW ? 0 : si + 1;
            back(0) = cur[j];    // raw (SRC_X: NaN kept for the blank test)
            // output plane zo = zi - hm is back(hm); plane zo + e is back(hm - e)
            const int zo = zi - hm;
            if (zo < z0) continue;
            if (zo == z0 || (++steps & 31) == 0) {
                // (re-)anchor every width's window sum directly from the ring
#pragma unroll
                for (int i = 0; i < NW; ++i) {
                    double s = 0.0;
                    for (int d = hm - hw[i]; d <= hm + hw[i]; ++d) s += (double)fin(back(d));
                    S[i] = s;
                }
            } else {
#pragma unroll
                for (int i = 0; i < NW; ++i)
                    S[i] += (double)fin(back(hm - hw[i])) - (double)fin(back(hm + hw[i] + 1));
            }
            // columns past the plane's end take no part
            const bool blank = !active | (SRC == SRC_X ? !isfinite(back(hm))
                                                     : lane_bit(lane_word(bcur, j)));
            const bool zsel = a.zstride <= 1 || zo % a.zstride == 0;
            if (MOP == MOP_STATS) {
#pragma unroll
                for (int i = 0; i < NW; ++i) {
                    const double s = S[i] * inv_w[i];
                    const bool sel = !blank & zsel & (all_range | (s * rsgn > 0.0));
                    acc[i] += sel ? s * s : 0.0;
                    cnt[i] += sel ? 1u : 0u;
                }
            } else if (MOP == MOP_SELECT) {
#pragma unroll
                for (int i = 0; i < NW; ++i) {
                    const double s = S[i] * inv_w[i];
                    const bool sel = !blank & zsel & (all_range | (s * rsgn > 0.0));
                    const uint32_t key = __float_as_uint(fabsf((float)s));
                    cnt[i] += sel ? 1u : 0u;
                    nbelow[i] += (sel & (key < klo[i])) ? 1u : 0u;
                    const bool want = sel & (key >= klo[i]) & (key <= khi[i]);
                    const uint64_t bal = wave_mask(want);
                    if (bal) {
                        if (want) {
                            const int below = (int)__builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(bal >> 32),
                                __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                            stagew[(size_t)i * kMultiStage + fill[i] + below] = key;
                        }
                        fill[i] += __popcll(bal);
                        if (fill[i] > kMultiStage - 64) flush(i);
                    }
                }
            } else {
                bool det = false;
#pragma unroll
                for (int i = 0; i < NW; ++i)
                    det |= !blank & (fabs(S[i] * inv_w[i]) > T[i]);
                const uint64_t bits = wave_mask(det) | lane_word(dcur, j);
                if (lane == 0) a.det_out[(int64_t)zo * a.wpp + wcol] = bits;
            }
        }
#pragma unroll
        for (int j = 0; j < G; ++j) cur[j] = nxt[j];
        bcur = bnxt;
        dcur = dnxt;
    }

    if (MOP == MOP_SELECT) {
#pragma unroll
        for (int i = 0; i < NW; ++i)
            if (fill[i]) flush(i);
        // per-block counts of every width: selected voxels, keys below the window
        __shared__ unsigned long long rc2[2][B];
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            rc2[0][tid] = cnt[i];
            rc2[1][tid] = nbelow[i];
            __syncthreads();
            for (int off = B / 2; off > 0; off >>= 1) {
                if (tid < off) {
                    rc2[0][tid] += rc2[0][tid + off];
                    rc2[1][tid] += rc2[1][tid + off];
                }
                __syncthreads();
            }
            if (tid == 0) {
                a.sel_part[i][2 * tile] = rc2[0][0];
                a.sel_part[i][2 * tile + 1] = rc2[1][0];
            }
            __syncthreads();
        }
    }

    if (MOP == MOP_STATS) {
        // block reduction per width in a fixed order: deterministic partials
        __shared__ double rs[B];
        __shared__ unsigned long long rc[B];
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            rs[tid] = acc[i];
            rc[tid] = cnt[i];
            __syncthreads();
            for (int off = B / 2; off > 0; off >>= 1) {
                if (tid < off) { rs[tid] += rs[tid + off]; rc[tid] += rc[tid + off]; }
                __syncthreads();
            }
            if (tid == 0) {
                a.part_sum[(int64_t)i * a.nparts + tile] = rs[0];
                a.part_cnt[(int64_t)i * a.nparts + tile] = rc[0];
            }
            __syncthreads();
        }
    }
}

// sigma of every width: RMS about zero of its selected voxels; none selected
// -> NaN and the run's status flag.
__global__ __launch_bounds__(256) void k_multi_finalize(MultiArgs a) {
    __shared__ double ss[256];
    __shared__ unsigned long long sc[256];
    const int tid = threadIdx.x;
    for (int i = 0; i < a.nw; ++i) {
        double v = 0.0;
        unsigned long long c = 0;
        for (int p = tid; p < a.nparts; p += 256) {
            v += a.part_sum[(int64_t)i * a.nparts + p];
            c += a.part_cnt[(int64_t)i * a.nparts + p];
        }
        ss[tid] = v;
        sc[tid] = c;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (tid < off) { ss[tid] += ss[tid + off]; sc[tid] += sc[tid + off]; }
            __syncthreads();
        }
        if (tid == 0) {
            double sig = NAN;
            if (sc[0] > 0) sig = sqrt(ss[0] / (double)sc[0]);
            else a.st->status |= 1;
            a.st->sigma[a.k[i]] = sig;
        }
        __syncthreads();
    }
}

template <int SRC, int MOP>
hipError_t launch_multi_t(const MultiArgs &a, int nblocks, size_t lds, hipStream_t s) {
    const dim3 grid((unsigned)nblocks), block(kColThreads);
    switch (a.nw) {
#define SC_M(N) case N: hipLaunchKernelGGL((k_multi<SRC, MOP, N>), grid, block, lds, s, a); break;
        SC_M(1) SC_M(2) SC_M(3) SC_M(4) SC_M(5) SC_M(6) SC_M(7) SC_M(8)
#undef SC_M
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_multi(int src, int mop, const MultiArgs &a, int nblocks, hipStream_t s) {
    if ((src == SRC_P && !a.blank) || (mop == MOP_CLIP && !a.det_out)) return hipErrorInvalidValue;
    size_t lds = (size_t)(2 * a.hmax + 2) * kColThreads * sizeof(float);
    if (mop == MOP_SELECT)
        lds += (size_t)(kColThreads / 64) * a.nw * kMultiStage * sizeof(uint32_t);
    if (src == SRC_X) {
        if (mop == MOP_STATS) return launch_multi_t<SRC_X, MOP_STATS>(a, nblocks, lds, s);
        if (mop == MOP_SELECT) return launch_multi_t<SRC_X, MOP_SELECT>(a, nblocks, lds, s);
        return launch_multi_t<SRC_X, MOP_CLIP>(a, nblocks, lds, s);
    }
    if (mop == MOP_STATS) return launch_multi_t<SRC_P, MOP_STATS>(a, nblocks, lds, s);
    if (mop == MOP_SELECT) return launch_multi_t<SRC_P, MOP_SELECT>(a, nblocks, lds, s);
    return launch_multi_t<SRC_P, MOP_CLIP>(a, nblocks, lds, s);
}

__global__ void k_multi_gather(MultiArgs a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = 0; i < a.nw; ++i) {
        const DevState *si = a.sti[i];
        a.st->sigma[a.k[i]] = si->sigma[a.k[i]];
        a.st->status |= si->status;
        a.st->fallback |= si->fallback;
        a.st->clip_fallback |= si->clip_fallback;
    }
}

hipError_t launch_multi_gather(const MultiArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_multi_gather, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_multi_finalize(const MultiArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_multi_finalize, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace sc
