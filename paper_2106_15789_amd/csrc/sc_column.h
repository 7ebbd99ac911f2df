// Column-streaming kernel (spectral boxcar + one per-voxel operation),
// shared by the per-operation translation units sc_col_*.hip so that its many
// instantiations compile in parallel.
#pragma once

#include "sc_device.h"

namespace sc {

// ------------------------------------------------------ column streaming

struct ColAcc {
    double sum;
    unsigned long long cnt;
};

// One thread per (x, y) column. The column is streamed as a sequence of
// input planes zi = z0 - h .. z1 - 1 + h (the leading edge of the spectral
// window); after input zi the window sum S covers planes zi - 2h .. zi, i.e.
// the output plane z = zi - h. Inputs are fetched in groups of G planes and
// the next group is requested before the current one is consumed, so every
// wave keeps up to 2G plane reads in flight. Every plane access of a block is
// one contiguous run of 256 voxels: a uniform row pointer plus the lane.
//
// W is the spectral width: 1 = no spectral smoothing; an odd W >= 3 keeps the
// window in registers with compile-time ring slots (G is a multiple of W, so
// every group starts at slot 0); W = 0 takes the width at run time and keeps
// the window ring in LDS. The window sum is an FP64 running sum of the FP32
// inputs (exact while the inputs span fewer than 2^29 ulps), recomputed from
// the ring every eight groups.
template <int W>
struct ColGroup {
    static constexpr int G = W >= 3 ? W * ((8 + W - 1) / W) : 8;
};

template <int SRC, int OP, int W, int XT>
__global__ __launch_bounds__(kColThreads) void k_column(ColArgs a) {
    extern __shared__ float dyn_lds[];
    constexpr int B = kColThreads;
    constexpr bool SPEC = W != 1;
    constexpr bool LDSRING = W == 0;
    constexpr int G = ColGroup<W>::G;
    const int tid = threadIdx.x;
    if ((OP == OP_HIST1 || OP == OP_HIST2) && a.skip_if_captured && a.st->use_capture) return;
    if (OP == OP_CLIP && a.skip_if_fused && a.st->fused_ok) return;
    // Tile of this block, XCD-aware: neighbouring column blocks share the
    // cache lines of the bit planes, so they run on the same XCD (one L2).
    const int tile = (int)xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x);
    const int cb = tile % a.ncb;
    const int zc = tile / a.ncb;
    const int64_t ncol = a.ncol;
    // A sampling pass (cb_stride > 1) gives each wave its own 64-column
    // segment, every cb_stride-th of the plane, so that the sample spreads
    // evenly over x and y; the other passes take B adjacent columns per block.
    // Either way thread tid owns column col0 + tid.
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int64_t col0 =
        a.cb_stride > 1
            ? (((int64_t)cb * (B / 64) + wave) * a.cb_stride - wave) * 64
            : (int64_t)cb * B;
    const bool active = col0 + tid < ncol;
    // The wave's 64 columns start at a multiple of 64: they are word wcol of
    // every plane of the packed bits. A wave with no column in the plane
    // idles; in a partly filled wave the lanes past the plane's end run
    // along as blanked voxels and load nothing.
    const int64_t wcol = (col0 >> 6) + wave;
    const bool live = col0 + 64 * wave < ncol;
    const uint64_t live_m = wave_mask(active);   // the wave's columns inside the plane
    const int nz = (int)a.nz;
    const int z0 = zc * a.zchunk;
    const int z1 = min(nz, z0 + a.zchunk);
    const int w = W == 0 ? a.w : (W >= 3 ? W : 1);
    const int h = (w - 1) / 2;

    // LDS: [ring floats [w][B] | ring bytes [w][B] (W = 0 only)] | histogram | capture
    float *lring = dyn_lds;
    uint8_t *lbring = (uint8_t *)(dyn_lds + (LDSRING ? w * B : 0));
    unsigned *hist = (unsigned *)(lbring + ((LDSRING && SRC == SRC_X) ? ((w * B + 3) & ~3) : 0));
    constexpr int kHistWords = OP == OP_HIST1 ? kL1Bins : (OP == OP_HIST2 ? 2 * kL2Coarse : 0);
    if (kHistWords) {
        for (int i = tid; i < kHistWords; i += B) hist[i] = 0u;
    }
    if (LDSRING) {
        for (int j = 0; j < w; ++j) {
            lring[j * B + tid] = 0.f;
            if (SRC == SRC_X) lbring[j * B + tid] = 0;
        }
    }
    if (kHistWords) __syncthreads();

    const bool repl = SRC == SRC_X && a.det_in && a.repl_on;
    const float rv = repl ? (float)(a.repl_n * a.st->sigma0) : 0.f;
    constexpr bool SELCLIP = OP == OP_SELCLIP;
    const double T = (OP == OP_CLIP) ? a.st->thr : 0.0;
    const double Tlo = SELCLIP ? a.st->thr_lo : 0.0, Thi = SELCLIP ? a.st->thr_hi : 0.0;
    uint32_t b0 = 0xffffffffu, b1 = 0xffffffffu;
    if (OP == OP_HIST2) { b0 = a.st->bin[0]; b1 = a.st->bin[1]; }
    // Flux range as a lane mask: all voxels, or those with s * range > 0
    // (s < 0 for range -1, s > 0 for range +1).
    const uint64_t all_m = a.range == 0 ? ~0ull : 0ull;
    const double rsgn = (double)a.range;
    auto range_mask = [&](double s) { return all_m | wave_mask(s * rsgn > 0.0); };
    ColAcc acc{0.0, 0ull};   // sum: this lane's; cnt: the wave's (same in every lane)
    const float *src = SRC == SRC_X ? a.x : a.p;

    // Selection pass: count the selected voxels and the keys below the
    // predicted window [klo, khi], and append the keys inside it, per wave, to
    // an LDS buffer that is flushed to the global key list with one atomic
    // per flush.
    constexpr bool capture = OP == OP_SELECT || OP == OP_SELCLIP;
    uint32_t klo = 1, khi = 0;
    if (capture) { klo = a.st->klo; khi = a.st->khi; }
    // selected voxels and keys below the window: wave totals (same in every
    // lane), counted from lane masks
    unsigned n_sel = 0, n_below = 0;
    uint32_t *capw = (uint32_t *)(hist + kHistWords) + (tid >> 6) * kCapStride(G);
    int fill = 0;   // entries in this wave's buffer (same in every lane)
    auto flush = [&]() {
        __builtin_amdgcn_wave_barrier();
        const unsigned long long act = __ballot(1);
        const int leader = __ffsll((long long)act) - 1;
        const int wlane = tid & 63;
        unsigned long long base = 0;
        if (wlane == leader) base = atomicAdd(a.cap_count, (unsigned long long)fill);
        const uint32_t lo32 = __shfl((uint32_t)base, leader);
        const uint32_t hi32 = __shfl((uint32_t)(base >> 32), leader);
        base = ((unsigned long long)hi32 << 32) | lo32;
        // copy with the lanes that are active (a wave may be partly idle)
        const int rank = (int)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
        const int nact = __popcll(act);
        for (int i = rank; i < fill; i += nact)
            if (base + i < a.cap_capacity) a.cap_buf[base + i] = capw[i];
        __builtin_amdgcn_wave_barrier();
        fill = 0;
    };

    // Fused clip: undecided voxels are collected per wave in LDS and appended
    // to the global list in bulk, once per group of planes (one atomic per
    // flush: a single shared counter hit once per voxel-plane would serialise
    // the whole pass). Entries beyond the buffer are dropped and the count is
    // pushed past the list's capacity, which sends the pass to the full clip.
    const size_t amb_off =
        ((size_t)((const char *)(capw + (B / 64 - (tid >> 6)) * kCapStride(G)) -
                  (const char *)dyn_lds) + 15) & ~(size_t)15;
    AmbEntry *ambw = (AmbEntry *)((char *)dyn_lds + amb_off) + (tid >> 6) * kAmbPerWave;
    int afill = 0;   // entries in this wave's buffer (same in every lane)
    auto flush_amb = [&]() {
        __builtin_amdgcn_wave_barrier();
        const unsigned long long act = __ballot(1);
        const int leader = __ffsll((long long)act) - 1;
        const int kept = afill < kAmbPerWave ? afill : kAmbPerWave;
        const unsigned long long add =
            (unsigned long long)afill + (afill > kAmbPerWave ? a.amb_capacity + 1 : 0ull);
        unsigned long long base = 0;
        if ((tid & 63) == leader) base = atomicAdd(a.amb_count, add);
        const uint32_t lo32 = __shfl((uint32_t)base, leader);
        const uint32_t hi32 = __shfl((uint32_t)(base >> 32), leader);
        base = ((unsigned long long)hi32 << 32) | lo32;
        const int rank = (int)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
        const int nact = __popcll(act);
        for (int i = rank; i < kept; i += nact)
            if (base + i < a.amb_capacity) a.amb[base + i] = ambw[i];
        __builtin_amdgcn_wave_barrier();
        afill = 0;
    };

    // Clip output: the wave's words of the group's planes, lane j holding
    // plane j's (its earlier detections ORed with this kernel's; for a pass
    // over the raw cube also its blank bits), stored once per group.
    uint64_t oacc = 0, bacc = 0;
    auto put_word = [&](int j, uint64_t det_word, uint64_t blank_m) {
        oacc = with_lane_word(oacc, j, det_word);
        if (SRC == SRC_X) bacc = with_lane_word(bacc, j, blank_m & live_m);
    };

    // Per-voxel operation on the smoothed value s of plane j of the group
    // (output plane zo). Predicates are lane masks: blank_m marks blanked
    // voxels and lanes past the plane's end, dprev the plane's detections so
    // far; zsel: all ones if the plane is one the noise is measured on (every plane
    // unless the noise is subsampled; the clip takes every plane).
    auto consume = [&](int j, int zo, double s, uint64_t blank_m, uint64_t dprev, uint64_t zsel) {
        const uint64_t ok_m = ~blank_m;
        if (OP == OP_STD) {
            const uint64_t sel_m = zsel & ok_m & range_mask(s);
            acc.sum += lane_bit(sel_m) ? s * s : 0.0;
            acc.cnt += (unsigned long long)__popcll(sel_m);
        } else if (OP == OP_HIST1) {
            const uint64_t sel_m = zsel & ok_m & range_mask(s);
            if (lane_bit(sel_m)) {
                const uint32_t key = __float_as_uint(fabsf((float)s));
                atomicAdd(&hist[key >> kL1Shift], 1u);
            }
        } else if (OP == OP_SELECT || OP == OP_SELCLIP) {
            const uint64_t sel_m = zsel & ok_m & range_mask(s);
            const uint32_t key = __float_as_uint(fabsf((float)s));
            const uint64_t below_m = wave_mask(key < klo);
            n_sel += (unsigned)__popcll(sel_m);
            n_below += (unsigned)__popcll(sel_m & below_m);
            const uint64_t want_m = sel_m & ~below_m & wave_mask(key <= khi);
            // every lane writes: a capturing lane to its place in the list,
            // the others to a slot of their own past the list's end (the
            // rank is taken in every lane, so no lane mask is switched)
            int at = fill + lanes_below(want_m);
            __asm__ volatile("" : "+v"(at));
            capw[lane_bit(want_m) ? at : kCapPerWave(G) + lane] = key;
            fill += __popcll(want_m);
            if (SELCLIP) {
                // clip now unless |s| lies in (thr_lo, thr_hi], where the
                // decision waits for the exact threshold
                const double as = fabs(s);
                const uint64_t det_m = ok_m & wave_mask(as > Thi);
                const uint64_t amb_m = ok_m & wave_mask(as > Tlo) & ~det_m;
                put_word(j, det_m | dprev, blank_m);
                if (amb_m) {
                    if (lane_bit(amb_m)) {
                        const int at = afill + lanes_below(amb_m);
                        if (at < kAmbPerWave)
                            ambw[at] = AmbEntry{(uint64_t)((int64_t)zo * ncol + col0 + tid), s};
                    }
                    afill += __popcll(amb_m);
                }
            }
        } else if (OP == OP_HIST2) {
            const uint64_t sel_m = zsel & ok_m & range_mask(s);
            if (lane_bit(sel_m)) {
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
            put_word(j, (ok_m & wave_mask(fabs(s) > T)) | dprev, blank_m);
        } else {  // OP_WRITE
            if (active)
                buf_st_f32(lane_bit(blank_m) ? NAN : (float)s,
                           plane_rsrc(a.s_out + (int64_t)zo * ncol + col0), 4u * (uint32_t)tid, 0u);
        }
    };

    // Spectral input of a raw voxel: blanked -> 0, detected -> +-n sigma_0.
    auto raw_value = [&](float xv, bool det) -> float {
        if (!isfinite(xv)) return 0.f;
        if (repl & det) return copysignf(rv, xv);
        return xv;
    };

    // 16-bit storage is kept as raw bits until the group is consumed, so that
    // prefetching the next group never waits on its loads.
    constexpr bool Q16 = SRC == SRC_X && XT != ST_F32;
    struct Group {
        float v[G];
        uint16_t q[G];
        // Packed bits of the group's planes: lane j holds the wave's word of
        // plane j (the input plane for SRC_X, the output plane for SRC_P),
        // detection bits in dw and blank bits in bw (SRC_P), so that one load
        // per group fetches them and each plane's word is read back from its
        // lane.
        uint64_t dw, bw;
    };
    auto in_value = [&](const Group &g, int j) -> float {
        if (!Q16) return g.v[j];
        return XT == ST_F16 ? f16_bits_to_float(g.q[j]) : bf16_bits_to_float(g.q[j]);
    };
    const int zs = SPEC ? z0 - h : z0;
    const int ze = SPEC ? z1 + h : z1;   // exclusive
    // Lanes past the plane's end load their block's first column (in bounds;
    // they count as blanked).
    constexpr uint32_t XB = Q16 ? 2u : 4u;
    const uint32_t vo = (uint32_t)(active ? tid : 0) * XB;
    // A group whose planes are all inside the stream and the cube loads them
    // through one buffer descriptor with per-plane scalar offsets, when the
    // group's span fits the 32-bit offsets.
    const int zhi = min(ze, nz);
    const bool one_rsrc = (int64_t)(G - 1) * ncol * XB + (int64_t)B * XB < (1ll << 32);
    const uint32_t pbytes = (uint32_t)(ncol * XB);
    auto load_group = [&](int zb, Group &g) {
        const int64_t off0 = (int64_t)zb * ncol + col0;
        if (one_rsrc && zb >= 0 && zb + G <= zhi) {
            const __amdgpu_buffer_rsrc_t r =
                plane_rsrc(Q16 ? (const void *)(a.xq + off0) : (const void *)(src + off0));
#pragma unroll
            for (int j = 0; j < G; ++j) {
                if (Q16) g.q[j] = buf_u16(r, vo, (uint32_t)j * pbytes);
                else g.v[j] = buf_f32(r, vo, (uint32_t)j * pbytes);
            }
        } else {
            int64_t off = off0;   // running: plane zb + j
#pragma unroll
            for (int j = 0; j < G; ++j, off += ncol) {
                const int zi = zb + j;
                g.v[j] = 0.f;
                g.q[j] = 0;
                if (zi < ze && zi >= 0 && zi < nz) {
                    if (Q16) g.q[j] = buf_u16(plane_rsrc(a.xq + off), vo, 0u);
                    else g.v[j] = buf_f32(plane_rsrc(src + off), vo, 0u);
                }
            }
        }
        g.dw = 0;
        g.bw = 0;
        if (lane < G) {
            const int zi = zb + lane;
            const int zp = SRC == SRC_P ? zi - h : zi;
            const bool ok = zi < ze && (SRC == SRC_P ? zp >= z0 : (zi >= 0 && zi < nz));
            if (ok) {
                const int64_t wi = (int64_t)zp * a.wpp + wcol;
                if (a.det_in) g.dw = a.det_in[wi];
                if (SRC == SRC_P) g.bw = a.blank_in[wi];
            }
        }
    };
    // After the group zb: its clip words to the bit planes (lane j: plane j,
    // where that plane was an output plane of this block).
    auto store_words = [&](int zb) {
        const int zi = zb + lane;
        const int zo = SPEC ? zi - h : zi;
        if (lane < G && zi < ze && zo >= z0) {
            const int64_t wi = (int64_t)zo * a.wpp + wcol;
            a.det_out[wi] = oacc;
            if (SRC == SRC_X && a.blank_out) a.blank_out[wi] = bacc;
        }
    };

    float ring[W >= 3 ? W : 1];
    uint8_t bring[W >= 3 ? W : 1];   // SRC_X: working bytes of the window's planes
#pragma unroll
    for (int j = 0; j < (W >= 3 ? W : 1); ++j) { ring[j] = 0.f; bring[j] = 0; }
    int lslot = 0;           // W = 0: LDS ring slot of the next input
    double S = 0.0;
    const double inv_w = 1.0 / (double)w;
    int groups = 0;

    auto process_group = [&](int zb, const Group &g) {
        // output plane of step j: zb + j (no spectral smoothing) or zb + j - h
        const int zo0 = SPEC ? zb - h : zb;
        // bit j: output plane zo0 + j is one the noise is measured on
        uint32_t zbits = 0xffffffffu;
        if (a.zstride > 1) {
            zbits = 0u;
            for (int j = 0; j < G; ++j)
                if ((zo0 + j) % a.zstride == 0) zbits |= 1u << j;
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int zi = zb + j;
            if (zi >= ze) break;
            const int zo = zo0 + j;
            const uint64_t zsel = (zbits >> j) & 1u ? ~0ull : 0ull;
            if (!SPEC) {
                const float xv = in_value(g, j);
                const uint64_t dprev = lane_word(g.dw, j);
                if (SRC == SRC_X)
                    consume(j, zo, (double)raw_value(xv, lane_bit(dprev)),
                            ~live_m | wave_mask(!isfinite(xv)), dprev, zsel);
                else
                    consume(j, zo, (double)xv, ~live_m | lane_word(g.bw, j), dprev, zsel);
                continue;
            }
            // SRC_X keeps the working byte (kDet, kBlank) of every plane of
            // the window in a ring next to the values
            float vn;
            uint8_t wb_in = 0;
            if (SRC == SRC_X) {
                const float xv = in_value(g, j);
                const bool det = lane_bit(lane_word(g.dw, j));
                const bool blank = !active | !isfinite(xv);
                wb_in = (uint8_t)((det ? kDet : 0) | (blank ? kBlank : 0));
                vn = raw_value(xv, det);
            } else {
                vn = g.v[j];
            }
            float vo;
            uint8_t wb_out = 0;
            if (LDSRING) {
                vo = lring[lslot * B + tid];
                lring[lslot * B + tid] = vn;
                if (SRC == SRC_X) {
                    lbring[lslot * B + tid] = wb_in;
                    int os = lslot + h + 1;
                    if (os >= w) os -= w;
                    wb_out = lbring[os * B + tid];
                }
                if (++lslot == w) lslot = 0;
            } else {
                constexpr int kW = W >= 3 ? W : 1;
                const int sl = j % kW;
                vo = ring[sl];
                ring[sl] = vn;
                if (SRC == SRC_X) {
                    bring[sl] = wb_in;
                    wb_out = bring[(j + kW - (kW - 1) / 2) % kW];
                }
            }
            S += (double)vn - (double)vo;
            if (zo >= z0) {
                // output plane zo: its blank bits and earlier detections
                uint64_t blank_m, dprev;
                if (SRC == SRC_P) {
                    blank_m = ~live_m | lane_word(g.bw, j);
                    dprev = lane_word(g.dw, j);
                } else {
                    blank_m = wave_mask(wb_out >= kBlank);
                    dprev = wave_mask((wb_out & kDet) != 0);
                }
                consume(j, zo, S * inv_w, blank_m, dprev, zsel);
            }
        }
        if (OP == OP_CLIP || OP == OP_SELCLIP) store_words(zb);
        // The buffer holds one more group on top of kCapFlushAt entries.
        if (capture && fill > kCapFlushAt) flush();
        if (SELCLIP && afill > kAmbFlushAt) flush_amb();
        if (SPEC && (++groups & 7) == 0) {   // re-anchor the running sum
            S = 0.0;
            if (LDSRING) {
                for (int j = 0; j < w; ++j) S += (double)lring[j * B + tid];
            } else {
#pragma unroll
                for (int j = 0; j < (W >= 3 ? W : 1); ++j) S += (double)ring[j];
            }
        }
    };

    if (live) {
        Group ga, gb;
        load_group(zs, ga);
        for (int zb = zs; zb < ze; zb += 2 * G) {
            if (zb + G < ze) load_group(zb + G, gb);
            process_group(zb, ga);
            if (zb + G >= ze) break;
            if (zb + 2 * G < ze) load_group(zb + 2 * G, ga);
            process_group(zb + G, gb);
        }
    }
    if (capture) {
        // End of the block: what the waves still hold goes to the global lists
        // with one atomic per list for the whole block (a counter shared by
        // the whole grid serialises its atomics, so they are kept few).
        __shared__ unsigned wfill[2][B / 64];
        __shared__ unsigned long long wbase[2];
        if (lane == 0) {
            wfill[0][wave] = (unsigned)fill;
            wfill[1][wave] = (unsigned)afill;
        }
        __syncthreads();
        if (tid == 0) {
            unsigned long long nk = 0, na = 0;
            bool over = false;
            for (int v = 0; v < B / 64; ++v) {
                nk += wfill[0][v];
                na += min(wfill[1][v], (unsigned)kAmbPerWave);
                over |= wfill[1][v] > (unsigned)kAmbPerWave;
            }
            wbase[0] = nk ? atomicAdd(a.cap_count, nk) : 0ull;
            wbase[1] = 0ull;
            if (SELCLIP && (na || over))
                wbase[1] = atomicAdd(a.amb_count, na + (over ? a.amb_capacity + 1 : 0ull));
        }
        __syncthreads();
        unsigned long long bk = wbase[0], ba = wbase[1];
        for (int v = 0; v < wave; ++v) {
            bk += wfill[0][v];
            ba += min(wfill[1][v], (unsigned)kAmbPerWave);
        }
        const int nk = (int)wfill[0][wave];
        for (int i = lane; i < nk; i += 64)
            if (bk + i < a.cap_capacity) a.cap_buf[bk + i] = capw[i];
        if (SELCLIP) {
            const int na = (int)min(wfill[1][wave], (unsigned)kAmbPerWave);
            for (int i = lane; i < na; i += 64)
                if (ba + i < a.amb_capacity) a.amb[ba + i] = ambw[i];
        }
    }

    if (OP == OP_STD) {
        // Block reduction in a fixed order: deterministic partials.
        __shared__ double rs[B];
        __shared__ unsigned long long rc[B];
        rs[tid] = acc.sum;
        rc[tid] = lane == 0 ? acc.cnt : 0ull;   // the count is a wave total
        __syncthreads();
        for (int off = B / 2; off > 0; off >>= 1) {
            if (tid < off) { rs[tid] += rs[tid + off]; rc[tid] += rc[tid + off]; }
            __syncthreads();
        }
        if (tid == 0) { a.part_sum[tile] = rs[0]; a.part_cnt[tile] = rc[0]; }
    } else if (OP == OP_HIST1) {
        __syncthreads();
        for (int i = tid; i < kL1Bins; i += B)
            if (hist[i]) atomicAdd(&a.hist1[i], (unsigned long long)hist[i]);
    } else if (OP == OP_SELECT || OP == OP_SELCLIP) {
        __shared__ unsigned long long rc[2][B / 64];
        if (lane == 0) {   // wave totals
            rc[0][wave] = n_sel;
            rc[1][wave] = n_below;
        }
        __syncthreads();
        if (tid == 0) {   // per-block partials, summed by the finalize kernel
            unsigned long long ns = 0, nb = 0;
            for (int v = 0; v < B / 64; ++v) { ns += rc[0][v]; nb += rc[1][v]; }
            a.sel_part[2 * tile] = ns;
            a.sel_part[2 * tile + 1] = nb;
        }
    } else if (OP == OP_HIST2) {
        __syncthreads();
        for (int i = tid; i < 2 * kL2Coarse; i += B)
            if (hist[i]) atomicAdd(&a.hist2c[i], (unsigned long long)hist[i]);
    }
}

// Spectral widths with a register ring; any other odd width up to
// SOFIA_SC_MAX_WIDTH uses the LDS ring.
inline int ring_template_width(int w) {
    switch (w) {
        case 1: case 3: case 5: case 7: case 9: case 11: case 15: case 21: case 31: return w;
    }
    return 0;
}

inline size_t column_lds_bytes(int src, int op, bool spectral, int w) {
    size_t b = 0;
    const bool lds_ring = spectral && ring_template_width(w) == 0;
    if (lds_ring) b += (size_t)w * kColThreads * sizeof(float);
    if (lds_ring && src == SRC_X) b += ((size_t)w * kColThreads + 3) & ~(size_t)3;
    if (op == OP_HIST1) b += (size_t)kL1Bins * sizeof(unsigned);
    if (op == OP_SELECT || op == OP_SELCLIP) {
        const int tw = spectral ? ring_template_width(w) : 1;
        const int group = tw >= 3 ? tw * ((8 + tw - 1) / tw) : 8;
        b += (size_t)(kColThreads / 64) * kCapStride(group) * sizeof(uint32_t);
    }
    if (op == OP_SELCLIP) b += 16 + (size_t)(kColThreads / 64) * kAmbPerWave * sizeof(AmbEntry);
    if (op == OP_HIST2) b += (size_t)2 * kL2Coarse * sizeof(unsigned);
    return b;
}

template <int SRC, int OP, int W, int XT>
hipError_t column_inst(const ColArgs &a, int nblocks, hipStream_t s) {
    const size_t lds = column_lds_bytes(SRC, OP, W != 1, a.w);
    hipLaunchKernelGGL((k_column<SRC, OP, W, XT>), dim3(nblocks), dim3(kColThreads), lds, s, a);
    return hipGetLastError();
}

template <int SRC, int OP, int XT>
hipError_t column_width(int w, const ColArgs &a, int nb, hipStream_t s) {
    switch (ring_template_width(w)) {
        case 1: return column_inst<SRC, OP, 1, XT>(a, nb, s);
        case 3: return column_inst<SRC, OP, 3, XT>(a, nb, s);
        case 5: return column_inst<SRC, OP, 5, XT>(a, nb, s);
        case 7: return column_inst<SRC, OP, 7, XT>(a, nb, s);
        case 9: return column_inst<SRC, OP, 9, XT>(a, nb, s);
        case 11: return column_inst<SRC, OP, 11, XT>(a, nb, s);
        case 15: return column_inst<SRC, OP, 15, XT>(a, nb, s);
        case 21: return column_inst<SRC, OP, 21, XT>(a, nb, s);
        case 31: return column_inst<SRC, OP, 31, XT>(a, nb, s);
        default: return column_inst<SRC, OP, 0, XT>(a, nb, s);
    }
}

// Launch one operation of the column kernel; the raw cube's storage only
// matters for SRC_X (SRC_P is always the FP32 smoothed buffer).
template <int OP>
hipError_t launch_column_op(int src, bool spec, const ColArgs &a, int nb, hipStream_t s) {
    if (src == SRC_P && !a.blank_in) return hipErrorInvalidValue;
    if ((OP == OP_CLIP || OP == OP_SELCLIP) && !a.det_out) return hipErrorInvalidValue;
    const int w = spec ? a.w : 1;
    if (src == SRC_P) return column_width<SRC_P, OP, ST_F32>(w, a, nb, s);
    switch (a.xtype) {
        case ST_F32: return column_width<SRC_X, OP, ST_F32>(w, a, nb, s);
        case ST_F16: return column_width<SRC_X, OP, ST_F16>(w, a, nb, s);
        case ST_BF16: return column_width<SRC_X, OP, ST_BF16>(w, a, nb, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace sc
