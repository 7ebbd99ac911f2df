// Host side of the smooth-and-clip library: argument checks, the spatial
// cascade plan, workspace, the per-kernel launch sequence and the C ABI
// declared in include/sofia_sc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sc_internal.h"
#include "sofia_sc.h"

using namespace sc;

namespace {

enum Family {
    F_INIT = 0, F_FILL, F_SPATIAL, F_COL_STD, F_COL_SAMPLE, F_COL_SELECT, F_COL_HIST1,
    F_COL_HIST2, F_FALLBACK_SKIPPED, F_CAPTURE_SELECT, F_COL_CLIP, F_COL_WRITE, F_FINALIZE,
    F_QUANTIZE, F_COL_SELCLIP, F_CLIP_FIXUP, F_COUNT
};
const char *kFamilyName[F_COUNT] = {
    "init_mask", "fill", "spatial_cascade", "column_std", "column_sample",
    "column_select", "column_hist1", "column_hist2", "fallback_skipped", "capture_select",
    "column_clip", "column_write", "finalize", "quantize", "column_select_clip",
    "clip_fixup"};

struct LaunchRec {
    int fam;
    double bytes, vox;
    hipEvent_t e0, e1;
    int cond;   // >= 0: the launch only works if bit `cond` of DevState::fallback is set
};

struct Agg {
    int64_t launches = 0;
    double ms = 0, bytes = 0, vox = 0;
};

struct Plan {
    int n_iter, radius, width;   // spatial cascade; spectral width (1 = none)
    bool spatial() const { return n_iter > 0; }
    bool spectral() const { return width >= 3; }
    bool identity() const { return !spatial() && !spectral(); }
};

}  // namespace

struct sofia_sc {
    int device = 0;
    std::string err;
    uint8_t *wm[2] = {nullptr, nullptr};
    size_t wm_cap = 0;
    float *p = nullptr;
    size_t p_cap = 0;
    DevState *st = nullptr;
    DevState *st_host = nullptr;     // pinned
    unsigned long long *hist = nullptr;
    double *part_sum = nullptr;
    unsigned long long *part_cnt = nullptr;
    size_t part_cap = 0;
    uint32_t *cap_buf = nullptr;
    size_t cap_cap = 0;
    uint16_t *xq = nullptr;
    size_t xq_cap = 0;
    uint64_t *det = nullptr;         // packed detection bits (spatial replacement)
    size_t det_cap = 0;              // in words
    AmbEntry *amb = nullptr;         // undecided voxels of the fused clip
    size_t amb_cap = 0;
    bool prof = false;
    std::vector<LaunchRec> recs;
    std::vector<hipEvent_t> pool;
    Agg agg[F_COUNT];
};

namespace {

// Histogram workspace, zeroed before every MAD measurement: level 1 |
// level-2 coarse | level 2 | sampled level 1 | capture count | selection
// counts | count of voxels the fused clip left undecided.
constexpr size_t kOffL2c = kL1Bins;
constexpr size_t kOffL2 = kOffL2c + 2 * (size_t)kL2Coarse;
constexpr size_t kOffSample = kOffL2 + 2 * (size_t)kL2Bins;
constexpr size_t kOffCapCount = kOffSample + kL1Bins;
constexpr size_t kOffSelCounts = kOffCapCount + 2;
constexpr size_t kOffAmbCount = kOffSelCounts + 2;
constexpr size_t kHistWords = kOffAmbCount + 2;
// Columns blocks visited by the sampling pass: every 17th (a stride coprime
// to the usual blocks-per-row counts spreads the sample over x and y).
constexpr int kSampleStride = 17;

unsigned long long *hist1_of(sofia_sc *h) { return h->hist; }
unsigned long long *hist2c_of(sofia_sc *h) { return h->hist + kOffL2c; }
unsigned long long *hist2_of(sofia_sc *h) { return h->hist + kOffL2; }
unsigned long long *hist_s_of(sofia_sc *h) { return h->hist + kOffSample; }
unsigned long long *cap_count_of(sofia_sc *h) { return h->hist + kOffCapCount; }
unsigned long long *sel_counts_of(sofia_sc *h) { return h->hist + kOffSelCounts; }
unsigned long long *amb_count_of(sofia_sc *h) { return h->hist + kOffAmbCount; }

// Undecided-voxel list of the fused clip: up to N/256 entries (at least
// 2^16); beyond that the plain clip pass runs.
size_t amb_capacity(int64_t N) { return std::max<size_t>((size_t)N / 256, (size_t)1 << 16); }

// Capture buffer: up to N/8 keys (at least 2^20).
size_t capture_capacity(int64_t N) { return std::max<size_t>((size_t)N / 8, (size_t)1 << 20); }

int fail(sofia_sc *h, int code, const std::string &msg) {
    if (h) h->err = msg;
    return code;
}

int hip_fail(sofia_sc *h, hipError_t e, const char *what) {
    return fail(h, SOFIA_SC_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

// Reading of the Gaussian construction: sigma_g^2 = (FWHM / 2 sqrt(2 ln 2))^2
// is matched by n boxcars of width 2r+1 (variance n r (r+1) / 3 each axis).
// For each n the best r lies next to the positive root of
// n r (r+1) / 3 = sigma_g^2; candidates are compared by distance, then
// larger n, then smaller r.
int plan_cascade(double fwhm, int32_t *n_iter, int32_t *radius) {
    if (!std::isfinite(fwhm) || fwhm < 0.0) return SOFIA_SC_EINVAL;
    if (fwhm == 0.0) { *n_iter = 0; *radius = 0; return SOFIA_SC_OK; }
    const double sg = fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    const double var = sg * sg;
    int bn = 0, br = 0;
    double bd = INFINITY;
    for (int n = 6; n >= 3; --n) {
        const double root = 0.5 * (std::sqrt(1.0 + 12.0 * var / n) - 1.0);
        const int rf = std::max(1, (int)std::floor(root));
        for (int r = std::max(1, rf - 1); r <= rf + 2; ++r) {
            const double v = (double)((int64_t)n * r * (r + 1)) / 3.0;
            const double d = std::fabs(v - var);
            if (d < bd || (d == bd && n == bn && r < br)) { bd = d; bn = n; br = r; }
        }
    }
    *n_iter = bn;
    *radius = br;
    return SOFIA_SC_OK;
}

bool valid_width(int32_t w) {
    return w == 0 || w == 1 || (w >= 3 && (w & 1) && w <= SOFIA_SC_MAX_WIDTH);
}

int make_plan(sofia_sc *h, const sofia_sc_kernel &k, Plan *p) {
    int32_t n, r;
    if (plan_cascade(k.spatial_fwhm_px, &n, &r) != SOFIA_SC_OK)
        return fail(h, SOFIA_SC_EINVAL, "spatial FWHM must be finite and >= 0");
    if (n * r > SOFIA_SC_MAX_HALO)
        return fail(h, SOFIA_SC_EINVAL, "spatial FWHM too large (cascade halo above limit)");
    if (!valid_width(k.spectral_width_ch))
        return fail(h, SOFIA_SC_EINVAL, "spectral width must be 0, 1 or odd in 3..63");
    p->n_iter = n;
    p->radius = r;
    p->width = k.spectral_width_ch < 3 ? 1 : k.spectral_width_ch;
    return SOFIA_SC_OK;
}

int check_dims(sofia_sc *h, int64_t nx, int64_t ny, int64_t nz) {
    if (nx < 1 || ny < 1 || nz < 1)
        return fail(h, SOFIA_SC_EINVAL, "cube dimensions must be >= 1");
    const double n = (double)nx * (double)ny * (double)nz;
    if (n > 1099511627776.0) return fail(h, SOFIA_SC_EINVAL, "cube larger than 2^40 voxels");
    if (nx * ny > 0x7fffffffLL * 256LL)
        return fail(h, SOFIA_SC_EINVAL, "plane too large");
    return SOFIA_SC_OK;
}

int check_modes(sofia_sc *h, double t, int32_t mode, int32_t range) {
    if (!std::isfinite(t) || t <= 0.0)
        return fail(h, SOFIA_SC_EINVAL, "threshold must be finite and > 0");
    if (mode != SOFIA_SC_NOISE_STD && mode != SOFIA_SC_NOISE_MAD)
        return fail(h, SOFIA_SC_EINVAL, "unknown noise mode");
    if (range != SOFIA_SC_FLUX_NEGATIVE && range != SOFIA_SC_FLUX_ALL &&
        range != SOFIA_SC_FLUX_POSITIVE)
        return fail(h, SOFIA_SC_EINVAL, "unknown flux range");
    return SOFIA_SC_OK;
}

// Column-kernel grid: 256 columns per block; z is split only as far as
// needed to give the chip several waves of blocks.
struct ColGrid {
    int ncb, nzc, zchunk;
    int blocks() const { return ncb * nzc; }
};

ColGrid col_grid(int64_t ncol, int64_t nz) {
    ColGrid g;
    g.ncb = (int)((ncol + kColThreads - 1) / kColThreads);
    const int64_t target = 6144;
    int64_t nzc = (target + g.ncb - 1) / g.ncb;
    const int64_t max_nzc = std::max<int64_t>(1, nz / 64);
    nzc = std::max<int64_t>(1, std::min(nzc, max_nzc));
    g.zchunk = (int)((nz + nzc - 1) / nzc);
    g.nzc = (int)((nz + g.zchunk - 1) / g.zchunk);
    return g;
}

// 16-bit copy of the cube for F16/BF16 storage.
int ensure_q16(sofia_sc *h, int64_t N) {
    if ((size_t)N <= h->xq_cap) return SOFIA_SC_OK;
    if (h->xq) (void)hipFree(h->xq);
    h->xq = nullptr;
    h->xq_cap = 0;
    const hipError_t e = hipMalloc(&h->xq, (size_t)N * sizeof(uint16_t));
    if (e != hipSuccess)
        return fail(h, SOFIA_SC_ENOMEM, std::string("16-bit cube: ") + hipGetErrorString(e));
    h->xq_cap = (size_t)N;
    return SOFIA_SC_OK;
}

// Packed detection bits: words per plane of nx * ny voxels.
int64_t det_words_per_plane(int64_t ncol) { return (ncol + 63) / 64; }

int ensure_workspace(sofia_sc *h, int64_t N, bool need_p, size_t parts,
                     int64_t det_words = 0) {
    hipError_t e;
    if ((size_t)det_words > h->det_cap) {
        if (h->det) (void)hipFree(h->det);
        h->det = nullptr;
        h->det_cap = 0;
        if ((e = hipMalloc(&h->det, (size_t)det_words * sizeof(uint64_t))) != hipSuccess)
            return fail(h, SOFIA_SC_ENOMEM, std::string("detection bits: ") + hipGetErrorString(e));
        h->det_cap = (size_t)det_words;
    }
    if (!h->st) {
        if ((e = hipMalloc(&h->st, sizeof(DevState))) != hipSuccess)
            return fail(h, SOFIA_SC_ENOMEM, std::string("state: ") + hipGetErrorString(e));
        if ((e = hipHostMalloc(&h->st_host, sizeof(DevState), hipHostMallocDefault)) != hipSuccess)
            return fail(h, SOFIA_SC_ENOMEM, std::string("host state: ") + hipGetErrorString(e));
        if ((e = hipMalloc(&h->hist, kHistWords * sizeof(unsigned long long))) != hipSuccess)
            return fail(h, SOFIA_SC_ENOMEM, std::string("histograms: ") + hipGetErrorString(e));
    }
    if ((size_t)N > h->wm_cap) {
        for (int i = 0; i < 2; ++i) {
            if (h->wm[i]) (void)hipFree(h->wm[i]);
            h->wm[i] = nullptr;
        }
        h->wm_cap = 0;
        for (int i = 0; i < 2; ++i)
            if ((e = hipMalloc(&h->wm[i], (size_t)N)) != hipSuccess)
                return fail(h, SOFIA_SC_ENOMEM, std::string("working mask: ") + hipGetErrorString(e));
        h->wm_cap = (size_t)N;
    }
    if (need_p && (size_t)N > h->p_cap) {
        if (h->p) (void)hipFree(h->p);
        h->p = nullptr;
        h->p_cap = 0;
        if ((e = hipMalloc(&h->p, (size_t)N * sizeof(float))) != hipSuccess)
            return fail(h, SOFIA_SC_ENOMEM, std::string("plane buffer: ") + hipGetErrorString(e));
        h->p_cap = (size_t)N;
    }
    const size_t acap = amb_capacity(N);
    if (acap > h->amb_cap) {
        if (h->amb) (void)hipFree(h->amb);
        h->amb = nullptr;
        h->amb_cap = 0;
        if ((e = hipMalloc(&h->amb, acap * sizeof(AmbEntry))) != hipSuccess)
            return fail(h, SOFIA_SC_ENOMEM, std::string("undecided list: ") + hipGetErrorString(e));
        h->amb_cap = acap;
    }
    const size_t cap = capture_capacity(N);
    if (cap > h->cap_cap) {
        if (h->cap_buf) (void)hipFree(h->cap_buf);
        h->cap_buf = nullptr;
        h->cap_cap = 0;
        if ((e = hipMalloc(&h->cap_buf, cap * sizeof(uint32_t))) != hipSuccess)
            return fail(h, SOFIA_SC_ENOMEM, std::string("capture buffer: ") + hipGetErrorString(e));
        h->cap_cap = cap;
    }
    if (parts > h->part_cap) {
        if (h->part_sum) (void)hipFree(h->part_sum);
        if (h->part_cnt) (void)hipFree(h->part_cnt);
        h->part_sum = nullptr;
        h->part_cnt = nullptr;
        h->part_cap = 0;
        if ((e = hipMalloc(&h->part_sum, parts * sizeof(double))) != hipSuccess ||
            (e = hipMalloc(&h->part_cnt, parts * sizeof(unsigned long long))) != hipSuccess)
            return fail(h, SOFIA_SC_ENOMEM, std::string("partials: ") + hipGetErrorString(e));
        h->part_cap = parts;
    }
    return SOFIA_SC_OK;
}

// ---- launch bookkeeping (HIP events around each launch while profiling)

hipEvent_t take_event(sofia_sc *h) {
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

template <typename F>
int launch(sofia_sc *h, hipStream_t s, int fam, double bytes, double vox, F &&f,
           int cond = -1) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (h->prof) {
        e0 = take_event(h);
        e1 = take_event(h);
        if (e0) (void)hipEventRecord(e0, s);
    }
    const hipError_t e = f();
    if (e != hipSuccess) return hip_fail(h, e, kFamilyName[fam]);
    if (h->prof && e0 && e1) {
        (void)hipEventRecord(e1, s);
        h->recs.push_back({fam, bytes, vox, e0, e1, cond});
    }
    return SOFIA_SC_OK;
}

// Called after the stream has been synchronised.
void collect_profile(sofia_sc *h) {
    for (auto &r : h->recs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
            // cond k < 64: runs only when kernel k needed the full histogram
            // passes; cond 64 + k: only when it needed the full clip pass
            const DevState &hs = *h->st_host;
            const bool skipped =
                r.cond >= 0 && !(r.cond < 64 ? (hs.fallback >> r.cond) & 1ull
                                              : (hs.clip_fallback >> (r.cond - 64)) & 1ull);
            Agg &a = h->agg[skipped ? F_FALLBACK_SKIPPED : r.fam];
            if (skipped) { r.bytes = 0; r.vox = 0; }
            a.launches += 1;
            a.ms += ms;
            a.bytes += r.bytes;
            a.vox += r.vox;
        }
        h->pool.push_back(r.e0);
        h->pool.push_back(r.e1);
    }
    h->recs.clear();
}

struct Dims {
    int64_t nx, ny, nz, ncol, N;
};

// One S+C iteration on the device. k >= 0 stores sigma_k; k = -1 measures
// sigma_0 only. wm_in (may be null only for the first, unsmoothed kernel)
// carries the detections so far and the blank bits. clip_out = null skips
// the clip; write_out != null writes s instead of measuring the noise.
struct PairJob {
    const float *x;
    const uint16_t *xq;   // 16-bit noise-scaled cube (xtype != ST_F32)
    int xtype;
    Dims d;
    Plan pl;
    int k;
    bool repl_active;
    double repl_n;
    int mode, range;
    double t;
    const uint8_t *wm_in;
    uint8_t *clip_out;
    bool out_user;
    bool also_sigma0;
    float *write_out;
    bool det_live = false;  // this call sized h->det for the cube: the clip keeps
                            // the packed detection bits, the spatial pass reads them
    bool det_next = false;  // the next kernel is spatial with replacement: the
                            // clip must write the packed bits
};

int run_pair(sofia_sc *h, hipStream_t s, const PairJob &j) {
    const Dims &d = j.d;
    const double N = (double)d.N;
    int rc;
    const bool spatial = j.pl.spatial();
    const bool spec = j.pl.spectral();
    const bool has_wm = j.wm_in != nullptr;
    const double bx = j.xtype != ST_F32 ? 2.0 : 4.0;   // bytes per raw voxel
    if ((spatial || spec) && !has_wm)
        return fail(h, SOFIA_SC_EINVAL, "internal: smoothing without working mask");

    const ColGrid g = col_grid(d.ncol, d.nz);
    if ((int64_t)g.ncb * g.nzc > 0x7fffffffLL)
        return fail(h, SOFIA_SC_EINVAL, "cube too large for the column grid");
    if (spatial) {
        StripArgs a{};
        a.x = j.xtype == ST_F32 ? j.x : nullptr;
        a.xq = j.xtype != ST_F32 ? j.xq : nullptr;
        a.wpp = det_words_per_plane(d.ncol);
        a.det = nullptr;
        if (j.repl_active) {
            if (!j.det_live || h->det_cap < (size_t)(d.nz * a.wpp))
                return fail(h, SOFIA_SC_EINVAL, "internal: detection bits not sized");
            a.det = h->det;
        }
        a.p = h->p;
        a.nx = d.nx; a.ny = d.ny; a.nz = d.nz;
        spatial_strips(a, j.pl.n_iter, j.pl.radius);
        if (a.tiles > 0x7fffffffLL)
            return fail(h, SOFIA_SC_EINVAL, "cube too large for the spatial grid");
        a.repl_n = j.repl_n;
        a.st = h->st;
        const double bytes = N * (bx + (j.repl_active ? 1.0 : 0.0) + 4.0);
        rc = launch(h, s, F_SPATIAL, bytes, N, [&] {
            return launch_spatial(j.pl.n_iter, j.pl.radius, j.xtype, j.repl_active, a, s);
        });
        if (rc) return rc;
    }

    ColArgs c{};
    c.x = j.x;
    c.xq = j.xq;
    c.xtype = j.xtype;
    c.p = h->p;
    c.wm_in = j.wm_in;
    c.ncol = d.ncol;
    c.nz = d.nz;
    c.w = j.pl.width;
    c.h = (j.pl.width - 1) / 2;
    c.zchunk = g.zchunk;
    c.ncb = g.ncb;
    c.range = j.range;
    c.repl_on = (!spatial && j.repl_active) ? 1 : 0;
    c.repl_n = j.repl_n;
    c.st = h->st;
    c.part_sum = h->part_sum;
    c.part_cnt = h->part_cnt;
    c.hist1 = hist1_of(h);
    c.hist2 = hist2_of(h);
    c.hist2c = hist2c_of(h);
    c.cb_stride = 1;
    c.cap_buf = h->cap_buf;
    c.cap_count = cap_count_of(h);
    c.cap_capacity = (unsigned long long)h->cap_cap;
    c.sel_counts = sel_counts_of(h);
    const int src = spatial ? SRC_P : SRC_X;
    const double rd = N * ((spatial ? 4.0 : bx) + (has_wm ? 1.0 : 0.0));
    auto col = [&](int op, int fam, double bytes) {
        return launch(h, s, fam, bytes, N, [&] {
            return launch_column(src, op, spec, has_wm, c, g.blocks(), s);
        });
    };

    if (j.write_out) {
        c.s_out = j.write_out;
        return col(OP_WRITE, F_COL_WRITE, rd + 4.0 * N);
    }

    // Clip target: the next working mask (with the packed detection bits a
    // later spatial kernel replaces from) or, for the last kernel, the
    // caller's 0/1 mask.
    double clip_bytes = 0.0;
    if (j.clip_out) {
        c.mask_out = j.clip_out;
        c.out_user = j.out_user ? 1 : 0;
        c.wpp = det_words_per_plane(d.ncol);
        c.det_bits = nullptr;
        if (j.det_live && j.det_next && !j.out_user) {
            if (h->det_cap < (size_t)(d.nz * c.wpp))
                return fail(h, SOFIA_SC_EINVAL, "internal: detection bits not sized");
            c.det_bits = h->det;
        }
        clip_bytes = N + (c.det_bits ? N / 8.0 : 0.0);
    }
    const int cond = j.k >= 0 ? j.k : 63;
    // With MAD noise the clip rides on the selection pass (see below).
    const bool fused = j.clip_out && j.mode != SOFIA_SC_NOISE_STD;

    if (j.mode == SOFIA_SC_NOISE_STD) {
        if ((rc = col(OP_STD, F_COL_STD, rd))) return rc;
        rc = launch(h, s, F_FINALIZE, 16.0 * g.blocks(), 0, [&] {
            return launch_finalize_std(h->st, h->part_sum, h->part_cnt, g.blocks(),
                                       j.k, j.t, j.also_sigma0 ? 1 : 0, s);
        });
        if (rc) return rc;
    } else {
        // Exact MAD. A sample of columns predicts the median; one pass counts
        // the selected voxels and those below a window around the prediction
        // and captures the keys inside it; the two central order statistics
        // are then found among the captured keys (radix walk, 12+10+9 bits).
        // If the window missed them, full level-1 and level-2 passes over the
        // cube run instead (each launch checks the flag and exits otherwise).
        rc = launch(h, s, F_FILL, 8.0 * kHistWords, 0, [&] {
            return launch_fill_u64(h->hist, (int64_t)kHistWords, s);
        });
        if (rc) return rc;
        {
            // The sample touches 1/17 of the columns: split z finer so the
            // launch still has a few blocks per CU.
            ColArgs cs = c;
            cs.cb_stride = kSampleStride;
            cs.ncb = (g.ncb + kSampleStride - 1) / kSampleStride;
            cs.hist1 = hist_s_of(h);
            int nzc = (int)std::min<int64_t>((2048 + cs.ncb - 1) / cs.ncb,
                                             std::max<int64_t>(1, d.nz / 32));
            nzc = std::max(nzc, 1);
            cs.zchunk = (int)((d.nz + nzc - 1) / nzc);
            nzc = (int)((d.nz + cs.zchunk - 1) / cs.zchunk);
            const int nb = cs.ncb * nzc;
            rc = launch(h, s, F_COL_SAMPLE, rd * cs.ncb / g.ncb, N * cs.ncb / g.ncb, [&] {
                return launch_column(src, OP_HIST1, spec, has_wm, cs, nb, s);
            });
            if (rc) return rc;
        }
        rc = launch(h, s, F_FINALIZE, 8.0 * kL1Bins, 0, [&] {
            return launch_finalize_predict(h->st, hist_s_of(h), j.t, s);
        });
        if (rc) return rc;
        // Fused clip: the predicted median window bounds the threshold, so
        // the selection pass also clips every voxel whose |s| lies outside
        // (thr_lo, thr_hi] and lists the others for an exact decision later.
        if (fused) {
            c.amb = h->amb;
            c.amb_count = amb_count_of(h);
            c.amb_capacity = (unsigned long long)h->amb_cap;
            if ((rc = col(OP_SELCLIP, F_COL_SELCLIP, rd + clip_bytes))) return rc;
        } else {
            if ((rc = col(OP_SELECT, F_COL_SELECT, rd))) return rc;
        }
        rc = launch(h, s, F_FINALIZE, 0, 0, [&] {
            return launch_finalize_select(h->st, sel_counts_of(h), cap_count_of(h),
                                          (unsigned long long)h->cap_cap, j.k,
                                          fused ? amb_count_of(h) : nullptr,
                                          (unsigned long long)h->amb_cap, s);
        });
        if (rc) return rc;
        rc = launch(h, s, F_CAPTURE_SELECT, 0, 0, [&] {
            return launch_capture_l1(h->st, h->cap_buf, cap_count_of(h), hist1_of(h), s);
        });
        if (rc) return rc;
        c.skip_if_captured = 1;
        rc = launch(h, s, F_COL_HIST1, rd, N, [&] {
            return launch_column(src, OP_HIST1, spec, has_wm, c, g.blocks(), s);
        }, cond);
        if (rc) return rc;
        rc = launch(h, s, F_FINALIZE, 8.0 * kL1Bins, 0, [&] {
            return launch_finalize_mad1(h->st, hist1_of(h), s);
        });
        if (rc) return rc;
        rc = launch(h, s, F_CAPTURE_SELECT, 0, 0, [&] {
            return launch_capture_coarse(h->st, h->cap_buf, cap_count_of(h), hist2c_of(h), s);
        });
        if (rc) return rc;
        rc = launch(h, s, F_COL_HIST2, rd, N, [&] {
            return launch_column(src, OP_HIST2, spec, has_wm, c, g.blocks(), s);
        }, cond);
        c.skip_if_captured = 0;
        if (rc) return rc;
        rc = launch(h, s, F_FINALIZE, 8.0 * 2 * kL2Coarse, 0, [&] {
            return launch_finalize_mad2a(h->st, hist2c_of(h), s);
        });
        if (rc) return rc;
        rc = launch(h, s, F_CAPTURE_SELECT, 0, 0, [&] {
            return launch_capture_fine(h->st, h->cap_buf, cap_count_of(h), hist2_of(h), s);
        });
        if (rc) return rc;
        rc = launch(h, s, F_FINALIZE, 8.0 * 2 * kL2Fine, 0, [&] {
            return launch_finalize_mad2b(h->st, hist2_of(h), j.k, j.t,
                                         j.also_sigma0 ? 1 : 0, s);
        });
        if (rc) return rc;
    }
    if (fused) {
        // decide the listed voxels; the full clip pass below runs only when
        // the median missed the window or the list overflowed
        rc = launch(h, s, F_CLIP_FIXUP, 0, 0, [&] {
            return launch_clip_fixup(h->st, h->amb, amb_count_of(h),
                                     (unsigned long long)h->amb_cap, c.mask_out, c.out_user,
                                     c.det_bits, d.ncol, c.wpp, s);
        });
        if (rc) return rc;
        c.skip_if_fused = 1;
        rc = launch(h, s, F_COL_CLIP, rd + clip_bytes, N, [&] {
            return launch_column(src, OP_CLIP, spec, has_wm, c, g.blocks(), s);
        }, 64 + cond);
        c.skip_if_fused = 0;
        if (rc) return rc;
    } else if (j.clip_out) {
        if ((rc = col(OP_CLIP, F_COL_CLIP, rd + clip_bytes))) return rc;
    }
    return SOFIA_SC_OK;
}

// Scoped device selection; restores the caller's current device.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int finish(sofia_sc *h, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(h->st_host, h->st, sizeof(DevState),
                                  hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(h, e, "copy of noise values");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(h, e, "stream");
    if (h->prof) collect_profile(h);
    return SOFIA_SC_OK;
}

void nan_fill(double *v, int n) {
    if (v)
        for (int i = 0; i < n; ++i) v[i] = NAN;
}

int run_impl(sofia_sc *h, const float *cube, int64_t nx, int64_t ny, int64_t nz,
             const sofia_sc_kernel *kernels, int32_t K, double t, int32_t mode,
             int32_t range, uint8_t *mask, double *noise, const sofia_sc_options *opt,
             double *sigma0_out) {
    if (!h) return SOFIA_SC_EINVAL;
    h->err.clear();
    if (noise && K > 0 && K <= SOFIA_SC_MAX_KERNELS) nan_fill(noise, K);
    if (sigma0_out) *sigma0_out = NAN;
    if (!cube || !kernels || !mask || !noise)
        return fail(h, SOFIA_SC_EINVAL, "NULL argument");
    if (K < 1 || K > SOFIA_SC_MAX_KERNELS)
        return fail(h, SOFIA_SC_EINVAL, "number of kernels must be 1..64");
    if (!opt || opt->struct_size != sizeof(sofia_sc_options))
        return fail(h, SOFIA_SC_EINVAL, "options missing or struct_size mismatch");
    int rc;
    if ((rc = check_dims(h, nx, ny, nz))) return rc;
    if ((rc = check_modes(h, t, mode, range))) return rc;
    if (std::isnan(opt->replacement) || opt->replacement == INFINITY)
        return fail(h, SOFIA_SC_EINVAL, "replacement must be finite");
    const int storage = opt->storage;
    if (storage != SOFIA_SC_STORE_F32 && storage != SOFIA_SC_STORE_F16 &&
        storage != SOFIA_SC_STORE_BF16)
        return fail(h, SOFIA_SC_EINVAL, "unknown storage");
    if (opt->reserved != 0) return fail(h, SOFIA_SC_EINVAL, "reserved option field must be 0");
    const bool given0 = !std::isnan(opt->sigma0);
    if (given0 && !(std::isfinite(opt->sigma0) && opt->sigma0 > 0.0))
        return fail(h, SOFIA_SC_EINVAL, "sigma0 must be NaN (measure) or finite and > 0");
    std::vector<Plan> plans((size_t)K);
    bool any_spatial = false;
    for (int k = 0; k < K; ++k) {
        if ((rc = make_plan(h, kernels[k], &plans[k]))) return rc;
        any_spatial |= plans[k].spatial();
    }
    DeviceGuard dg(h->device);
    if (dg.err != hipSuccess) return hip_fail(h, dg.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)opt->stream;
    Dims d{nx, ny, nz, nx * ny, nx * ny * nz};
    const ColGrid g = col_grid(d.ncol, d.nz);
    const bool q16 = storage != SOFIA_SC_STORE_F32;
    if ((rc = ensure_workspace(h, d.N, any_spatial, (size_t)g.blocks(),
                               any_spatial ? d.nz * det_words_per_plane(d.ncol) : 0)))
        return rc;
    if (q16 && (rc = ensure_q16(h, d.N))) return rc;

    const bool repl_on = opt->replacement >= 0.0;
    const bool first_identity = plans[0].identity();
    rc = launch(h, s, F_FINALIZE, 0, 0, [&] {
        return launch_set_sigma0(h->st, given0 ? opt->sigma0 : NAN, s);
    });
    if (rc) return rc;
    int cur = 0;
    bool have_wm = false;
    if (!first_identity) {
        rc = launch(h, s, F_INIT, 5.0 * d.N, (double)d.N, [&] {
            return launch_init_mask(cube, nullptr, h->wm[0], d.N, s);
        });
        if (rc) return rc;
        have_wm = true;
    }
    // sigma_0 on the FP32 cube when replacement or 16-bit scaling needs it and
    // it cannot come from kernel 1 (a (0, 0) kernel measured on FP32 data).
    if (!given0 && (q16 || (repl_on && !first_identity))) {
        PairJob j{cube, nullptr, ST_F32, d, Plan{0, 0, 1}, -1, false, 0.0, mode, range, t,
                  have_wm ? h->wm[cur] : nullptr, nullptr, false, false, nullptr};
        if ((rc = run_pair(h, s, j))) return rc;
    }
    int xtype = ST_F32;
    if (q16) {
        xtype = storage == SOFIA_SC_STORE_F16 ? ST_F16 : ST_BF16;
        rc = launch(h, s, F_QUANTIZE, 6.0 * d.N, (double)d.N, [&] {
            return launch_quantize(cube, h->st, 0.0, xtype, h->xq, d.N, s);
        });
        if (rc) return rc;
        rc = launch(h, s, F_FINALIZE, 0, 0, [&] { return launch_enter_scaled(h->st, s); });
        if (rc) return rc;
    }
    for (int k = 0; k < K; ++k) {
        const bool last = k == K - 1;
        uint8_t *out = last ? mask : (have_wm ? h->wm[1 - cur] : h->wm[cur]);
        PairJob j{cube, q16 ? h->xq : nullptr, xtype, d, plans[k], k, repl_on && k >= 1,
                  opt->replacement, mode, range, t, have_wm ? h->wm[cur] : nullptr, out, last,
                  k == 0 && first_identity && repl_on && !given0 && !q16, nullptr,
                  any_spatial, !last && plans[k + 1].spatial() && repl_on};
        if ((rc = run_pair(h, s, j))) return rc;
        if (!last) {
            if (have_wm) cur = 1 - cur;
            have_wm = true;
        }
    }
    if ((rc = finish(h, s))) return rc;
    const DevState &hs = *h->st_host;
    const double scale = q16 ? hs.scale : 1.0;   // stored units -> cube units
    for (int k = 0; k < K; ++k) noise[k] = hs.sigma[k] * scale;
    if (sigma0_out) *sigma0_out = q16 ? hs.scale : (repl_on || given0 ? hs.sigma0 : NAN);
    if (hs.status) return fail(h, SOFIA_SC_ENOSTAT, "no finite voxel in the flux range for some kernel");
    return SOFIA_SC_OK;
}

}  // namespace

extern "C" {

void sofia_sc_default_options(sofia_sc_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->struct_size = sizeof(sofia_sc_options);
    opt->replacement = 2.0;
    opt->sigma0 = NAN;
    opt->storage = SOFIA_SC_STORE_F32;
    opt->reserved = 0;
    opt->stream = nullptr;
}

int sofia_sc_quantize(sofia_sc *h, const float *cube, int64_t n, double scale,
                      int32_t storage, uint16_t *out, void *stream) {
    if (!h) return SOFIA_SC_EINVAL;
    h->err.clear();
    if (!cube || !out || n < 1) return fail(h, SOFIA_SC_EINVAL, "NULL argument or n < 1");
    if (!(std::isfinite(scale) && scale > 0.0))
        return fail(h, SOFIA_SC_EINVAL, "scale must be finite and > 0");
    if (storage != SOFIA_SC_STORE_F16 && storage != SOFIA_SC_STORE_BF16)
        return fail(h, SOFIA_SC_EINVAL, "storage must be F16 or BF16");
    DeviceGuard dg(h->device);
    if (dg.err != hipSuccess) return hip_fail(h, dg.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const int type = storage == SOFIA_SC_STORE_F16 ? ST_F16 : ST_BF16;
    int rc = launch(h, s, F_QUANTIZE, 6.0 * n, (double)n, [&] {
        return launch_quantize(cube, nullptr, scale, type, out, n, s);
    });
    if (rc) return rc;
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "stream");
    if (h->prof) collect_profile(h);
    return SOFIA_SC_OK;
}

int sofia_sc_create(sofia_sc **out, int device_ordinal) {
    if (!out) return SOFIA_SC_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return SOFIA_SC_EDEVICE;
    if (device_ordinal < 0 || device_ordinal >= n) return SOFIA_SC_EINVAL;
    sofia_sc *h = new (std::nothrow) sofia_sc();
    if (!h) return SOFIA_SC_ENOMEM;
    h->device = device_ordinal;
    *out = h;
    return SOFIA_SC_OK;
}

void sofia_sc_destroy(sofia_sc *h) {
    if (!h) return;
    {
        DeviceGuard dg(h->device);
        for (auto &r : h->recs) { (void)hipEventDestroy(r.e0); (void)hipEventDestroy(r.e1); }
        for (auto e : h->pool) (void)hipEventDestroy(e);
        if (h->wm[0]) (void)hipFree(h->wm[0]);
        if (h->wm[1]) (void)hipFree(h->wm[1]);
        if (h->p) (void)hipFree(h->p);
        if (h->st) (void)hipFree(h->st);
        if (h->st_host) (void)hipHostFree(h->st_host);
        if (h->hist) (void)hipFree(h->hist);
        if (h->part_sum) (void)hipFree(h->part_sum);
        if (h->part_cnt) (void)hipFree(h->part_cnt);
        if (h->cap_buf) (void)hipFree(h->cap_buf);
        if (h->xq) (void)hipFree(h->xq);
        if (h->det) (void)hipFree(h->det);
        if (h->amb) (void)hipFree(h->amb);
    }
    delete h;
}

int sofia_sc_run(sofia_sc *h, const float *cube, int64_t nx, int64_t ny,
                 int64_t nz, const sofia_sc_kernel *kernels, int32_t n_kernels,
                 double threshold, int32_t noise_mode, int32_t flux_range,
                 uint8_t *mask, double *noise) {
    sofia_sc_options opt;
    sofia_sc_default_options(&opt);
    return run_impl(h, cube, nx, ny, nz, kernels, n_kernels, threshold, noise_mode,
                    flux_range, mask, noise, &opt, nullptr);
}

int sofia_sc_run_ex(sofia_sc *h, const float *cube, int64_t nx, int64_t ny,
                    int64_t nz, const sofia_sc_kernel *kernels,
                    int32_t n_kernels, double threshold, int32_t noise_mode,
                    int32_t flux_range, uint8_t *mask, double *noise,
                    const sofia_sc_options *opt, double *sigma0) {
    return run_impl(h, cube, nx, ny, nz, kernels, n_kernels, threshold, noise_mode,
                    flux_range, mask, noise, opt, sigma0);
}

static int single_kernel(sofia_sc *h, const float *cube, int64_t nx, int64_t ny,
                         int64_t nz, sofia_sc_kernel kernel, double threshold,
                         int32_t mode, int32_t range, double replacement,
                         double sigma0, const uint8_t *mask_in, uint8_t *mask_out,
                         double *noise, float *write_out, int32_t storage, void *stream) {
    if (!h) return SOFIA_SC_EINVAL;
    h->err.clear();
    if (noise) *noise = NAN;
    if (!cube || (!write_out && (!mask_out || !noise)))
        return fail(h, SOFIA_SC_EINVAL, "NULL argument");
    if (mask_out && mask_in == mask_out)
        return fail(h, SOFIA_SC_EINVAL, "mask_out must not alias mask_in");
    int rc;
    if ((rc = check_dims(h, nx, ny, nz))) return rc;
    if (!write_out && (rc = check_modes(h, threshold, mode, range))) return rc;
    if (std::isnan(replacement) || std::isinf(replacement))
        return fail(h, SOFIA_SC_EINVAL, "replacement must be finite");
    const bool repl = replacement >= 0.0;
    if (repl && !std::isfinite(sigma0))
        return fail(h, SOFIA_SC_EINVAL, "sigma0 must be finite when replacement is on");
    if (storage != SOFIA_SC_STORE_F32 && storage != SOFIA_SC_STORE_F16 &&
        storage != SOFIA_SC_STORE_BF16)
        return fail(h, SOFIA_SC_EINVAL, "unknown storage");
    const bool q16 = storage != SOFIA_SC_STORE_F32;
    if (q16 && write_out) return fail(h, SOFIA_SC_EINVAL, "internal: 16-bit smoothed output");
    if (q16 && !(std::isfinite(sigma0) && sigma0 > 0.0))
        return fail(h, SOFIA_SC_EINVAL, "16-bit storage needs sigma0 finite and > 0");
    Plan pl;
    if ((rc = make_plan(h, kernel, &pl))) return rc;
    DeviceGuard dg(h->device);
    if (dg.err != hipSuccess) return hip_fail(h, dg.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    Dims d{nx, ny, nz, nx * ny, nx * ny * nz};
    const ColGrid g = col_grid(d.ncol, d.nz);
    if ((rc = ensure_workspace(h, d.N, pl.spatial(), (size_t)g.blocks(),
                               pl.spatial() ? d.nz * det_words_per_plane(d.ncol) : 0)))
        return rc;
    if (q16 && (rc = ensure_q16(h, d.N))) return rc;
    rc = launch(h, s, F_FINALIZE, 0, 0, [&] {
        return launch_set_sigma0(h->st, (repl || q16) ? sigma0 : NAN, s);
    });
    if (rc) return rc;
    rc = launch(h, s, F_INIT, (mask_in ? 6.0 : 5.0) * d.N, (double)d.N, [&] {
        return launch_init_mask(cube, mask_in, h->wm[0], d.N, s);
    });
    if (rc) return rc;
    if (pl.spatial() && repl) {
        rc = launch(h, s, F_INIT, 1.125 * d.N, (double)d.N, [&] {
            return launch_pack_det(h->wm[0], h->det, d.ncol, d.nz,
                                   det_words_per_plane(d.ncol), s);
        });
        if (rc) return rc;
    }
    int xtype = ST_F32;
    if (q16) {
        xtype = storage == SOFIA_SC_STORE_F16 ? ST_F16 : ST_BF16;
        rc = launch(h, s, F_QUANTIZE, 6.0 * d.N, (double)d.N, [&] {
            return launch_quantize(cube, h->st, 0.0, xtype, h->xq, d.N, s);
        });
        if (rc) return rc;
        rc = launch(h, s, F_FINALIZE, 0, 0, [&] { return launch_enter_scaled(h->st, s); });
        if (rc) return rc;
    }
    PairJob j{cube, q16 ? h->xq : nullptr, xtype, d, pl, 0, repl, replacement,
              write_out ? 0 : mode, write_out ? 0 : range, write_out ? 1.0 : threshold,
              h->wm[0], write_out ? nullptr : mask_out, true, false, write_out,
              pl.spatial()};
    if ((rc = run_pair(h, s, j))) return rc;
    if ((rc = finish(h, s))) return rc;
    if (write_out) return SOFIA_SC_OK;
    *noise = h->st_host->sigma[0] * (q16 ? h->st_host->scale : 1.0);
    if (h->st_host->status)
        return fail(h, SOFIA_SC_ENOSTAT, "no finite voxel in the flux range");
    return SOFIA_SC_OK;
}

int sofia_sc_step(sofia_sc *h, const float *cube, int64_t nx, int64_t ny,
                  int64_t nz, sofia_sc_kernel kernel, double threshold,
                  int32_t noise_mode, int32_t flux_range, double replacement,
                  double sigma0, const uint8_t *mask_in, uint8_t *mask_out,
                  double *noise, void *stream) {
    return single_kernel(h, cube, nx, ny, nz, kernel, threshold, noise_mode,
                         flux_range, replacement, sigma0, mask_in, mask_out, noise,
                         nullptr, SOFIA_SC_STORE_F32, stream);
}

int sofia_sc_step_ex(sofia_sc *h, const float *cube, int64_t nx, int64_t ny,
                     int64_t nz, sofia_sc_kernel kernel, double threshold,
                     int32_t noise_mode, int32_t flux_range, const uint8_t *mask_in,
                     uint8_t *mask_out, double *noise, const sofia_sc_options *opt) {
    if (!h) return SOFIA_SC_EINVAL;
    if (noise) *noise = NAN;
    if (!opt || opt->struct_size != sizeof(sofia_sc_options))
        return fail(h, SOFIA_SC_EINVAL, "options missing or of another size");
    if (opt->reserved != 0) return fail(h, SOFIA_SC_EINVAL, "reserved option field must be 0");
    return single_kernel(h, cube, nx, ny, nz, kernel, threshold, noise_mode, flux_range,
                         opt->replacement, opt->sigma0, mask_in, mask_out, noise, nullptr,
                         opt->storage, opt->stream);
}

int sofia_sc_smooth(sofia_sc *h, const float *cube, int64_t nx, int64_t ny,
                    int64_t nz, sofia_sc_kernel kernel, double replacement,
                    double sigma0, const uint8_t *mask_in, float *out,
                    void *stream) {
    if (!out) return fail(h, SOFIA_SC_EINVAL, "NULL argument");
    return single_kernel(h, cube, nx, ny, nz, kernel, 1.0, SOFIA_SC_NOISE_STD,
                         SOFIA_SC_FLUX_ALL, replacement, sigma0, mask_in, nullptr,
                         nullptr, out, SOFIA_SC_STORE_F32, stream);
}

int sofia_sc_plan(double spatial_fwhm_px, int32_t *n_iter, int32_t *radius) {
    if (!n_iter || !radius) return SOFIA_SC_EINVAL;
    return plan_cascade(spatial_fwhm_px, n_iter, radius);
}

int sofia_sc_profile(sofia_sc *h, int enable) {
    if (!h) return SOFIA_SC_EINVAL;
    h->prof = enable != 0;
    if (h->prof)
        for (auto &a : h->agg) a = Agg{};
    return SOFIA_SC_OK;
}

int sofia_sc_profile_read(const sofia_sc *h, sofia_sc_kernel_stat *stats,
                          int32_t cap, int32_t *n_out) {
    if (!h || !n_out || (cap > 0 && !stats)) return SOFIA_SC_EINVAL;
    int n = 0;
    for (int f = 0; f < F_COUNT; ++f) {
        if (h->agg[f].launches == 0) continue;
        if (n < cap) {
            sofia_sc_kernel_stat &o = stats[n];
            std::memset(&o, 0, sizeof(o));
            std::snprintf(o.name, sizeof(o.name), "%s", kFamilyName[f]);
            o.launches = h->agg[f].launches;
            o.total_ms = h->agg[f].ms;
            o.bytes = h->agg[f].bytes;
            o.voxels = h->agg[f].vox;
        }
        ++n;
    }
    *n_out = n;
    return SOFIA_SC_OK;
}

const char *sofia_sc_last_error(const sofia_sc *h) {
    return h ? h->err.c_str() : "NULL handle";
}

const char *sofia_sc_strerror(int code) {
    switch (code) {
        case SOFIA_SC_OK: return "success";
        case SOFIA_SC_EINVAL: return "invalid argument";
        case SOFIA_SC_ENOMEM: return "device allocation failed";
        case SOFIA_SC_EDEVICE: return "HIP device error";
        case SOFIA_SC_ENOSTAT: return "no voxel available for the noise measurement";
    }
    return "unknown error";
}

}  // extern "C"
