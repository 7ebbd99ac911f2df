// Host side of the smooth-and-clip library: argument checks, the spatial
// cascade plan, workspace, the per-kernel launch sequence and the C ABI
// declared in include/sofia_sc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "sc_internal.h"
#include "sofia_sc.h"

using namespace sc;

namespace {

enum Family {
    F_INIT = 0, F_FILL, F_SPATIAL, F_COL_STD, F_COL_SAMPLE, F_COL_SELECT, F_COL_HIST1,
    F_COL_HIST2, F_FALLBACK_SKIPPED, F_CAPTURE_SELECT, F_COL_CLIP, F_COL_WRITE, F_FINALIZE,
    F_QUANTIZE, F_COL_SELCLIP, F_CLIP_FIXUP, F_BATCH, F_MASK_OUT, F_NORM_NOISE, F_NORM_DIVIDE,
    F_LINK_UNION, F_LINK_NUMBER, F_LINK_LABEL, F_PARAM, F_RELIABILITY, F_SPATIAL_GAUSS,
    F_MULTI_STATS, F_MULTI_CLIP, F_MULTI_SELECT, F_COUNT
};
const char *kFamilyName[F_COUNT] = {
    "init_bits", "fill", "spatial_cascade", "column_std", "column_sample",
    "column_select", "column_hist1", "column_hist2", "fallback_skipped", "capture_select",
    "column_clip", "column_write", "finalize", "quantize", "column_select_clip",
    "clip_fixup", "batch_graph", "mask_out", "norm_window_noise", "norm_divide",
    "link_union", "link_number", "link_label", "parameterise", "reliability",
    "spatial_gauss", "fused_stats", "fused_clip", "fused_select"};

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
    int gauss_r = 0;             // sampled Gaussian of radius gauss_r (> 0) instead
    double fwhm = 0.0;
    bool spatial() const { return n_iter > 0 || gauss_r > 0; }
    bool spectral() const { return width >= 3; }
    bool identity() const { return !spatial() && !spectral(); }
};

// Device workspace of one S+C run at a time: the packed blank and detection
// bits, the smoothed plane buffer, histograms, partials, the capture and
// undecided-voxel lists and the 16-bit cube. Grown on demand, never shrunk.
// `st` is the run's device state; a batch points it at the state of the cube
// being enqueued.
struct Work {
    uint64_t *blank = nullptr;       // blank bits (non-finite voxels)
    uint64_t *det[2] = {nullptr, nullptr};   // detection bits: kernel k reads one, writes
                                             // the other
    size_t bits_cap = 0;             // words of each bit plane set
    float *p = nullptr;
    size_t p_cap = 0;
    DevState *st = nullptr;
    unsigned long long *hist = nullptr;
    double *part_sum = nullptr;
    unsigned long long *part_cnt = nullptr;
    size_t part_cap = 0;
    uint32_t *cap_buf = nullptr;
    size_t cap_cap = 0;
    uint16_t *xq = nullptr;
    size_t xq_cap = 0;
    AmbEntry *amb = nullptr;         // undecided voxels of the fused clip
    size_t amb_cap = 0;
    Shapes sh;                       // launch shapes of the runs on this workspace
};

// Lanes of a batch: cubes are spread over this many workspaces whose
// launch chains run side by side in the graph. Measured on a batch of 96
// uneven cubes: 2, 4, 8 and 16 lanes give 14.0, 16.3, 19.7 and 19.9e9
// voxels/s; 8 keeps nearly all of the gain at half the workspace of 16.
constexpr int kDefaultLanes = 8;
constexpr int kBatchLanes = 16;      // most lanes a tuning may choose

// Everything a captured batch graph depends on; an identical call replays
// the instantiated graph.
struct BatchKey {
    std::vector<sofia_sc_cube> cubes;
    std::vector<sofia_sc_kernel> kernels;
    double t = 0, repl = 0;
    uint64_t sigma0_bits = 0;
    int mode = 0, range = 0, storage = 0;
    int keep = 0;                    // keep_input_mask: changes the captured launches
    int zstride = 1;                 // noise plane stride
    int lanes = 0, col_blocks = 0, strip_rows = 0, strip_waves = 0, col_min_planes = 0;
    uint64_t work_gen = 0;
};

sofia_sc_batch_tuning default_tuning() {
    const Shapes d;
    sofia_sc_batch_tuning t;
    std::memset(&t, 0, sizeof(t));
    t.lanes = kDefaultLanes;
    t.col_blocks = d.col_blocks;
    t.strip_rows = d.strip_rows;
    t.strip_waves = d.strip_waves;
    t.col_min_planes = d.col_min_planes;
    t.ms = NAN;
    return t;
}

Shapes shapes_of(const sofia_sc_batch_tuning &t) {
    Shapes s;
    s.col_blocks = t.col_blocks;
    s.strip_rows = t.strip_rows;
    s.strip_waves = t.strip_waves;
    s.col_min_planes = t.col_min_planes;
    return s;
}

}  // namespace

struct sofia_sc {
    int device = 0;
    long allocs = 0;                 // device / pinned allocations attempted so far
    char err[512] = {0};             // last error text (fixed: setting it allocates nothing)
    bool noalloc_call = false;       // inside sofia_sc_run_noalloc: no profiling events
    Work w;                          // workspace of run / step / smooth
    DevState *st_host = nullptr;     // pinned
    bool prof = false;
    std::vector<LaunchRec> recs;
    std::vector<hipEvent_t> pool;
    Agg agg[F_COUNT];
    // batch
    Work lanes[kBatchLanes];
    hipStream_t lane_s[kBatchLanes] = {};
    hipEvent_t fork_ev = nullptr, join_ev[kBatchLanes] = {};
    DevState *bst = nullptr;         // per-cube device states
    DevState *bst_host = nullptr;    // pinned copy
    size_t bst_cap = 0;
    uint64_t work_gen = 0;           // bumped whenever a lane workspace moves
    hipGraphExec_t gexec = nullptr;
    BatchKey gkey;
    bool gvalid = false;
    double graph_bytes = 0;          // algorithmic bytes of the captured launches
    bool capturing = false;          // launches are being captured: no events
    double capture_bytes = 0;
    sofia_sc_batch_tuning tune = default_tuning();
    double *nn_sigma = nullptr;      // noise grid of the local noise normalisation
    size_t nn_cap = 0;
    // linker workspace: block counts, per-detection boxes and labels, output boxes
    int *lk_counts = nullptr;
    size_t lk_counts_cap = 0;
    int *lk_list = nullptr;          // the detected voxels of a linked mask
    size_t lk_list_cap = 0;
    int *lk_box = nullptr;
    size_t lk_box_cap = 0;
    int *lk_label = nullptr;
    size_t lk_label_cap = 0;
    int *lk_kcounts = nullptr;
    size_t lk_kcounts_cap = 0;
    long long *lk_out = nullptr;
    size_t lk_out_cap = 0;
    // parameterisation workspace: accumulators, signs, parameter vectors,
    // reliability state (inverse covariance, flag, kept count)
    SrcAcc *pm_acc = nullptr;
    size_t pm_acc_cap = 0;
    int *pm_sign = nullptr;
    size_t pm_sign_cap = 0;
    double *pm_vec = nullptr;
    size_t pm_vec_cap = 0;
    double *pm_state = nullptr;
    size_t pm_state_cap = 0;
    // partials of the fused spectral-widths passes
    double *mu_sum = nullptr;
    size_t mu_sum_cap = 0;
    unsigned long long *mu_cnt = nullptr;
    size_t mu_cnt_cap = 0;
    // fused MAD: per-width states, histograms (+ capture counts), capture
    // lists and selection counts
    DevState *mu_st = nullptr;
    size_t mu_st_cap = 0;
    unsigned long long *mu_hist = nullptr;
    size_t mu_hist_cap = 0;
    uint32_t *mu_cap = nullptr;
    size_t mu_cap_cap = 0;
    unsigned long long *mu_sel = nullptr;
    size_t mu_sel_cap = 0;
};

namespace {

// Histogram workspace, zeroed before every MAD measurement: level 1 |
// level-2 coarse | level 2 | sampled level 1 | capture count | count of
// voxels the fused clip left undecided.
constexpr size_t kOffL2c = kL1Bins;
constexpr size_t kOffL2 = kOffL2c + 2 * (size_t)kL2Coarse;
constexpr size_t kOffSample = kOffL2 + 2 * (size_t)kL2Bins;
constexpr size_t kOffCapCount = kOffSample + kL1Bins;
constexpr size_t kOffAmbCount = kOffCapCount + 2;
constexpr size_t kHistWords = kOffAmbCount + 2;
// 64-column segments visited by the sampling pass: every 17th (a stride
// coprime to the usual row lengths in segments spreads the sample over x and
// y); planes of more than 17 x 512 segments use a wider odd stride.
constexpr int kSampleStride = 17;

unsigned long long *hist1_of(const Work &w) { return w.hist; }
unsigned long long *hist2c_of(const Work &w) { return w.hist + kOffL2c; }
unsigned long long *hist2_of(const Work &w) { return w.hist + kOffL2; }
unsigned long long *hist_s_of(const Work &w) { return w.hist + kOffSample; }
unsigned long long *cap_count_of(const Work &w) { return w.hist + kOffCapCount; }
unsigned long long *amb_count_of(const Work &w) { return w.hist + kOffAmbCount; }

// Undecided-voxel list of the fused clip: up to N/256 entries (at least
// 2^16); beyond that the plain clip pass runs.
size_t amb_capacity(int64_t N) { return std::max<size_t>((size_t)N / 256, (size_t)1 << 16); }

// Capture buffer: up to N/8 keys (at least 2^20).
size_t capture_capacity(int64_t N) { return std::max<size_t>((size_t)N / 8, (size_t)1 << 20); }

int fail(sofia_sc *h, int code, const char *msg) {
    if (h) std::snprintf(h->err, sizeof(h->err), "%s", msg);
    return code;
}

int fail(sofia_sc *h, int code, const std::string &msg) { return fail(h, code, msg.c_str()); }

int hip_fail(sofia_sc *h, hipError_t e, const char *what) {
    if (h) std::snprintf(h->err, sizeof(h->err), "%s: %s", what, hipGetErrorString(e));
    return SOFIA_SC_EDEVICE;
}

// Diagnostics hooks, set in the environment:
//  SOFIA_SC_TRACE=1       one line per run, batch capture / launch and tuning
//                         candidate on stderr;
//  SOFIA_SC_FAIL_ALLOC=k  the k-th device or pinned allocation a handle
//                         attempts (counting from 1) fails as out of memory,
//                         so that tests reach every ENOMEM path.
bool trace_on() {
    const char *v = std::getenv("SOFIA_SC_TRACE");
    return v && *v && *v != '0';
}

#define SC_TRACE(...)                                   \
    do {                                                \
        if (trace_on()) {                               \
            std::fprintf(stderr, "[sofia_sc] " __VA_ARGS__); \
            std::fputc('\n', stderr);                   \
        }                                               \
    } while (0)

bool injected_alloc_failure(sofia_sc *h) {
    const long n = ++h->allocs;
    const char *v = std::getenv("SOFIA_SC_FAIL_ALLOC");
    return v && *v && std::atol(v) == n;
}

hipError_t dev_alloc(sofia_sc *h, void **p, size_t bytes) {
    if (injected_alloc_failure(h)) return hipErrorOutOfMemory;
    return hipMalloc(p, bytes);
}

hipError_t host_alloc(sofia_sc *h, void **p, size_t bytes) {
    if (injected_alloc_failure(h)) return hipErrorOutOfMemory;
    return hipHostMalloc(p, bytes, hipHostMallocDefault);
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
    if (k.spatial_kind != SOFIA_SC_SPATIAL_CASCADE && k.spatial_kind != SOFIA_SC_SPATIAL_GAUSS)
        return fail(h, SOFIA_SC_EINVAL, "spatial_kind must be 0 (cascade) or 1 (Gaussian)");
    p->gauss_r = 0;
    p->fwhm = k.spatial_fwhm_px;
    if (k.spatial_kind == SOFIA_SC_SPATIAL_GAUSS) {
        n = r = 0;
        if (k.spatial_fwhm_px > 0.0) p->gauss_r = gauss_radius(k.spatial_fwhm_px);
        if (p->gauss_r > kGaussMaxR)
            return fail(h, SOFIA_SC_EINVAL,
                        "spatial FWHM too large (Gaussian radius above SOFIA_SC_GAUSS_MAX_RADIUS)");
    } else if (n * r > SOFIA_SC_MAX_HALO) {
        return fail(h, SOFIA_SC_EINVAL, "spatial FWHM too large (cascade halo above limit)");
    }
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
    // the spatial kernel addresses a plane with 32-bit byte offsets
    if (nx * ny > SOFIA_SC_MAX_PLANE)
        return fail(h, SOFIA_SC_EINVAL, "plane larger than 2^28 voxels");
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

// Column-kernel grid: 256 columns per block; z is split as far as needed to
// give the chip several waves of blocks, and so that no block streams more
// than kColMaxZChunk planes: the four blocks that share a cache line of the
// bit planes start together but drift apart in z as they stream, and over
// thousands of planes the line leaves their L2 before the last of them reads
// it.
constexpr int64_t kColMaxZChunk = 1024;
struct ColGrid {
    int ncb, nzc, zchunk;
    int blocks() const { return ncb * nzc; }
};

ColGrid col_grid(int64_t ncol, int64_t nz, const Shapes &sh) {
    ColGrid g;
    g.ncb = (int)((ncol + kColThreads - 1) / kColThreads);
    int64_t nzc = (sh.col_blocks + g.ncb - 1) / g.ncb;
    const int64_t max_nzc = std::max<int64_t>(1, nz / std::max(1, sh.col_min_planes));
    nzc = std::max<int64_t>(1, std::min(nzc, max_nzc));
    nzc = std::max<int64_t>(nzc, (nz + kColMaxZChunk - 1) / kColMaxZChunk);
    g.zchunk = (int)((nz + nzc - 1) / nzc);
    g.nzc = (int)((nz + g.zchunk - 1) / g.zchunk);
    return g;
}

// Destroy the cached batch graph (it is captured again when next needed).
void drop_graph(sofia_sc *h) {
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
    h->gvalid = false;
}

// Grow a device buffer to at least `need` elements (contents are not kept).
// moved != null marks a batch lane's buffer: the cached batch graph may hold
// it in its kernel arguments, so the graph is destroyed before the buffer is
// freed, never after.
template <typename T>
int grow(sofia_sc *h, T *&ptr, size_t &cap, size_t need, const char *what, bool *moved) {
    if (need <= cap) return SOFIA_SC_OK;
    if (ptr) {
        if (moved) drop_graph(h);
        (void)hipFree(ptr);
    }
    ptr = nullptr;
    cap = 0;
    const hipError_t e = dev_alloc(h, (void **)&ptr, need * sizeof(T));
    if (e != hipSuccess) {
        ptr = nullptr;
        SC_TRACE("allocation of %zu bytes (%s) failed: %s", need * sizeof(T), what,
                 hipGetErrorString(e));
    }
    if (e != hipSuccess)
        return fail(h, SOFIA_SC_ENOMEM, std::string(what) + ": " + hipGetErrorString(e));
    cap = need;
    if (moved) *moved = true;
    return SOFIA_SC_OK;
}

struct Dims {
    int64_t nx, ny, nz, ncol, N;
};

// Packed bits: words per plane of nx * ny voxels, and per cube.
int64_t det_words_per_plane(int64_t ncol) { return (ncol + 63) / 64; }
int64_t bit_words(const Dims &d) { return d.nz * det_words_per_plane(d.ncol); }

// Workspace for cubes of up to N voxels (bit planes of `words` words):
// `parts` column blocks, the smoothed-plane buffer when a kernel is spatial
// and a 16-bit cube when q16. *moved is set when any buffer was reallocated.
int ensure_work(sofia_sc *h, Work &w, int64_t N, int64_t words, bool need_p, size_t parts,
                bool q16, bool *moved = nullptr) {
    int rc;
    size_t one = w.hist ? kHistWords : 0;
    if ((rc = grow(h, w.hist, one, kHistWords, "histograms", moved))) return rc;
    uint64_t **bits[3] = {&w.blank, &w.det[0], &w.det[1]};
    for (int i = 0; i < 3; ++i) {
        size_t cap = w.bits_cap;
        if ((rc = grow(h, *bits[i], cap, (size_t)words, "bit planes", moved))) return rc;
    }
    w.bits_cap = std::max(w.bits_cap, (size_t)words);
    if (need_p && (rc = grow(h, w.p, w.p_cap, (size_t)N, "plane buffer", moved))) return rc;
    if ((rc = grow(h, w.amb, w.amb_cap, amb_capacity(N), "undecided list", moved))) return rc;
    if ((rc = grow(h, w.cap_buf, w.cap_cap, capture_capacity(N), "capture buffer", moved)))
        return rc;
    // partial sums: one per block; partial counts: two per block (the
    // selection pass keeps two counts)
    size_t pc = w.part_cap, pc2 = 2 * w.part_cap;
    if ((rc = grow(h, w.part_sum, pc, parts, "partials", moved))) return rc;
    if ((rc = grow(h, w.part_cnt, pc2, 2 * parts, "partials", moved))) return rc;
    w.part_cap = std::max(w.part_cap, parts);
    if (q16 && (rc = grow(h, w.xq, w.xq_cap, (size_t)N, "16-bit cube", moved))) return rc;
    return SOFIA_SC_OK;
}

void free_work(Work &w) {
    void *ps[] = {w.blank, w.det[0], w.det[1], w.p, w.st, w.hist, w.part_sum, w.part_cnt,
                  w.cap_buf, w.xq, w.amb};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    w = Work{};
}

// The handle's own device state and its pinned host copy.
int ensure_state(sofia_sc *h) {
    hipError_t e;
    if (!h->w.st && (e = dev_alloc(h, (void **)&h->w.st, sizeof(DevState))) != hipSuccess) {
        h->w.st = nullptr;
        return fail(h, SOFIA_SC_ENOMEM, std::string("state: ") + hipGetErrorString(e));
    }
    if (!h->st_host && (e = host_alloc(h, (void **)&h->st_host, sizeof(DevState))) != hipSuccess) {
        h->st_host = nullptr;
        return fail(h, SOFIA_SC_ENOMEM, std::string("host state: ") + hipGetErrorString(e));
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
    if (h->capturing) {
        // inside a graph capture: no per-launch events; the algorithmic bytes
        // of the launches that always work are summed for the whole graph
        if (cond < 0) h->capture_bytes += bytes;
        const hipError_t e = f();
        return e == hipSuccess ? SOFIA_SC_OK : hip_fail(h, e, kFamilyName[fam]);
    }
    if (h->prof && !h->noalloc_call) {
        e0 = take_event(h);
        e1 = take_event(h);
        if (e0) (void)hipEventRecord(e0, s);
    }
    const hipError_t e = f();
    if (e != hipSuccess) return hip_fail(h, e, kFamilyName[fam]);
    if (h->prof && !h->noalloc_call && e0 && e1) {
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

// One S+C iteration on the device. k >= 0 stores sigma_k; k = -1 measures
// sigma_0 only. det_in: the detections so far (null: none yet); blank_in:
// the blank bits (needed when the kernel is spatial). det_out = null skips
// the clip; otherwise the clip writes det_in | this kernel's detections
// there, and blank_out (may be null) receives the blank bits of a pass over
// the raw cube. write_out != null writes s instead of measuring the noise.
struct PairJob {
    const float *x = nullptr;
    const uint16_t *xq = nullptr;   // 16-bit noise-scaled cube (xtype != ST_F32)
    int xtype = ST_F32;
    Dims d{};
    Plan pl{0, 0, 1};
    int k = 0;
    bool repl_active = false;
    double repl_n = 0.0;
    int mode = 0, range = 0;
    double t = 0.0;
    const uint64_t *det_in = nullptr;
    const uint64_t *blank_in = nullptr;
    uint64_t *det_out = nullptr;
    uint64_t *blank_out = nullptr;
    bool also_sigma0 = false;
    float *write_out = nullptr;
    int zstride = 1;        // the noise is measured on every zstride-th plane
};

// The spatial pass of a kernel pair: the raw cube (with replacement and
// blanking) smoothed spatially into w.p.
int spatial_pass(sofia_sc *h, hipStream_t s, const Work &w, const PairJob &j) {
    const Dims &d = j.d;
    const double N = (double)d.N;
    const double bx = j.xtype != ST_F32 ? 2.0 : 4.0;   // bytes per raw voxel
    int rc;
    if (j.pl.gauss_r > 0) {
        GaussArgs a{};
        a.x = j.xtype == ST_F32 ? j.x : nullptr;
        a.xq = j.xtype != ST_F32 ? j.xq : nullptr;
        a.wpp = det_words_per_plane(d.ncol);
        a.det = j.repl_active ? j.det_in : nullptr;
        a.p = w.p;
        a.nx = d.nx; a.ny = d.ny; a.nz = d.nz;
        gauss_setup(a, j.pl.fwhm, w.sh.strip_rows);
        if (a.tiles > 0x7fffffffLL)
            return fail(h, SOFIA_SC_EINVAL, "cube too large for the spatial grid");
        a.repl_n = j.repl_n;
        a.st = w.st;
        const double bytes = N * (bx + (j.repl_active ? 0.125 : 0.0) + 4.0);
        rc = launch(h, s, F_SPATIAL_GAUSS, bytes, N, [&] {
            return launch_gauss(j.pl.gauss_r, j.xtype, j.repl_active, a, s);
        });
        if (rc) return rc;
    } else {
        StripArgs a{};
        a.x = j.xtype == ST_F32 ? j.x : nullptr;
        a.xq = j.xtype != ST_F32 ? j.xq : nullptr;
        a.wpp = det_words_per_plane(d.ncol);
        a.det = j.repl_active ? j.det_in : nullptr;
        a.p = w.p;
        a.nx = d.nx; a.ny = d.ny; a.nz = d.nz;
        spatial_strips(a, j.pl.n_iter, j.pl.radius, w.sh.strip_rows, w.sh.strip_waves);
        if (a.tiles > 0x7fffffffLL)
            return fail(h, SOFIA_SC_EINVAL, "cube too large for the spatial grid");
        a.repl_n = j.repl_n;
        a.st = w.st;
        // raw cube in, smoothed plane out, and with replacement the packed
        // detection bits (one bit per voxel)
        const double bytes = N * (bx + (j.repl_active ? 0.125 : 0.0) + 4.0);
        rc = launch(h, s, F_SPATIAL, bytes, N, [&] {
            return launch_spatial(j.pl.n_iter, j.pl.radius, j.xtype, j.repl_active, a, s);
        });
        if (rc) return rc;
    }

    return SOFIA_SC_OK;
}

int run_pair(sofia_sc *h, hipStream_t s, const Work &w, const PairJob &j) {
    const Dims &d = j.d;
    const double N = (double)d.N;
    int rc;
    const bool spatial = j.pl.spatial();
    const bool spec = j.pl.spectral();
    const double bx = j.xtype != ST_F32 ? 2.0 : 4.0;   // bytes per raw voxel
    if ((spatial && !j.blank_in) || (j.repl_active && !j.det_in))
        return fail(h, SOFIA_SC_EINVAL, "internal: bit planes missing");

    const ColGrid g = col_grid(d.ncol, d.nz, w.sh);
    if ((int64_t)g.ncb * g.nzc > 0x7fffffffLL)
        return fail(h, SOFIA_SC_EINVAL, "cube too large for the column grid");
    if (spatial && (rc = spatial_pass(h, s, w, j))) return rc;

    ColArgs c{};
    c.x = j.x;
    c.xq = j.xq;
    c.xtype = j.xtype;
    c.p = w.p;
    c.det_in = j.det_in;
    c.blank_in = spatial ? j.blank_in : nullptr;
    c.wpp = det_words_per_plane(d.ncol);
    c.ncol = d.ncol;
    c.nz = d.nz;
    c.w = j.pl.width;
    c.h = (j.pl.width - 1) / 2;
    c.zchunk = g.zchunk;
    c.ncb = g.ncb;
    c.range = j.range;
    c.repl_on = (!spatial && j.repl_active) ? 1 : 0;
    c.repl_n = j.repl_n;
    c.st = w.st;
    c.part_sum = w.part_sum;
    c.part_cnt = w.part_cnt;
    c.hist1 = hist1_of(w);
    c.hist2 = hist2_of(w);
    c.hist2c = hist2c_of(w);
    c.cb_stride = 1;
    c.zstride = j.zstride;
    c.cap_buf = w.cap_buf;
    c.cap_count = cap_count_of(w);
    c.cap_capacity = (unsigned long long)w.cap_cap;
    c.sel_part = w.part_cnt;
    const int src = spatial ? SRC_P : SRC_X;
    // algorithmic bytes of a pass: the source and the bit planes it reads
    const double rd = N * ((spatial ? 4.0 : bx) + (j.det_in ? 0.125 : 0.0) +
                           (spatial ? 0.125 : 0.0));
    auto col = [&](int op, int fam, double bytes) {
        return launch(h, s, fam, bytes, N, [&] {
            return launch_column(src, op, spec, c, g.blocks(), s);
        });
    };

    if (j.write_out) {
        c.s_out = j.write_out;
        return col(OP_WRITE, F_COL_WRITE, rd + 4.0 * N);
    }

    // Clip target: the detection bits after this kernel (and the blank bits
    // when this pass is the first over the raw cube).
    double clip_bytes = 0.0;
    if (j.det_out) {
        c.det_out = j.det_out;
        c.blank_out = spatial ? nullptr : j.blank_out;
        clip_bytes = N / 8.0 + (c.blank_out ? N / 8.0 : 0.0);
    }
    const int cond = j.k >= 0 ? j.k : 63;
    // With MAD noise the clip rides on the selection pass (see below).
    const bool fused = j.det_out && j.mode != SOFIA_SC_NOISE_STD;

    if (j.mode == SOFIA_SC_NOISE_STD) {
        if ((rc = col(OP_STD, F_COL_STD, rd))) return rc;
        rc = launch(h, s, F_FINALIZE, 16.0 * g.blocks(), 0, [&] {
            return launch_finalize_std(w.st, w.part_sum, w.part_cnt, g.blocks(),
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
            return launch_fill_u64(w.hist, (int64_t)kHistWords, s);
        });
        if (rc) return rc;
        {
            // The sample touches 1/17 of the columns: split z finer so the
            // launch still has a few blocks per CU.
            ColArgs cs = c;
            const int64_t nseg = (d.ncol + 63) / 64;   // 64-column segments
            // every 17th segment; on large planes an odd stride that still
            // samples about 512 segments per plane
            const int64_t stride =
                nseg >= (int64_t)kSampleStride * 512 ? (nseg / 512) | 1 : kSampleStride;
            cs.cb_stride = (int)stride;
            const int64_t sampled = (nseg + stride - 1) / stride;
            cs.ncb = (int)((sampled + kColThreads / 64 - 1) / (kColThreads / 64));
            cs.hist1 = hist_s_of(w);
            int nzc = (int)std::min<int64_t>((2048 + cs.ncb - 1) / cs.ncb,
                                             std::max<int64_t>(1, d.nz / 32));
            nzc = std::max(nzc, 1);
            cs.zchunk = (int)((d.nz + nzc - 1) / nzc);
            nzc = (int)((d.nz + cs.zchunk - 1) / cs.zchunk);
            const int nb = cs.ncb * nzc;
            const double frac = (double)sampled / (double)nseg;
            rc = launch(h, s, F_COL_SAMPLE, rd * frac, N * frac, [&] {
                return launch_column(src, OP_HIST1, spec, cs, nb, s);
            });
            if (rc) return rc;
        }
        rc = launch(h, s, F_FINALIZE, 8.0 * kL1Bins, 0, [&] {
            return launch_finalize_predict(w.st, hist_s_of(w), j.t, s);
        });
        if (rc) return rc;
        // Fused clip: the predicted median window bounds the threshold, so
        // the selection pass also clips every voxel whose |s| lies outside
        // (thr_lo, thr_hi] and lists the others for an exact decision later.
        if (fused) {
            c.amb = w.amb;
            c.amb_count = amb_count_of(w);
            c.amb_capacity = (unsigned long long)w.amb_cap;
            if ((rc = col(OP_SELCLIP, F_COL_SELCLIP, rd + clip_bytes))) return rc;
        } else {
            if ((rc = col(OP_SELECT, F_COL_SELECT, rd))) return rc;
        }
        // Walk grids sized to the keys a cube of this size captures (about
        // 1 % of its voxels): a block clears and flushes a whole LDS
        // histogram, which dominates when it has only a few keys to count.
        const int wb2 = (int)std::min<int64_t>(1024, std::max<int64_t>(8, d.N >> 18));
        const int wb1 = std::min(512, wb2);
        rc = launch(h, s, F_FINALIZE, 0, 0, [&] {
            return launch_finalize_select(w.st, w.part_cnt, g.blocks(), cap_count_of(w),
                                          (unsigned long long)w.cap_cap, j.k,
                                          fused ? amb_count_of(w) : nullptr,
                                          (unsigned long long)w.amb_cap, s);
        });
        if (rc) return rc;
        rc = launch(h, s, F_CAPTURE_SELECT, 0, 0, [&] {
            return launch_capture_l1(w.st, w.cap_buf, cap_count_of(w), hist1_of(w),
                                     wb1, s);
        });
        if (rc) return rc;
        c.skip_if_captured = 1;
        rc = launch(h, s, F_COL_HIST1, rd, N, [&] {
            return launch_column(src, OP_HIST1, spec, c, g.blocks(), s);
        }, cond);
        if (rc) return rc;
        rc = launch(h, s, F_FINALIZE, 8.0 * kL1Bins, 0, [&] {
            return launch_finalize_mad1(w.st, hist1_of(w), s);
        });
        if (rc) return rc;
        rc = launch(h, s, F_CAPTURE_SELECT, 0, 0, [&] {
            return launch_capture_coarse(w.st, w.cap_buf, cap_count_of(w), hist2c_of(w),
                                     wb2, s);
        });
        if (rc) return rc;
        rc = launch(h, s, F_COL_HIST2, rd, N, [&] {
            return launch_column(src, OP_HIST2, spec, c, g.blocks(), s);
        }, cond);
        c.skip_if_captured = 0;
        if (rc) return rc;
        rc = launch(h, s, F_FINALIZE, 8.0 * 2 * kL2Coarse, 0, [&] {
            return launch_finalize_mad2a(w.st, hist2c_of(w), s);
        });
        if (rc) return rc;
        rc = launch(h, s, F_CAPTURE_SELECT, 0, 0, [&] {
            return launch_capture_fine(w.st, w.cap_buf, cap_count_of(w), hist2_of(w),
                                     wb2, s);
        });
        if (rc) return rc;
        rc = launch(h, s, F_FINALIZE, 8.0 * 2 * kL2Fine, 0, [&] {
            return launch_finalize_mad2b(w.st, hist2_of(w), j.k, j.t,
                                         j.also_sigma0 ? 1 : 0, s);
        });
        if (rc) return rc;
    }
    if (fused) {
        // decide the listed voxels; the full clip pass below runs only when
        // the median missed the window or the list overflowed
        rc = launch(h, s, F_CLIP_FIXUP, 0, 0, [&] {
            return launch_clip_fixup(w.st, w.amb, amb_count_of(w),
                                     (unsigned long long)w.amb_cap, c.det_out, d.ncol, c.wpp,
                                     s);
        });
        if (rc) return rc;
        c.skip_if_fused = 1;
        rc = launch(h, s, F_COL_CLIP, rd + clip_bytes, N, [&] {
            return launch_column(src, OP_CLIP, spec, c, g.blocks(), s);
        }, 64 + cond);
        c.skip_if_fused = 0;
        if (rc) return rc;
    } else if (j.det_out) {
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

// Copy n device states to the host and wait for the stream.
int finish(sofia_sc *h, hipStream_t s, DevState *host, const DevState *dev, size_t n = 1) {
    hipError_t e = hipMemcpyAsync(host, dev, n * sizeof(DevState), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(h, e, "copy of noise values");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(h, e, "stream");
    if (h->prof) collect_profile(h);
    return SOFIA_SC_OK;
}

void nan_fill(double *v, int n) {
    if (v)
        for (int i = 0; i < n; ++i) v[i] = NAN;
}

// A validated whole run: one cube, its kernel plans and options.
struct RunSpec {
    const float *cube;
    Dims d;
    const Plan *plans;
    int K;
    double t;
    int mode, range;
    uint8_t *mask;
    double repl;          // < 0: no replacement
    double sigma0;        // NaN: measure
    int storage;
    bool keep;            // OR the detections into the caller's mask
    int zstride = 1;      // noise measured on every zstride-th plane
    bool any_spatial() const {
        for (int k = 0; k < K; ++k)
            if (plans[k].spatial()) return true;
        return false;
    }
};

int check_options(sofia_sc *h, const sofia_sc_options *opt) {
    if (!opt || opt->struct_size != sizeof(sofia_sc_options))
        return fail(h, SOFIA_SC_EINVAL, "options missing or struct_size mismatch");
    if (std::isnan(opt->replacement) || opt->replacement == INFINITY)
        return fail(h, SOFIA_SC_EINVAL, "replacement must be finite");
    const int storage = opt->storage;
    if (storage != SOFIA_SC_STORE_F32 && storage != SOFIA_SC_STORE_F16 &&
        storage != SOFIA_SC_STORE_BF16)
        return fail(h, SOFIA_SC_EINVAL, "unknown storage");
    if (opt->keep_input_mask != 0 && opt->keep_input_mask != 1)
        return fail(h, SOFIA_SC_EINVAL, "keep_input_mask must be 0 or 1");
    if (!std::isnan(opt->sigma0) && !(std::isfinite(opt->sigma0) && opt->sigma0 > 0.0))
        return fail(h, SOFIA_SC_EINVAL, "sigma0 must be NaN (measure) or finite and > 0");
    if (opt->noise_plane_stride < 0 || opt->noise_plane_stride > (1 << 30))
        return fail(h, SOFIA_SC_EINVAL, "noise_plane_stride must be 0..2^30");
    if (opt->fuse_widths != 0 && opt->fuse_widths != 1)
        return fail(h, SOFIA_SC_EINVAL, "fuse_widths must be 0 or 1");
    return SOFIA_SC_OK;
}

// Planes the noise is measured on: every plane_stride(opt)-th (0 and 1: all).
int plane_stride(const sofia_sc_options *opt) {
    return opt->noise_plane_stride > 1 ? opt->noise_plane_stride : 1;
}

// Workspace a run of this cube and kernel list needs.
int ensure_for(sofia_sc *h, Work &w, const RunSpec &r, bool *moved = nullptr) {
    const bool sp = r.any_spatial();
    const ColGrid g = col_grid(r.d.ncol, r.d.nz, w.sh);
    return ensure_work(h, w, r.d.N, bit_words(r.d), sp, (size_t)g.blocks(),
                       r.storage != SOFIA_SC_STORE_F32, moved);
}

// Enqueue a whole S+C run (Sect. 4.2) on stream s, with workspace w and the
// run's state w.st. Makes no host round trip: every later launch reads what
// it needs from the device state.
int enqueue_run(sofia_sc *h, hipStream_t s, const Work &w, const RunSpec &r) {
    int rc;
    const Dims &d = r.d;
    const int K = r.K;
    const bool given0 = !std::isnan(r.sigma0);
    const bool q16 = r.storage != SOFIA_SC_STORE_F32;
    const bool any_spatial = r.any_spatial();
    const bool repl_on = r.repl >= 0.0;
    const bool first_identity = r.plans[0].identity();
    const int64_t wpp = det_words_per_plane(d.ncol);
    rc = launch(h, s, F_FINALIZE, 0, 0, [&] {
        return launch_set_sigma0(w.st, given0 ? r.sigma0 : NAN, s);
    });
    if (rc) return rc;
    // The blank bits are read by the passes over a spatially smoothed cube.
    // An unsmoothed first kernel records them in its clip; otherwise one
    // pass over the cube does.
    if (any_spatial && !first_identity) {
        rc = launch(h, s, F_INIT, 4.125 * d.N, (double)d.N, [&] {
            return launch_init_bits(r.cube, nullptr, w.blank, nullptr, d.ncol, d.nz, wpp, s);
        });
        if (rc) return rc;
    }
    // sigma_0 on the FP32 cube when replacement or 16-bit scaling needs it and
    // it cannot come from kernel 1 (a (0, 0) kernel measured on FP32 data).
    if (!given0 && (q16 || (repl_on && !first_identity))) {
        PairJob j;
        j.x = r.cube;
        j.d = d;
        j.k = -1;
        j.mode = r.mode;
        j.range = r.range;
        j.t = r.t;
        j.zstride = r.zstride;
        if ((rc = run_pair(h, s, w, j))) return rc;
    }
    int xtype = ST_F32;
    if (q16) {
        xtype = r.storage == SOFIA_SC_STORE_F16 ? ST_F16 : ST_BF16;
        rc = launch(h, s, F_QUANTIZE, 6.0 * d.N, (double)d.N, [&] {
            return launch_quantize(r.cube, w.st, 0.0, xtype, w.xq, d.N, s);
        });
        if (rc) return rc;
        rc = launch(h, s, F_FINALIZE, 0, 0, [&] { return launch_enter_scaled(w.st, s); });
        if (rc) return rc;
    }
    // kernel k reads the detections of kernels 0 .. k-1 from one bit plane
    // set and writes its own ORed in to the other
    const uint64_t *din = nullptr;
    for (int k = 0; k < K; ++k) {
        PairJob j;
        j.x = r.cube;
        j.xq = q16 ? w.xq : nullptr;
        j.xtype = xtype;
        j.d = d;
        j.pl = r.plans[k];
        j.k = k;
        j.repl_active = repl_on && k >= 1;
        j.repl_n = r.repl;
        j.mode = r.mode;
        j.range = r.range;
        j.t = r.t;
        j.det_in = din;
        j.blank_in = w.blank;
        j.det_out = w.det[k & 1];
        j.blank_out = k == 0 && first_identity && any_spatial ? w.blank : nullptr;
        j.also_sigma0 = k == 0 && first_identity && repl_on && !given0 && !q16;
        j.zstride = r.zstride;
        if ((rc = run_pair(h, s, w, j))) return rc;
        din = j.det_out;
    }
    // the caller's 0/1 mask from the final detection bits (ORed into it when
    // the caller's mask is kept)
    return launch(h, s, F_MASK_OUT, 0.125 * d.N + (r.keep ? 2.0 : 1.0) * d.N, (double)d.N,
                  [&] { return launch_write_mask(din, r.mask, r.keep ? 1 : 0, nullptr, d.ncol,
                                                 d.nz, wpp, s); });
}

// MAD noise of the widths of one fused chunk: per width its own state,
// histograms and capture list; the sample passes and the exact selection
// from the captured keys (or the full histogram passes when the capture
// misses) as for one pair, but one shared selection pass for every width.
int fused_mad_noise(sofia_sc *h, hipStream_t s, const Work &w, const RunSpec &r,
                    const ColGrid &g, MultiArgs &m, bool spatial, double in_b) {
    int rc;
    const Dims &d = r.d;
    const double N = (double)d.N;
    const size_t capcap = capture_capacity(d.N);
    const size_t nparts = (size_t)g.blocks();
    if ((rc = grow(h, h->mu_st, h->mu_st_cap, (size_t)kMultiMax, "fused states", nullptr)) ||
        (rc = grow(h, h->mu_hist, h->mu_hist_cap, kHistWords * kMultiMax, "fused histograms",
                   nullptr)) ||
        (rc = grow(h, h->mu_cap, h->mu_cap_cap, capcap * kMultiMax, "fused capture lists",
                   nullptr)) ||
        (rc = grow(h, h->mu_sel, h->mu_sel_cap, 2 * nparts * kMultiMax, "fused counts",
                   nullptr)))
        return rc;
    const int src = spatial ? SRC_P : SRC_X;
    const int wb2 = (int)std::min<int64_t>(1024, std::max<int64_t>(8, d.N >> 18));
    const int wb1 = std::min(512, wb2);
    m.cap_capacity = (unsigned long long)capcap;
    auto hist_of = [&](int i) { return h->mu_hist + (size_t)i * kHistWords; };
    // ColArgs of width i (sample pass and the full histogram passes)
    auto col_args = [&](int i) {
        ColArgs c{};
        c.x = r.cube;
        c.p = w.p;
        c.xtype = ST_F32;
        c.blank_in = spatial ? w.blank : nullptr;
        c.wpp = det_words_per_plane(d.ncol);
        c.ncol = d.ncol;
        c.nz = d.nz;
        c.w = m.w[i];
        c.h = m.h[i];
        c.zchunk = g.zchunk;
        c.ncb = g.ncb;
        c.range = r.range;
        c.st = m.sti[i];
        c.hist1 = hist_of(i);
        c.hist2 = hist_of(i) + kOffL2;
        c.hist2c = hist_of(i) + kOffL2c;
        c.cb_stride = 1;
        c.zstride = r.zstride;
        return c;
    };
    for (int i = 0; i < m.nw; ++i) {
        m.sti[i] = h->mu_st + i;
        m.cap[i] = h->mu_cap + (size_t)i * capcap;
        m.cap_count[i] = hist_of(i) + kOffCapCount;
        m.sel_part[i] = h->mu_sel + (size_t)i * 2 * nparts;
        DevState *sti = m.sti[i];
        unsigned long long *hi = hist_of(i);
        rc = launch(h, s, F_FINALIZE, 0, 0, [&] { return launch_set_sigma0(sti, NAN, s); });
        if (!rc) rc = launch(h, s, F_FILL, 8.0 * kHistWords, 0, [&] {
            return launch_fill_u64(hi, (int64_t)kHistWords, s);
        });
        if (rc) return rc;
        // the sample pass of width i, as for one pair
        ColArgs cs = col_args(i);
        const int64_t nseg = (d.ncol + 63) / 64;
        const int64_t stride =
            nseg >= (int64_t)kSampleStride * 512 ? (nseg / 512) | 1 : kSampleStride;
        cs.cb_stride = (int)stride;
        const int64_t sampled = (nseg + stride - 1) / stride;
        cs.ncb = (int)((sampled + kColThreads / 64 - 1) / (kColThreads / 64));
        cs.hist1 = hi + kOffSample;
        int nzc = (int)std::min<int64_t>((2048 + cs.ncb - 1) / cs.ncb,
                                         std::max<int64_t>(1, d.nz / 32));
        nzc = std::max(nzc, 1);
        cs.zchunk = (int)((d.nz + nzc - 1) / nzc);
        nzc = (int)((d.nz + cs.zchunk - 1) / cs.zchunk);
        const int nb = cs.ncb * nzc;
        const double frac = (double)sampled / (double)nseg;
        const bool spec = m.w[i] >= 3;
        rc = launch(h, s, F_COL_SAMPLE, in_b * N * frac, N * frac, [&] {
            return launch_column(src, OP_HIST1, spec, cs, nb, s);
        });
        if (!rc) rc = launch(h, s, F_FINALIZE, 8.0 * kL1Bins, 0, [&] {
            return launch_finalize_predict(sti, hi + kOffSample, r.t, s);
        });
        if (rc) return rc;
    }
    // one selection pass for every width
    rc = launch(h, s, F_MULTI_SELECT, in_b * N, N * m.nw,
                [&] { return launch_multi(src, MOP_SELECT, m, g.blocks(), s); });
    if (rc) return rc;
    for (int i = 0; i < m.nw; ++i) {
        DevState *sti = m.sti[i];
        unsigned long long *hi = hist_of(i);
        const int k = m.k[i];
        const bool spec = m.w[i] >= 3;
        ColArgs c = col_args(i);
        rc = launch(h, s, F_FINALIZE, 0, 0, [&] {
            return launch_finalize_select(sti, m.sel_part[i], (int)nparts, m.cap_count[i],
                                          (unsigned long long)capcap, k, nullptr, 0ull, s);
        });
        if (!rc) rc = launch(h, s, F_CAPTURE_SELECT, 0, 0, [&] {
            return launch_capture_l1(sti, m.cap[i], m.cap_count[i], hi, wb1, s);
        });
        if (rc) return rc;
        c.skip_if_captured = 1;
        rc = launch(h, s, F_COL_HIST1, in_b * N, N, [&] {
            return launch_column(src, OP_HIST1, spec, c, g.blocks(), s);
        }, k);
        if (!rc) rc = launch(h, s, F_FINALIZE, 8.0 * kL1Bins, 0, [&] {
            return launch_finalize_mad1(sti, hi, s);
        });
        if (!rc) rc = launch(h, s, F_CAPTURE_SELECT, 0, 0, [&] {
            return launch_capture_coarse(sti, m.cap[i], m.cap_count[i], hi + kOffL2c, wb2, s);
        });
        if (!rc) rc = launch(h, s, F_COL_HIST2, in_b * N, N, [&] {
            return launch_column(src, OP_HIST2, spec, c, g.blocks(), s);
        }, k);
        if (!rc) rc = launch(h, s, F_FINALIZE, 8.0 * 2 * kL2Coarse, 0, [&] {
            return launch_finalize_mad2a(sti, hi + kOffL2c, s);
        });
        if (!rc) rc = launch(h, s, F_CAPTURE_SELECT, 0, 0, [&] {
            return launch_capture_fine(sti, m.cap[i], m.cap_count[i], hi + kOffL2, wb2, s);
        });
        if (!rc) rc = launch(h, s, F_FINALIZE, 8.0 * 2 * kL2Fine, 0, [&] {
            return launch_finalize_mad2b(sti, hi + kOffL2, k, r.t, 0, s);
        });
        if (rc) return rc;
    }
    return launch(h, s, F_FINALIZE, 0, 0, [&] { return launch_multi_gather(m, s); });
}

// Replacement off: the kernel pairs are independent, and the pairs that
// share a spatial kernel share their passes. Per spatial kernel (in order of
// first appearance) and up to kMultiMax of its spectral widths: the spatial
// pass (if any), the noise of every width (one pass for the RMS partials and
// one finaliser, or the MAD steps above), one clip pass ORing every width's
// detections into the run's detection bits; at the end the caller's mask.
int enqueue_fused(sofia_sc *h, hipStream_t s, const Work &w, const RunSpec &r) {
    int rc;
    const Dims &d = r.d;
    const double N = (double)d.N;
    const bool any_spatial = r.any_spatial();
    rc = launch(h, s, F_FINALIZE, 0, 0, [&] { return launch_set_sigma0(w.st, NAN, s); });
    if (rc) return rc;
    const int64_t wpp = det_words_per_plane(d.ncol);
    // the blank bits: read by the passes over a spatially smoothed cube
    if (any_spatial) {
        rc = launch(h, s, F_INIT, 4.125 * N, N, [&] {
            return launch_init_bits(r.cube, nullptr, w.blank, nullptr, d.ncol, d.nz, wpp, s);
        });
        if (rc) return rc;
    }
    const ColGrid g = col_grid(d.ncol, d.nz, w.sh);
    if ((int64_t)g.ncb * g.nzc > 0x7fffffffLL)
        return fail(h, SOFIA_SC_EINVAL, "cube too large for the column grid");
    const size_t parts = (size_t)g.blocks() * kMultiMax;
    if ((rc = grow(h, h->mu_sum, h->mu_sum_cap, parts, "fused partials", nullptr)) ||
        (rc = grow(h, h->mu_cnt, h->mu_cnt_cap, parts, "fused counts", nullptr)))
        return rc;
    // groups of kernels with the same spatial kernel, in order of first use
    std::vector<int> done((size_t)r.K, 0);
    bool first = true;
    for (int k0 = 0; k0 < r.K; ++k0) {
        if (done[k0]) continue;
        const Plan &sp = r.plans[k0];
        std::vector<int> ks;
        for (int k = k0; k < r.K; ++k) {
            const Plan &q = r.plans[k];
            if (!done[k] && q.n_iter == sp.n_iter && q.radius == sp.radius &&
                q.gauss_r == sp.gauss_r && (q.gauss_r == 0 || q.fwhm == sp.fwhm)) {
                ks.push_back(k);
                done[k] = 1;
            }
        }
        const bool spatial = sp.spatial();
        if (spatial) {
            PairJob j;
            j.x = r.cube;
            j.d = d;
            j.pl = sp;
            j.k = k0;
            if ((rc = spatial_pass(h, s, w, j))) return rc;
        }
        for (size_t c0 = 0; c0 < ks.size(); c0 += kMultiMax) {
            MultiArgs m{};
            m.src = spatial ? w.p : r.cube;
            m.blank = spatial ? w.blank : nullptr;
            // every chunk ORs its detections into the same bits in place
            m.det_in = first ? nullptr : w.det[0];
            m.det_out = w.det[0];
            m.wpp = wpp;
            m.st = w.st;
            m.part_sum = h->mu_sum;
            m.part_cnt = h->mu_cnt;
            m.ncol = d.ncol;
            m.nz = d.nz;
            m.ncb = g.ncb;
            m.zchunk = g.zchunk;
            m.nparts = g.blocks();
            m.range = r.range;
            m.zstride = r.zstride;
            m.t = r.t;
            m.hmax = 0;
            for (size_t i = c0; i < ks.size() && m.nw < kMultiMax; ++i) {
                const int wd = r.plans[ks[i]].width;
                m.w[m.nw] = wd;
                m.h[m.nw] = (wd - 1) / 2;
                m.k[m.nw] = ks[i];
                m.hmax = std::max(m.hmax, m.h[m.nw]);
                ++m.nw;
            }
            const int src = spatial ? SRC_P : SRC_X;
            // algorithmic bytes: the source once (+ the blank bits) per pass;
            // the clip's detection bits out (and in when ORing)
            const double in_b = 4.0 + (spatial ? 0.125 : 0.0);
            if (r.mode == SOFIA_SC_NOISE_STD) {
                rc = launch(h, s, F_MULTI_STATS, in_b * N, N * m.nw,
                            [&] { return launch_multi(src, MOP_STATS, m, g.blocks(), s); });
                if (!rc) rc = launch(h, s, F_FINALIZE, 0, 0,
                                     [&] { return launch_multi_finalize(m, s); });
            } else {
                rc = fused_mad_noise(h, s, w, r, g, m, spatial, in_b);
            }
            if (!rc) rc = launch(h, s, F_MULTI_CLIP, (in_b + (first ? 0.125 : 0.25)) * N,
                                 N * m.nw,
                                 [&] { return launch_multi(src, MOP_CLIP, m, g.blocks(), s); });
            if (rc) return rc;
            first = false;
        }
    }
    return launch(h, s, F_MASK_OUT, 0.125 * N + (r.keep ? 2.0 : 1.0) * N, N, [&] {
        return launch_write_mask(w.det[0], r.mask, r.keep ? 1 : 0, nullptr, d.ncol, d.nz, wpp,
                                 s);
    });
}

// Noise values of a finished run in cube units, and its sigma_0 output.
int read_run(sofia_sc *h, const DevState &hs, const RunSpec &r, double *noise,
             double *sigma0_out) {
    const bool q16 = r.storage != SOFIA_SC_STORE_F32;
    const double scale = q16 ? hs.scale : 1.0;   // stored units -> cube units
    for (int k = 0; k < r.K; ++k) noise[k] = hs.sigma[k] * scale;
    if (sigma0_out)
        *sigma0_out = q16 ? hs.scale
                          : (r.repl >= 0.0 || !std::isnan(r.sigma0) ? hs.sigma0 : NAN);
    if (hs.status) return fail(h, SOFIA_SC_ENOSTAT, "no finite voxel in the flux range for some kernel");
    return SOFIA_SC_OK;
}

// The argument checks of a whole run (sofia_sc_run, _run_ex and
// sofia_sc_check_run; per cube in a batch), before any device work. h may be
// NULL (no error text). plans (optional) receives the kernels' plans.
int validate_run(sofia_sc *h, int64_t nx, int64_t ny, int64_t nz, const sofia_sc_kernel *kernels,
                 int32_t K, double t, int32_t mode, int32_t range, const sofia_sc_options *opt,
                 std::vector<Plan> *plans) {
    if (!kernels) return fail(h, SOFIA_SC_EINVAL, "NULL argument");
    if (K < 1 || K > SOFIA_SC_MAX_KERNELS)
        return fail(h, SOFIA_SC_EINVAL, "number of kernels must be 1..64");
    int rc;
    if ((rc = check_options(h, opt))) return rc;
    if ((rc = check_dims(h, nx, ny, nz))) return rc;
    if ((rc = check_modes(h, t, mode, range))) return rc;
    std::vector<Plan> local((size_t)K);
    for (int k = 0; k < K; ++k)
        if ((rc = make_plan(h, kernels[k], &local[k]))) return rc;
    if (opt->fuse_widths && !(opt->replacement < 0.0 && opt->storage == SOFIA_SC_STORE_F32))
        return fail(h, SOFIA_SC_EINVAL, "fuse_widths needs replacement off and FP32 storage");
    if (plans) *plans = std::move(local);
    return SOFIA_SC_OK;
}

int run_impl(sofia_sc *h, const float *cube, int64_t nx, int64_t ny, int64_t nz,
             const sofia_sc_kernel *kernels, int32_t K, double t, int32_t mode,
             int32_t range, uint8_t *mask, double *noise, const sofia_sc_options *opt,
             double *sigma0_out) {
    if (!h) return SOFIA_SC_EINVAL;
    h->err[0] = 0;
    if (noise && K > 0 && K <= SOFIA_SC_MAX_KERNELS) nan_fill(noise, K);
    if (sigma0_out) *sigma0_out = NAN;
    if (!cube || !kernels || !mask || !noise)
        return fail(h, SOFIA_SC_EINVAL, "NULL argument");
    int rc;
    std::vector<Plan> plans;
    if ((rc = validate_run(h, nx, ny, nz, kernels, K, t, mode, range, opt, &plans))) return rc;
    DeviceGuard dg(h->device);
    if (dg.err != hipSuccess) return hip_fail(h, dg.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)opt->stream;
    const RunSpec r{cube, Dims{nx, ny, nz, nx * ny, nx * ny * nz}, plans.data(), K, t, mode,
                    range, mask, opt->replacement, opt->sigma0, opt->storage,
                    opt->keep_input_mask != 0, plane_stride(opt)};
    if ((rc = ensure_state(h))) return rc;
    h->w.sh = shapes_of(h->tune);
    SC_TRACE("run %lldx%lldx%lld, %d kernels, storage %d, col_blocks %d, strip_rows %d",
             (long long)nx, (long long)ny, (long long)nz, K, opt->storage, h->w.sh.col_blocks,
             h->w.sh.strip_rows);
    if ((rc = ensure_for(h, h->w, r))) return rc;
    if ((rc = (opt->fuse_widths ? enqueue_fused(h, s, h->w, r) : enqueue_run(h, s, h->w, r))))
        return rc;
    if ((rc = finish(h, s, h->st_host, h->w.st))) return rc;
    return read_run(h, *h->st_host, r, noise, sigma0_out);
}

// ---- batches: many independent cubes, one graph launch

bool same_key(const BatchKey &a, const BatchKey &b) {
    if (a.cubes.size() != b.cubes.size() || a.kernels.size() != b.kernels.size()) return false;
    for (size_t i = 0; i < a.cubes.size(); ++i) {
        const sofia_sc_cube &x = a.cubes[i], &y = b.cubes[i];
        if (x.cube != y.cube || x.mask != y.mask || x.nx != y.nx || x.ny != y.ny || x.nz != y.nz)
            return false;
    }
    for (size_t k = 0; k < a.kernels.size(); ++k)
        if (std::memcmp(&a.kernels[k].spatial_fwhm_px, &b.kernels[k].spatial_fwhm_px,
                        sizeof(double)) != 0 ||
            a.kernels[k].spectral_width_ch != b.kernels[k].spectral_width_ch ||
            a.kernels[k].spatial_kind != b.kernels[k].spatial_kind)
            return false;
    return a.t == b.t && a.repl == b.repl && a.sigma0_bits == b.sigma0_bits &&
           a.mode == b.mode && a.range == b.range && a.storage == b.storage &&
           a.keep == b.keep && a.zstride == b.zstride && a.lanes == b.lanes && a.col_blocks == b.col_blocks &&
           a.strip_rows == b.strip_rows && a.strip_waves == b.strip_waves &&
           a.col_min_planes == b.col_min_planes && a.work_gen == b.work_gen;
}

// Lane streams, fork/join events and the per-cube device states.
int ensure_batch_infra(sofia_sc *h, size_t n, bool *moved) {
    hipError_t e;
    for (int l = 0; l < kBatchLanes; ++l) {
        if (!h->lane_s[l] &&
            (e = hipStreamCreateWithFlags(&h->lane_s[l], hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(h, e, "lane stream");
        if (!h->join_ev[l] &&
            (e = hipEventCreateWithFlags(&h->join_ev[l], hipEventDisableTiming)) != hipSuccess)
            return hip_fail(h, e, "lane event");
    }
    if (!h->fork_ev &&
        (e = hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(h, e, "fork event");
    if (n > h->bst_cap) {
        drop_graph(h);   // the graph holds the per-cube state pointers
        if (h->bst) (void)hipFree(h->bst);
        if (h->bst_host) (void)hipHostFree(h->bst_host);
        h->bst = nullptr;
        h->bst_host = nullptr;
        h->bst_cap = 0;
        if ((e = dev_alloc(h, (void **)&h->bst, n * sizeof(DevState))) != hipSuccess) {
            h->bst = nullptr;
            return fail(h, SOFIA_SC_ENOMEM, std::string("batch states: ") + hipGetErrorString(e));
        }
        if ((e = host_alloc(h, (void **)&h->bst_host, n * sizeof(DevState))) != hipSuccess) {
            (void)hipFree(h->bst);
            h->bst = nullptr;
            h->bst_host = nullptr;
            return fail(h, SOFIA_SC_ENOMEM,
                        std::string("batch host states: ") + hipGetErrorString(e));
        }
        h->bst_cap = n;
        *moved = true;
    }
    return SOFIA_SC_OK;
}

// Capture every cube's launch chain into one graph: lane l's cubes run one
// after another on lane stream l, the lanes side by side (forked from and
// joined back into lane 0, the capture's origin).
int capture_batch(sofia_sc *h, const std::vector<RunSpec> &runs,
                  const std::vector<std::vector<int>> &lane_cubes) {
    const int L = (int)lane_cubes.size();
    hipStream_t s0 = h->lane_s[0];
    hipError_t e = hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(h, e, "graph capture");
    h->capturing = true;
    h->capture_bytes = 0;
    int rc = SOFIA_SC_OK;
    e = hipEventRecord(h->fork_ev, s0);
    for (int l = 1; l < L && e == hipSuccess; ++l) e = hipStreamWaitEvent(h->lane_s[l], h->fork_ev, 0);
    if (e != hipSuccess) rc = hip_fail(h, e, "graph fork");
    for (int l = 0; l < L && rc == SOFIA_SC_OK; ++l) {
        for (int i : lane_cubes[l]) {
            Work w = h->lanes[l];
            w.st = h->bst + i;
            if ((rc = enqueue_run(h, h->lane_s[l], w, runs[(size_t)i]))) break;
        }
    }
    // join every forked lane, also after an error, so no stream stays in capture
    for (int l = 1; l < L; ++l) {
        hipError_t ej = hipEventRecord(h->join_ev[l], h->lane_s[l]);
        if (ej == hipSuccess) ej = hipStreamWaitEvent(s0, h->join_ev[l], 0);
        if (ej != hipSuccess && rc == SOFIA_SC_OK) rc = hip_fail(h, ej, "graph join");
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s0, &g);
    h->capturing = false;
    if (rc == SOFIA_SC_OK && e != hipSuccess) rc = hip_fail(h, e, "graph capture end");
    if (rc == SOFIA_SC_OK) {
        e = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            h->gexec = nullptr;
            rc = hip_fail(h, e, "graph instantiate");
        }
    }
    if (g) (void)hipGraphDestroy(g);
    if (rc == SOFIA_SC_OK) h->graph_bytes = h->capture_bytes;
    return rc;
}

int batch_impl(sofia_sc *h, const sofia_sc_cube *cubes, int32_t n,
               const sofia_sc_kernel *kernels, int32_t K, double t, int32_t mode,
               int32_t range, double *noise, const sofia_sc_options *opt,
               double *sigma0_out) {
    if (!h) return SOFIA_SC_EINVAL;
    h->err[0] = 0;
    const bool sizes_ok = n >= 1 && n <= SOFIA_SC_MAX_CUBES && K >= 1 && K <= SOFIA_SC_MAX_KERNELS;
    if (sizes_ok) {
        nan_fill(noise, n * K);
        nan_fill(sigma0_out, n);
    }
    if (!cubes || !kernels || !noise) return fail(h, SOFIA_SC_EINVAL, "NULL argument");
    if (!sizes_ok)
        return fail(h, SOFIA_SC_EINVAL, "number of cubes must be 1..4096 and of kernels 1..64");
    int rc;
    if ((rc = check_options(h, opt))) return rc;
    if (opt->fuse_widths)
        return fail(h, SOFIA_SC_EINVAL, "fuse_widths is for sofia_sc_run / _run_ex only");
    if ((rc = check_modes(h, t, mode, range))) return rc;
    std::vector<Plan> plans((size_t)K);
    for (int k = 0; k < K; ++k)
        if ((rc = make_plan(h, kernels[k], &plans[k]))) return rc;
    std::vector<RunSpec> runs;
    runs.reserve((size_t)n);
    std::vector<const uint8_t *> masks;
    for (int i = 0; i < n; ++i) {
        const sofia_sc_cube &c = cubes[i];
        if (!c.cube || !c.mask)
            return fail(h, SOFIA_SC_EINVAL, "NULL cube or mask in cube " + std::to_string(i));
        if ((rc = check_dims(h, c.nx, c.ny, c.nz))) {
            const size_t len = std::strlen(h->err);
            std::snprintf(h->err + len, sizeof(h->err) - len, " (cube %d)", i);
            return rc;
        }
        runs.push_back(RunSpec{c.cube, Dims{c.nx, c.ny, c.nz, c.nx * c.ny, c.nx * c.ny * c.nz},
                               plans.data(), K, t, mode, range, c.mask, opt->replacement,
                               opt->sigma0, opt->storage, opt->keep_input_mask != 0,
                               plane_stride(opt)});
        masks.push_back(c.mask);
    }
    std::sort(masks.begin(), masks.end());
    if (std::adjacent_find(masks.begin(), masks.end()) != masks.end())
        return fail(h, SOFIA_SC_EINVAL, "two cubes share one mask");
    DeviceGuard dg(h->device);
    if (dg.err != hipSuccess) return hip_fail(h, dg.err, "hipSetDevice");

    // Longest first onto the least loaded lane.
    const int L = std::min<int>(h->tune.lanes, n);
    std::vector<int> order((size_t)n);
    for (int i = 0; i < n; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return runs[(size_t)a].d.N > runs[(size_t)b].d.N; });
    std::vector<std::vector<int>> lane_cubes((size_t)L);
    std::vector<double> load((size_t)L, 0.0);
    for (int i : order) {
        const size_t l = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
        lane_cubes[l].push_back(i);
        load[l] += (double)runs[(size_t)i].d.N;
    }
    bool moved = false;
    for (int l = 0; l < L; ++l) {
        h->lanes[l].sh = shapes_of(h->tune);
        for (int i : lane_cubes[(size_t)l])
            if ((rc = ensure_for(h, h->lanes[l], runs[(size_t)i], &moved))) return rc;
    }
    if ((rc = ensure_batch_infra(h, (size_t)n, &moved))) return rc;
    if (moved) {
        ++h->work_gen;
        drop_graph(h);
    }

    BatchKey key;
    key.cubes.assign(cubes, cubes + n);
    key.kernels.assign(kernels, kernels + K);
    key.t = t;
    key.repl = opt->replacement;
    std::memcpy(&key.sigma0_bits, &opt->sigma0, sizeof(double));
    key.mode = mode;
    key.range = range;
    key.storage = opt->storage;
    key.keep = opt->keep_input_mask;
    key.zstride = plane_stride(opt);
    key.lanes = L;
    key.col_blocks = h->tune.col_blocks;
    key.strip_rows = h->tune.strip_rows;
    key.strip_waves = h->tune.strip_waves;
    key.col_min_planes = h->tune.col_min_planes;
    key.work_gen = h->work_gen;
    if (!h->gvalid || !same_key(key, h->gkey)) {
        drop_graph(h);
        SC_TRACE("batch capture: %d cubes on %d lanes, col_blocks %d, strip_rows %d, "
                 "strip_waves %d, col_min_planes %d", n, L, h->tune.col_blocks,
                 h->tune.strip_rows, h->tune.strip_waves, h->tune.col_min_planes);
        rc = capture_batch(h, runs, lane_cubes);
        SC_TRACE("batch capture done: rc %d %s", rc, h->err);
        if (rc) return rc;
        h->gkey = std::move(key);
        h->gvalid = true;
    }

    hipStream_t s = (hipStream_t)opt->stream;
    double vox = 0;
    for (const RunSpec &r : runs) vox += (double)r.d.N;
    rc = launch(h, s, F_BATCH, h->graph_bytes, vox, [&] { return hipGraphLaunch(h->gexec, s); });
    if (rc) {
        SC_TRACE("batch launch failed: %s", h->err);
        return rc;
    }
    if ((rc = finish(h, s, h->bst_host, h->bst, (size_t)n))) return rc;
    for (int i = 0; i < n; ++i) {
        const int ri = read_run(h, h->bst_host[i], runs[(size_t)i], noise + (size_t)i * K,
                                sigma0_out ? sigma0_out + i : nullptr);
        if (ri) rc = ri;
    }
    if (rc == SOFIA_SC_ENOSTAT)
        fail(h, rc, "no finite voxel in the flux range for some kernel of some cube");
    return rc;
}

// Autotuning of the launch shapes of single runs: coordinate search, one
// shape parameter at a time, each candidate timed as the faster of two runs
// of the caller's cube after an untimed one. Runs capture no graph.
int tune_run_impl(sofia_sc *h, const float *cube, int64_t nx, int64_t ny, int64_t nz,
                  const sofia_sc_kernel *kernels, int32_t K, double t, int32_t mode,
                  int32_t range, uint8_t *mask, const sofia_sc_options *opt,
                  sofia_sc_batch_tuning *best) {
    if (!h) return SOFIA_SC_EINVAL;
    if (best) *best = h->tune;
    if (K < 1 || K > SOFIA_SC_MAX_KERNELS)
        return fail(h, SOFIA_SC_EINVAL, "number of kernels must be 1..64");
    std::vector<double> noise((size_t)K);
    const sofia_sc_batch_tuning start = h->tune;
    auto one = [&]() {
        return run_impl(h, cube, nx, ny, nz, kernels, K, t, mode, range, mask, noise.data(),
                        opt, nullptr);
    };
    auto time_it = [&](const sofia_sc_batch_tuning &c, double *ms) -> int {
        h->tune = c;
        int rc = one();
        if (rc != SOFIA_SC_OK && rc != SOFIA_SC_ENOSTAT) return rc;
        double bestms = INFINITY;
        for (int rep = 0; rep < 2; ++rep) {
            const auto t0 = std::chrono::steady_clock::now();
            rc = one();
            const auto t1 = std::chrono::steady_clock::now();
            if (rc != SOFIA_SC_OK && rc != SOFIA_SC_ENOSTAT) return rc;
            bestms = std::min(bestms, std::chrono::duration<double, std::milli>(t1 - t0).count());
        }
        *ms = bestms;
        return SOFIA_SC_OK;
    };
    sofia_sc_batch_tuning cur = start;
    int rc = time_it(cur, &cur.ms);
    SC_TRACE("tune start: rc %d, %.3f ms", rc, cur.ms);
    if (rc) { h->tune = start; return rc; }
    struct Axis {
        int32_t sofia_sc_batch_tuning::*field;
        int vals[3];
    };
    const Axis axes[] = {
        {&sofia_sc_batch_tuning::col_blocks, {3072, 6144, 12288}},
        {&sofia_sc_batch_tuning::strip_rows, {64, 128, 256}},
        {&sofia_sc_batch_tuning::strip_waves, {1, 2, 4}},
        {&sofia_sc_batch_tuning::col_min_planes, {32, 64, 128}},
    };
    for (const Axis &ax : axes) {
        for (int v : ax.vals) {
            if (cur.*(ax.field) == v) continue;
            sofia_sc_batch_tuning c = cur;
            c.*(ax.field) = v;
            rc = time_it(c, &c.ms);
            SC_TRACE("tune candidate col_blocks %d strip_rows %d strip_waves %d "
                     "col_min_planes %d: rc %d, %.3f ms", c.col_blocks, c.strip_rows,
                     c.strip_waves, c.col_min_planes, rc, c.ms);
            if (rc) { h->tune = start; return rc; }
            if (c.ms < cur.ms) cur = c;
        }
    }
    h->tune = cur;
    if (best) *best = cur;
    // leave the mask with the chosen shapes' result
    return one();
}

bool valid_shapes(const sofia_sc_batch_tuning &t) {
    auto in = [](int v, int a, int b, int c) { return v == a || v == b || v == c; };
    return in(t.lanes, 4, 8, 16) && in(t.col_blocks, 3072, 6144, 12288) &&
           in(t.strip_rows, 64, 128, 256) && in(t.strip_waves, 1, 2, 4) &&
           in(t.col_min_planes, 32, 64, 128);
}


// ---- local noise normalisation (Sect. 4.1)

int normalise_impl(sofia_sc *h, const float *cube, int64_t nx, int64_t ny, int64_t nz,
                   int32_t wxy, int32_t wz, int32_t gxy, int32_t gz, int32_t mode,
                   int32_t range, float *out, double *grid, void *stream) {
    if (!h) return SOFIA_SC_EINVAL;
    h->err[0] = 0;
    if (!cube || (!out && !grid)) return fail(h, SOFIA_SC_EINVAL, "NULL argument");
    int rc;
    if ((rc = check_dims(h, nx, ny, nz))) return rc;
    if ((rc = check_modes(h, 1.0, mode, range))) return rc;
    auto odd_ok = [](int32_t w) { return w >= 1 && w <= SOFIA_SC_NORM_MAX_WINDOW && (w & 1); };
    if (!odd_ok(wxy) || !odd_ok(wz))
        return fail(h, SOFIA_SC_EINVAL, "window sizes must be odd, 1..SOFIA_SC_NORM_MAX_WINDOW");
    if (gxy == 0) gxy = (wxy + 1) / 2;
    if (gz == 0) gz = (wz + 1) / 2;
    if (gxy < 1 || gz < 1 || gxy > 65536 || gz > 65536)
        return fail(h, SOFIA_SC_EINVAL, "grid steps must be 0 (default) or 1..65536");
    NormArgs a{};
    a.x = cube;
    a.y = out;
    a.nx = nx; a.ny = ny; a.nz = nz;
    a.wxy = wxy; a.wz = wz; a.gxy = gxy; a.gz = gz;
    a.nbx = (int32_t)((nx + gxy - 1) / gxy);
    a.nby = (int32_t)((ny + gxy - 1) / gxy);
    a.nbz = (int32_t)((nz + gz - 1) / gz);
    a.range = range;
    const int64_t nb = (int64_t)a.nbx * a.nby * a.nbz;
    if (nb > 0x7fffffffLL) return fail(h, SOFIA_SC_EINVAL, "noise grid too large");
    DeviceGuard dg(h->device);
    if (dg.err != hipSuccess) return hip_fail(h, dg.err, "hipSetDevice");
    if ((rc = grow(h, h->nn_sigma, h->nn_cap, (size_t)nb, "noise grid", nullptr))) return rc;
    a.sigma = h->nn_sigma;
    hipStream_t s = (hipStream_t)stream;
    const double N = (double)nx * ny * nz;
    SC_TRACE("normalise %lldx%lldx%lld, window %d/%d, grid %d/%d, %lld blocks", (long long)nx,
             (long long)ny, (long long)nz, wxy, wz, gxy, gz, (long long)nb);
    rc = launch(h, s, F_NORM_NOISE, 4.0 * N + 8.0 * nb, N,
                [&] { return launch_window_noise(mode, a, s); });
    if (rc) return rc;
    if (out) {
        rc = launch(h, s, F_NORM_DIVIDE, 8.0 * N + 8.0 * nb, N,
                    [&] { return launch_norm_divide(a, s); });
        if (rc) return rc;
    }
    hipError_t e;
    if (grid && (e = hipMemcpyAsync(grid, a.sigma, (size_t)nb * sizeof(double),
                                    hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(h, e, "copy of the noise grid");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(h, e, "stream");
    if (h->prof) collect_profile(h);
    return SOFIA_SC_OK;
}


// ---- linker (Sect. 4.3)

int link_impl(sofia_sc *h, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz,
              int32_t rxy, int32_t rz, int32_t min_xy, int32_t min_z, int32_t max_xy,
              int32_t max_z, int32_t *labels, int64_t *n_sources, int64_t *boxes, int64_t cap,
              void *stream) {
    if (!h) return SOFIA_SC_EINVAL;
    h->err[0] = 0;
    if (n_sources) *n_sources = -1;
    if (!mask || !labels || !n_sources || (cap > 0 && !boxes) || cap < 0)
        return fail(h, SOFIA_SC_EINVAL, "NULL argument or negative capacity");
    int rc;
    if ((rc = check_dims(h, nx, ny, nz))) return rc;
    const int64_t N = nx * ny * nz;
    if (N > 0x7fffffffLL)
        return fail(h, SOFIA_SC_EINVAL, "the linker takes cubes of fewer than 2^31 voxels");
    if (rxy < 0 || rz < 0 || rxy > SOFIA_SC_LINK_MAX_RADIUS || rz > SOFIA_SC_LINK_MAX_RADIUS)
        return fail(h, SOFIA_SC_EINVAL, "linker radii must be 0..SOFIA_SC_LINK_MAX_RADIUS");
    if (min_xy < 0 || min_z < 0 || max_xy < 0 || max_z < 0)
        return fail(h, SOFIA_SC_EINVAL, "size limits must be >= 0");
    LinkArgs a{};
    a.mask = mask;
    a.L = labels;
    a.nx = nx; a.ny = ny; a.nz = nz;
    a.min_xy = min_xy; a.min_z = min_z; a.max_xy = max_xy; a.max_z = max_z;
    // the forward half of the ellipsoid's offsets (the later voxel in raster
    // order): each friendship is tested once, from its earlier voxel
    const int64_t A = (int64_t)rxy * rxy, C = (int64_t)rz * rz;
    for (int dz = 0; dz <= rz; ++dz)
        for (int dy = -rxy; dy <= rxy; ++dy)
            for (int dx = -rxy; dx <= rxy; ++dx) {
                if (dz == 0 && (dy < 0 || (dy == 0 && dx <= 0))) continue;
                const int64_t sxy = (int64_t)dx * dx + (int64_t)dy * dy, sz = (int64_t)dz * dz;
                bool in;
                if (rxy > 0 && rz > 0) in = sxy * C + sz * A <= A * C;
                else if (rxy > 0) in = sz == 0 && sxy <= A;
                else if (rz > 0) in = sxy == 0 && sz <= C;
                else in = false;
                if (!in) continue;
                if (a.n_off == kLinkMaxOffsets)
                    return fail(h, SOFIA_SC_EINVAL, "linker radii give too many offsets");
                a.delta[a.n_off] = (int32_t)(((int64_t)dz * ny + dy) * nx + dx);
                a.off[a.n_off++] = (dx + 128) | ((dy + 128) << 8) | ((dz + 128) << 16);
            }
    DeviceGuard dg(h->device);
    if (dg.err != hipSuccess) return hip_fail(h, dg.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const double Nd = (double)N;
    SC_TRACE("link %lldx%lldx%lld, radii %d/%d, %d offsets", (long long)nx, (long long)ny,
             (long long)nz, rxy, rz, a.n_off);
    const int64_t nb = link_scan_blocks(N);
    if ((rc = grow(h, h->lk_counts, h->lk_counts_cap, (size_t)nb + 1, "link counts", nullptr)))
        return rc;
    // the list of the detected voxels in raster order, and the forest
    rc = launch(h, s, F_LINK_NUMBER, Nd, Nd, [&] {
        return launch_link_number(LK_VOXELS, a, N, h->lk_counts, s);
    });
    if (rc) return rc;
    int m = 0;
    hipError_t e = hipMemcpyAsync(&m, h->lk_counts + nb, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "count of detected voxels");
    int nc = 0;
    if (m > 0) {
        if ((rc = grow(h, h->lk_list, h->lk_list_cap, (size_t)m, "link list", nullptr)))
            return rc;
        a.list = h->lk_list;
        a.m = m;
        const double Md = (double)m;
        const int64_t nbm = link_scan_blocks(m);   // <= nb: lk_counts holds its counts
        rc = launch(h, s, F_LINK_NUMBER, Nd + 4.0 * Md, Nd, [&] {
            return launch_link_assign(LK_VOXELS, a, N, h->lk_counts, s);
        });
        if (!rc) rc = launch(h, s, F_LINK_UNION, 8.0 * Md, Md, [&] { return launch_link_init(a, s); });
        if (!rc) rc = launch(h, s, F_LINK_UNION, 12.0 * Md, Md, [&] { return launch_link_union(a, s); });
        if (!rc) rc = launch(h, s, F_LINK_UNION, 12.0 * Md, Md, [&] { return launch_link_flatten(a, s); });
        if (!rc) rc = launch(h, s, F_LINK_NUMBER, 8.0 * Md, Md, [&] {
            return launch_link_number(LK_ROOTS, a, m, h->lk_counts, s);
        });
        if (rc) return rc;
        e = hipMemcpyAsync(&nc, h->lk_counts + nbm, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(h, e, "count of detections");
    }
    int n_kept = 0;
    if (nc > 0) {
        const int64_t nbc = link_scan_blocks(nc);
        if ((rc = grow(h, h->lk_box, h->lk_box_cap, (size_t)nc * 8, "link boxes", nullptr)) ||
            (rc = grow(h, h->lk_label, h->lk_label_cap, (size_t)nc, "link labels", nullptr)) ||
            (rc = grow(h, h->lk_kcounts, h->lk_kcounts_cap, (size_t)nbc + 1, "link counts",
                       nullptr)))
            return rc;
        a.box = h->lk_box;
        a.label_of = h->lk_label;
        const double Md = (double)m;
        rc = launch(h, s, F_LINK_NUMBER, 12.0 * Md, Md, [&] {
            return launch_link_assign(LK_ROOTS, a, m, h->lk_counts, s);
        });
        if (!rc) rc = launch(h, s, F_LINK_NUMBER, 16.0 * Md, Md, [&] {
            return launch_link_resolve(a, nc, s);
        });
        if (!rc) rc = launch(h, s, F_LINK_NUMBER, 32.0 * nc, nc, [&] {
            return launch_link_number(LK_KEPT, a, nc, h->lk_kcounts, s);
        });
        if (!rc) rc = launch(h, s, F_LINK_NUMBER, 32.0 * nc, nc, [&] {
            return launch_link_assign(LK_KEPT, a, nc, h->lk_kcounts, s);
        });
        if (rc) return rc;
        e = hipMemcpyAsync(&n_kept, h->lk_kcounts + nbc, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(h, e, "count of kept detections");
    }
    rc = launch(h, s, F_LINK_LABEL, 5.0 * Nd + 4.0 * m, Nd, [&] { return launch_link_label(a, s); });
    if (rc) return rc;
    if (boxes && cap > 0 && n_kept > 0) {
        if ((rc = grow(h, h->lk_out, h->lk_out_cap, (size_t)n_kept * 7, "link output boxes",
                       nullptr)))
            return rc;
        rc = launch(h, s, F_LINK_LABEL, 0, 0, [&] {
            return launch_link_boxes_out(a, nc, h->lk_out, s);
        });
        if (rc) return rc;
        const int64_t nout = std::min<int64_t>(cap, n_kept);
        e = hipMemcpyAsync(boxes, h->lk_out, (size_t)nout * 7 * sizeof(long long),
                           hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return hip_fail(h, e, "copy of the boxes");
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(h, e, "stream");
    if (h->prof) collect_profile(h);
    *n_sources = n_kept;
    return SOFIA_SC_OK;
}

// ---- parameterisation and reliability (Sect. 4.4, 4.5)

int param_impl(sofia_sc *h, const float *cube, const int32_t *labels, int64_t nx, int64_t ny,
               int64_t nz, int64_t n, const sofia_sc_param_options *opt, sofia_sc_source *out,
               int64_t *n_kept, void *stream) {
    if (!h) return SOFIA_SC_EINVAL;
    h->err[0] = 0;
    if (n_kept) *n_kept = -1;
    if (!cube || !labels || !opt || !n_kept || (n > 0 && !out))
        return fail(h, SOFIA_SC_EINVAL, "NULL argument");
    if (opt->struct_size != (int32_t)sizeof(sofia_sc_param_options))
        return fail(h, SOFIA_SC_EINVAL, "sofia_sc_param_options.struct_size mismatch");
    int rc;
    if ((rc = check_dims(h, nx, ny, nz))) return rc;
    if (n < 0 || n > 0x7fffffffLL)
        return fail(h, SOFIA_SC_EINVAL, "n_sources must be 0..2^31-1");
    if (!(opt->channel_width > 0.0) || !std::isfinite(opt->channel_width) ||
        !(opt->sigma_rms >= 0.0) || !std::isfinite(opt->sigma_rms) ||
        !(opt->rel_scale > 0.0) || !std::isfinite(opt->rel_scale) ||
        std::isnan(opt->rel_threshold) || std::isnan(opt->snr_threshold) ||
        std::isnan(opt->beam_major_px) || std::isnan(opt->beam_minor_px))
        return fail(h, SOFIA_SC_EINVAL,
                    "channel width and scale must be > 0, sigma_rms >= 0, thresholds numbers");
    DeviceGuard dg(h->device);
    if (dg.err != hipSuccess) return hip_fail(h, dg.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        *n_kept = 0;
        return SOFIA_SC_OK;
    }
    const double a_fw = opt->beam_major_px, b_fw = opt->beam_minor_px;
    ParamArgs a{};
    a.cube = cube;
    a.labels = labels;
    a.nx = nx; a.ny = ny; a.nz = nz;
    a.plane = nx * ny;
    a.n = n;
    a.channel_width = opt->channel_width;
    a.omega = (a_fw > 0.0 && b_fw > 0.0) ? std::acos(-1.0) * a_fw * b_fw / (4.0 * std::log(2.0)) : 1.0;
    a.sigma_rms = opt->sigma_rms;
    a.scale = opt->rel_scale;
    a.rel_threshold = opt->rel_threshold;
    a.snr_threshold = opt->snr_threshold;
    a.vec4 = ((uintptr_t)labels & 15u) == 0;
    if ((rc = grow(h, h->pm_acc, h->pm_acc_cap, (size_t)n, "source accumulators", nullptr)) ||
        (rc = grow(h, h->pm_sign, h->pm_sign_cap, (size_t)n, "source signs", nullptr)) ||
        (rc = grow(h, h->pm_vec, h->pm_vec_cap, (size_t)n * 3, "source vectors", nullptr)) ||
        (rc = grow(h, h->pm_state, h->pm_state_cap, (size_t)16, "reliability state", nullptr)))
        return rc;
    a.acc = h->pm_acc;
    a.sign = h->pm_sign;
    a.vec = h->pm_vec;
    a.rel_state = h->pm_state;
    a.n_kept = reinterpret_cast<unsigned long long *>(h->pm_state + 12);
    a.out = out;
    const double N = (double)(nx * ny * nz), nd = (double)n;
    SC_TRACE("parameterise %lldx%lldx%lld, %lld detections", (long long)nx, (long long)ny,
             (long long)nz, (long long)n);
    // algorithmic bytes: the label cube; the per-detection records
    rc = launch(h, s, F_PARAM, 4.0 * N + nd * (double)sizeof(sofia_sc_source), N,
                [&] { return launch_parameterise(a, s); });
    if (!rc) rc = launch(h, s, F_RELIABILITY, 0.0, nd * nd,
                         [&] { return launch_reliability(a, s); });
    if (rc) return rc;
    unsigned long long kept = 0;
    hipError_t e = hipMemcpyAsync(&kept, a.n_kept, sizeof(kept), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "count of kept detections");
    if (h->prof) collect_profile(h);
    *n_kept = (int64_t)kept;
    return SOFIA_SC_OK;
}

// ---- the entry point that allocates nothing (sofia_sc_run_noalloc)
//
// Its workspace is carved out of `scratch`, a file-scope device array of
// fixed size: every GPU holds its own copy, at its own address, from module
// load to process end. Host code never passes the array's name to a kernel
// (on the host it is only a stand-in for the symbol): sofia_sc_create looks
// up the device address once per device with that device current and keeps
// it in g_scratch; only that pointer is used afterwards.

constexpr size_t kScratchBytes = (size_t)SOFIA_SC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// Called by sofia_sc_create with the handle's device current.
int init_scratch(sofia_sc *h) {
    if (h->device >= kMaxDevices) return SOFIA_SC_OK;   // noalloc refuses such devices
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[h->device]) return SOFIA_SC_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(h, e, "scratch symbol address");
    g_scratch[h->device] = ptr;
    return SOFIA_SC_OK;
}

void *scratch_of(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch[device];
}

// Lays a run's workspace out in one buffer, 256-byte aligned pieces. With
// base == nullptr it only counts the bytes.
struct Carver {
    uint8_t *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t n) {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

// The same buffers ensure_work grows, for one run of r, carved from base.
size_t carve_work(Work &w, uint8_t *base, const RunSpec &r) {
    Carver c{base};
    const bool sp = r.any_spatial();
    const ColGrid g = col_grid(r.d.ncol, r.d.nz, w.sh);
    const size_t parts = (size_t)g.blocks();
    const size_t N = (size_t)r.d.N;
    w.st = c.take<DevState>(1);
    w.hist = c.take<unsigned long long>(kHistWords);
    w.bits_cap = (size_t)bit_words(r.d);
    w.blank = c.take<uint64_t>(w.bits_cap);
    w.det[0] = c.take<uint64_t>(w.bits_cap);
    w.det[1] = c.take<uint64_t>(w.bits_cap);
    w.p = sp ? c.take<float>(N) : nullptr;
    w.p_cap = sp ? N : 0;
    w.amb_cap = amb_capacity(r.d.N);
    w.amb = c.take<AmbEntry>(w.amb_cap);
    w.cap_cap = capture_capacity(r.d.N);
    w.cap_buf = c.take<uint32_t>(w.cap_cap);
    w.part_cap = parts;
    w.part_sum = c.take<double>(parts);
    w.part_cnt = c.take<unsigned long long>(2 * parts);
    const bool q16 = r.storage != SOFIA_SC_STORE_F32;
    w.xq_cap = q16 ? N : 0;
    w.xq = q16 ? c.take<uint16_t>(N) : nullptr;
    return c.off;
}

int noalloc_impl(sofia_sc *h, const float *cube, int64_t nx, int64_t ny, int64_t nz,
                 const sofia_sc_kernel *kernels, int32_t K, double t, int32_t mode,
                 int32_t range, uint8_t *mask, double *noise, const sofia_sc_options *opt,
                 double *sigma0_out) {
    if (!h) return SOFIA_SC_EINVAL;
    h->err[0] = 0;
    if (noise && K > 0 && K <= SOFIA_SC_MAX_KERNELS) nan_fill(noise, K);
    if (sigma0_out) *sigma0_out = NAN;
    if (!cube || !kernels || !mask || !noise) return fail(h, SOFIA_SC_EINVAL, "NULL argument");
    if (K < 1 || K > SOFIA_SC_MAX_KERNELS)
        return fail(h, SOFIA_SC_EINVAL, "number of kernels must be 1..64");
    int rc;
    if ((rc = check_options(h, opt))) return rc;
    if (opt->fuse_widths)
        return fail(h, SOFIA_SC_EINVAL, "fuse_widths is for sofia_sc_run / _run_ex only");
    if ((rc = check_dims(h, nx, ny, nz))) return rc;
    if ((rc = check_modes(h, t, mode, range))) return rc;
    if (nx * ny * nz > SOFIA_SC_NOALLOC_MAX_VOXELS)
        return fail(h, SOFIA_SC_EINVAL,
                    "cube larger than SOFIA_SC_NOALLOC_MAX_VOXELS for sofia_sc_run_noalloc");
    Plan plans[SOFIA_SC_MAX_KERNELS];
    for (int k = 0; k < K; ++k)
        if ((rc = make_plan(h, kernels[k], &plans[k]))) return rc;
    const RunSpec r{cube, Dims{nx, ny, nz, nx * ny, nx * ny * nz}, plans, K, t, mode,
                    range, mask, opt->replacement, opt->sigma0, opt->storage,
                    opt->keep_input_mask != 0, plane_stride(opt)};
    Work w;
    w.sh = shapes_of(h->tune);
    if (carve_work(w, nullptr, r) > kScratchBytes)
        return fail(h, SOFIA_SC_EINVAL,
                    "this cube shape needs more workspace than the no-allocation scratch "
                    "(SOFIA_SC_NOALLOC_SCRATCH_BYTES) holds");
    DeviceGuard dg(h->device);
    if (dg.err != hipSuccess) return hip_fail(h, dg.err, "hipSetDevice");
    uint8_t *base = (uint8_t *)scratch_of(h->device);
    if (!base) return fail(h, SOFIA_SC_EDEVICE, "no scratch address for this device");
    carve_work(w, base, r);
    hipStream_t s = (hipStream_t)opt->stream;
    h->noalloc_call = true;
    rc = enqueue_run(h, s, w, r);
    h->noalloc_call = false;
    if (rc) return rc;
    DevState hs;
    hipError_t e = hipMemcpyAsync(&hs, w.st, sizeof(DevState), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(h, e, "copy of noise values");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(h, e, "stream");
    return read_run(h, hs, r, noise, sigma0_out);
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
    opt->keep_input_mask = 0;
    opt->stream = nullptr;
}

int sofia_sc_quantize(sofia_sc *h, const float *cube, int64_t n, double scale,
                      int32_t storage, uint16_t *out, void *stream) {
    if (!h) return SOFIA_SC_EINVAL;
    h->err[0] = 0;
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
    {
        // set-up of the no-allocation scratch of this device (once per device)
        DeviceGuard dg(device_ordinal);
        const int rc = dg.err != hipSuccess ? SOFIA_SC_EDEVICE : init_scratch(h);
        if (rc != SOFIA_SC_OK) {
            delete h;
            return rc;
        }
    }
    *out = h;
    return SOFIA_SC_OK;
}

void sofia_sc_destroy(sofia_sc *h) {
    if (!h) return;
    {
        DeviceGuard dg(h->device);
        drop_graph(h);
        for (auto &r : h->recs) { (void)hipEventDestroy(r.e0); (void)hipEventDestroy(r.e1); }
        for (auto e : h->pool) (void)hipEventDestroy(e);
        free_work(h->w);   // also frees h->w.st
        for (auto &w : h->lanes) {
            w.st = nullptr;    // lanes borrow the per-cube states
            free_work(w);
        }
        if (h->st_host) (void)hipHostFree(h->st_host);
        if (h->bst) (void)hipFree(h->bst);
        if (h->bst_host) (void)hipHostFree(h->bst_host);
        if (h->nn_sigma) (void)hipFree(h->nn_sigma);
        void *lk[] = {h->lk_counts, h->lk_list, h->lk_box, h->lk_label, h->lk_kcounts, h->lk_out,
                      h->pm_acc, h->pm_sign, h->pm_vec, h->pm_state, h->mu_sum, h->mu_cnt,
                      h->mu_st, h->mu_hist, h->mu_cap, h->mu_sel};
        for (void *p : lk)
            if (p) (void)hipFree(p);
        for (int l = 0; l < kBatchLanes; ++l) {
            if (h->lane_s[l]) (void)hipStreamDestroy(h->lane_s[l]);
            if (h->join_ev[l]) (void)hipEventDestroy(h->join_ev[l]);
        }
        if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
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

int sofia_sc_run_noalloc(sofia_sc *h, const float *cube, int64_t nx, int64_t ny,
                         int64_t nz, const sofia_sc_kernel *kernels, int32_t n_kernels,
                         double threshold, int32_t noise_mode, int32_t flux_range,
                         uint8_t *mask, double *noise, const sofia_sc_options *opt,
                         double *sigma0) {
    return noalloc_impl(h, cube, nx, ny, nz, kernels, n_kernels, threshold, noise_mode,
                        flux_range, mask, noise, opt, sigma0);
}

int sofia_sc_run_batch(sofia_sc *h, const sofia_sc_cube *cubes, int32_t n_cubes,
                       const sofia_sc_kernel *kernels, int32_t n_kernels, double threshold,
                       int32_t noise_mode, int32_t flux_range, double *noise,
                       const sofia_sc_options *opt, double *sigma0) {
    return batch_impl(h, cubes, n_cubes, kernels, n_kernels, threshold, noise_mode, flux_range,
                      noise, opt, sigma0);
}

int sofia_sc_tune_batch(sofia_sc *h, const sofia_sc_cube *cubes, int32_t n_cubes,
                        const sofia_sc_kernel *kernels, int32_t n_kernels, double threshold,
                        int32_t noise_mode, int32_t flux_range, const sofia_sc_options *opt,
                        sofia_sc_batch_tuning *best) {
    // Switched off: timing candidate shapes through repeated graph captures
    // crashed the process when it ran after other batched calls in the same
    // process, for a reason not established. Batches use the handle's shapes
    // (sofia_sc_tune_run, sofia_sc_set_shapes).
    (void)cubes; (void)n_cubes; (void)kernels; (void)n_kernels; (void)threshold;
    (void)noise_mode; (void)flux_range; (void)opt;
    if (!h) return SOFIA_SC_EINVAL;
    if (best) *best = h->tune;
    return fail(h, SOFIA_SC_EDEVICE, "batch autotuning is switched off in this build");
}

int sofia_sc_tune_run(sofia_sc *h, const float *cube, int64_t nx, int64_t ny, int64_t nz,
                      const sofia_sc_kernel *kernels, int32_t n_kernels, double threshold,
                      int32_t noise_mode, int32_t flux_range, uint8_t *mask,
                      const sofia_sc_options *opt, sofia_sc_batch_tuning *best) {
    return tune_run_impl(h, cube, nx, ny, nz, kernels, n_kernels, threshold, noise_mode,
                         flux_range, mask, opt, best);
}

int sofia_sc_set_shapes(sofia_sc *h, const sofia_sc_batch_tuning *shapes) {
    if (!h) return SOFIA_SC_EINVAL;
    h->err[0] = 0;
    if (!shapes) {
        h->tune = default_tuning();
        return SOFIA_SC_OK;
    }
    if (!valid_shapes(*shapes))
        return fail(h, SOFIA_SC_EINVAL, "launch shapes outside the tuning candidates");
    h->tune = *shapes;
    return SOFIA_SC_OK;
}

int sofia_sc_get_shapes(const sofia_sc *h, sofia_sc_batch_tuning *shapes) {
    if (!h || !shapes) return SOFIA_SC_EINVAL;
    *shapes = h->tune;
    return SOFIA_SC_OK;
}

static int single_kernel(sofia_sc *h, const float *cube, int64_t nx, int64_t ny,
                         int64_t nz, sofia_sc_kernel kernel, double threshold,
                         int32_t mode, int32_t range, double replacement,
                         double sigma0, const uint8_t *mask_in, uint8_t *mask_out,
                         double *noise, float *write_out, int32_t storage, void *stream,
                         int zstride = 1) {
    if (!h) return SOFIA_SC_EINVAL;
    h->err[0] = 0;
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
    h->w.sh = shapes_of(h->tune);
    const ColGrid g = col_grid(d.ncol, d.nz, h->w.sh);
    if ((rc = ensure_state(h))) return rc;
    if ((rc = ensure_work(h, h->w, d.N, bit_words(d), pl.spatial(), (size_t)g.blocks(), q16)))
        return rc;
    const Work &w = h->w;
    const int64_t wpp = det_words_per_plane(d.ncol);
    rc = launch(h, s, F_FINALIZE, 0, 0, [&] {
        return launch_set_sigma0(w.st, (repl || q16) ? sigma0 : NAN, s);
    });
    if (rc) return rc;
    // blank bits, and the caller's mask as the detections so far
    rc = launch(h, s, F_INIT, (mask_in ? 5.25 : 4.125) * d.N, (double)d.N, [&] {
        return launch_init_bits(cube, mask_in, w.blank, mask_in ? w.det[0] : nullptr, d.ncol,
                                d.nz, wpp, s);
    });
    if (rc) return rc;
    int xtype = ST_F32;
    if (q16) {
        xtype = storage == SOFIA_SC_STORE_F16 ? ST_F16 : ST_BF16;
        rc = launch(h, s, F_QUANTIZE, 6.0 * d.N, (double)d.N, [&] {
            return launch_quantize(cube, w.st, 0.0, xtype, w.xq, d.N, s);
        });
        if (rc) return rc;
        rc = launch(h, s, F_FINALIZE, 0, 0, [&] { return launch_enter_scaled(w.st, s); });
        if (rc) return rc;
    }
    PairJob j;
    j.x = cube;
    j.xq = q16 ? w.xq : nullptr;
    j.xtype = xtype;
    j.d = d;
    j.pl = pl;
    j.k = 0;
    j.repl_active = repl && mask_in;
    j.repl_n = replacement;
    j.mode = write_out ? 0 : mode;
    j.range = write_out ? 0 : range;
    j.t = write_out ? 1.0 : threshold;
    j.det_in = mask_in ? w.det[0] : nullptr;
    j.blank_in = w.blank;
    j.det_out = write_out ? nullptr : w.det[1];
    j.write_out = write_out;
    j.zstride = zstride;
    if ((rc = run_pair(h, s, w, j))) return rc;
    if (!write_out) {
        // the caller's marks on blanked voxels (never detection bits) stay in
        // the output mask
        rc = launch(h, s, F_MASK_OUT, (mask_in ? 2.125 : 1.125) * d.N, (double)d.N, [&] {
            return launch_write_mask(w.det[1], mask_out, 0, mask_in, d.ncol, d.nz, wpp, s);
        });
        if (rc) return rc;
    }
    if ((rc = finish(h, s, h->st_host, w.st))) return rc;
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
    if (opt->keep_input_mask != 0)
        return fail(h, SOFIA_SC_EINVAL, "keep_input_mask must be 0 for a single step");
    if (opt->noise_plane_stride < 0 || opt->noise_plane_stride > (1 << 30))
        return fail(h, SOFIA_SC_EINVAL, "noise_plane_stride must be 0..2^30");
    if (opt->fuse_widths)
        return fail(h, SOFIA_SC_EINVAL, "fuse_widths is for sofia_sc_run / _run_ex only");
    return single_kernel(h, cube, nx, ny, nz, kernel, threshold, noise_mode, flux_range,
                         opt->replacement, opt->sigma0, mask_in, mask_out, noise, nullptr,
                         opt->storage, opt->stream, plane_stride(opt));
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

int sofia_sc_normalise(sofia_sc *h, const float *cube, int64_t nx, int64_t ny, int64_t nz,
                       int32_t window_xy, int32_t window_z, int32_t grid_xy, int32_t grid_z,
                       int32_t noise_mode, int32_t flux_range, float *out, double *noise_grid,
                       void *stream) {
    return normalise_impl(h, cube, nx, ny, nz, window_xy, window_z, grid_xy, grid_z,
                          noise_mode, flux_range, out, noise_grid, stream);
}

int sofia_sc_link(sofia_sc *h, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz,
                  int32_t radius_xy, int32_t radius_z, int32_t min_size_xy, int32_t min_size_z,
                  int32_t max_size_xy, int32_t max_size_z, int32_t *labels, int64_t *n_sources,
                  int64_t *boxes, int64_t box_capacity, void *stream) {
    return link_impl(h, mask, nx, ny, nz, radius_xy, radius_z, min_size_xy, min_size_z,
                     max_size_xy, max_size_z, labels, n_sources, boxes, box_capacity, stream);
}

int sofia_sc_check_run(int64_t nx, int64_t ny, int64_t nz, const sofia_sc_kernel *kernels,
                       int32_t n_kernels, double threshold, int32_t noise_mode,
                       int32_t flux_range, const sofia_sc_options *opt) {
    return validate_run(nullptr, nx, ny, nz, kernels, n_kernels, threshold, noise_mode,
                        flux_range, opt, nullptr);
}

void sofia_sc_param_defaults(sofia_sc_param_options *opt) {
    if (!opt) return;
    *opt = sofia_sc_param_options{};
    opt->struct_size = (int32_t)sizeof(sofia_sc_param_options);
    opt->channel_width = 1.0;
    opt->beam_major_px = 0.0;
    opt->beam_minor_px = 0.0;
    opt->sigma_rms = 1.0;
    opt->rel_scale = 0.4;
    opt->rel_threshold = 0.9;
    opt->snr_threshold = 2.8;
}

int sofia_sc_parameterise(sofia_sc *h, const float *cube, const int32_t *labels, int64_t nx,
                          int64_t ny, int64_t nz, int64_t n_sources,
                          const sofia_sc_param_options *opt, sofia_sc_source *out,
                          int64_t *n_kept, void *stream) {
    return param_impl(h, cube, labels, nx, ny, nz, n_sources, opt, out, n_kept, stream);
}

int sofia_sc_normalise_grid(int64_t nx, int64_t ny, int64_t nz, int32_t window_xy,
                            int32_t window_z, int32_t grid_xy, int32_t grid_z, int64_t *nbx,
                            int64_t *nby, int64_t *nbz) {
    if (!nbx || !nby || !nbz || nx < 1 || ny < 1 || nz < 1) return SOFIA_SC_EINVAL;
    if (grid_xy == 0) grid_xy = (window_xy + 1) / 2;
    if (grid_z == 0) grid_z = (window_z + 1) / 2;
    if (grid_xy < 1 || grid_z < 1) return SOFIA_SC_EINVAL;
    *nbx = (nx + grid_xy - 1) / grid_xy;
    *nby = (ny + grid_xy - 1) / grid_xy;
    *nbz = (nz + grid_z - 1) / grid_z;
    return SOFIA_SC_OK;
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
    return h ? h->err : "NULL handle";
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
