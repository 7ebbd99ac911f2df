// Internal interface between the host orchestration (sc_api.hip) and the
// gfx950 kernels (sc_kernels.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sofia_sc.h"

namespace sc {

// Working state of a run, packed one bit per voxel: word w of plane z holds
// columns 64w .. 64w+63 of that row-major plane (bit b = column 64w + b), so
// that a wave of 64 adjacent columns reads or writes one word per plane.
// Blank bits mark non-finite inputs (fixed for a run); detection bits mark
// the mask so far. The caller's byte mask only receives 0/1 at the end. In a
// kernel a voxel's working byte combines the two: kDet = detected so far,
// kBlank = blanked.
constexpr uint8_t kDet = 1;
constexpr uint8_t kBlank = 2;

// Histogram layout for the exact MAD selection on the bit pattern of |s|
// (a non-negative float's bits order like its value). Level 1 digit = bits
// 30..19 (4096 bins, counted in LDS); level 2 = bits 18..0 of the keys whose
// level-1 digit holds a wanted order statistic (2^19 bins in global memory,
// plus a coarse 1024-bin copy of bits 18..9 to speed up the rank walk).
constexpr int kL1Shift = 19;
constexpr int kL1Bins = 1 << 12;
constexpr int kL2Bins = 1 << 19;
constexpr int kL2CoarseShift = 9;
constexpr int kL2Coarse = 1 << 10;
constexpr int kL2Fine = 1 << kL2CoarseShift;

constexpr double kMadFactor = 1.4826;

// Device-resident state of one run: noise values and selection bookkeeping.
// Everything a later launch needs from an earlier one stays on the device,
// so a run makes no host round trip until the final copy of the noise.
struct DevState {
    double sigma0;          // noise of the unsmoothed input (replacement)
    double thr;             // current threshold t * sigma_k
    unsigned long long m;   // number of selected voxels (MAD)
    unsigned long long rank[2];  // residual ranks inside the level-1 bins
    uint32_t bin[2];        // level-1 bins holding ranks floor((m-1)/2), floor(m/2)
    int32_t status;         // nonzero: some noise had no selected voxel
    int32_t use_capture;    // order statistics resolved from the captured keys
    uint32_t klo, khi;      // captured key window [klo, khi] (bit patterns of |s|)
    unsigned long long below;  // selected keys below klo (capture path), else 0
    uint32_t cbin[2];       // level-2 coarse bins (bits 18..9) of the two ranks
    unsigned long long crank[2];  // residual ranks inside the coarse bins
    unsigned long long fallback;  // bit k: kernel k needed the full level-2 pass
    double scale;           // 16-bit storage: cube units per stored unit (sigma_0)
    double thr_lo, thr_hi;  // window the clip threshold t sigma_k lies in when the
                            // captured window holds the median (fused clip)
    int32_t fused_ok;       // fused clip valid: median captured, ambiguous list whole
    int32_t pad1;
    unsigned long long clip_fallback;  // bit k: kernel k needed the full clip pass
    double sigma[SOFIA_SC_MAX_KERNELS];
};

// A voxel whose clip decision the fused selection pass could not take yet:
// |s| lies in (thr_lo, thr_hi]. Decided once sigma_k is exact.
struct AmbEntry {
    uint64_t idx;           // voxel index z * nx * ny + y * nx + x
    double s;               // smoothed value, as the clip compares it
};

// Keys captured per wave in LDS before one bulk append to global memory:
// room for the flush threshold plus one whole group of planes (every lane
// of the wave may capture on every plane of a group).
constexpr int kCapFlushAt = 256;
constexpr int kCapPerWave(int group) { return kCapFlushAt + 64 * group; }
// Per-wave stride of that buffer: 64 more slots, one per lane, where lanes
// that capture nothing write (so the append needs no branch).
constexpr int kCapStride(int group) { return kCapPerWave(group) + 64; }
// Undecided voxels of the fused clip, per wave in LDS: flushed after a group
// of planes once more than kAmbFlushAt are held. A group of noise-like data
// adds well under one; a group that overflows the buffer sends the pass to
// the full clip.
constexpr int kAmbFlushAt = 64;
constexpr int kAmbPerWave = 160;

enum Src { SRC_X = 0, SRC_P = 1 };
enum Storage { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };
enum Op {
    OP_STD = 0, OP_HIST1 = 1, OP_HIST2 = 2, OP_CLIP = 3, OP_WRITE = 4, OP_SELECT = 5,
    OP_SELCLIP = 6   // OP_SELECT plus the clip for every voxel outside (thr_lo, thr_hi]
};

// Arguments of the column-streaming kernel (spectral boxcar + one of the
// per-voxel operations). One thread owns one (x, y) column and streams z.
struct ColArgs {
    const float *x;              // raw cube (SRC_X, ST_F32)
    const uint16_t *xq;          // raw cube stored as 16 bits (SRC_X, ST_F16/ST_BF16)
    int32_t xtype;               // Storage of the raw cube
    int32_t pad0;
    const float *p;              // spatially smoothed cube (SRC_P)
    const uint64_t *det_in;      // detection bits so far (null: none yet)
    const uint64_t *blank_in;    // blank bits (SRC_P; SRC_X tests its input)
    uint64_t *det_out;           // OP_CLIP / OP_SELCLIP: detection bits after this kernel
    uint64_t *blank_out;         // OP_CLIP / OP_SELCLIP on SRC_X: blank bits out (may be null)
    int64_t wpp;                 // 64-bit words per plane of the bit planes
    float *s_out;                // OP_WRITE output
    int64_t ncol;                // nx * ny
    int64_t nz;
    int32_t w, h;                // spectral width (odd >= 3, or 1) and (w-1)/2
    int32_t zchunk;              // planes per block
    int32_t ncb;                 // column blocks
    int32_t range;               // -1 negative, 0 all, +1 positive
    int32_t repl_on;             // replace detected voxels (SRC_X only)
    double repl_n;               // n of +-n sigma0
    DevState *st;
    double *part_sum;            // OP_STD per-block partials
    unsigned long long *part_cnt;
    unsigned long long *hist1;   // [kL1Bins]
    unsigned long long *hist2;   // [2][kL2Bins]
    unsigned long long *hist2c;  // [2][kL2Coarse]
    int32_t cb_stride;           // column blocks visited: every cb_stride-th
    int32_t skip_if_captured;    // OP_HIST1/2: do nothing when st->use_capture
    uint32_t *cap_buf;           // OP_SELECT: captured keys
    unsigned long long *cap_count;
    unsigned long long cap_capacity;
    unsigned long long *sel_part;    // OP_SELECT / OP_SELCLIP: per block [selected voxels,
                                     // keys below klo], 2 per block
    AmbEntry *amb;               // OP_SELCLIP: undecided voxels
    unsigned long long *amb_count;
    unsigned long long amb_capacity;
    int32_t skip_if_fused;       // OP_CLIP: do nothing when st->fused_ok
    int32_t zstride;             // noise passes select voxels of every zstride-th plane only
};

// Arguments of the strip-streaming spatial kernel. A strip is 128 adjacent
// columns of one plane (128 - 2H of them output columns, H = n r); a wave
// streams one chunk of `rows` rows of it.
struct StripArgs {
    const float *x;              // raw cube (ST_F32)
    const uint16_t *xq;          // raw cube stored as 16 bits (ST_F16 / ST_BF16)
    const uint64_t *det;         // packed detection bits (replacement only)
    int64_t wpp;                 // 64-bit words per plane of det
    float *p;                    // output: spatially smoothed cube
    int64_t nx, ny, nz;
    int32_t nstrips;             // strips across x
    int32_t wpb;                 // strips (waves) per workgroup
    int32_t ngroups;             // workgroups across x: ceil(nstrips / wpb)
    int32_t rows;                // output rows per chunk
    int32_t nchunks;             // chunks per plane
    int32_t pad;
    int64_t tiles;               // workgroups: ngroups * nchunks * nz
    double repl_n;               // n of +-n sigma_0
    const DevState *st;
};

// Arguments of the fused spectral-widths passes (sc_multi.hip): the widths
// w[i] (half-widths h[i], kernel indices k[i]) that share one source: the raw
// cube (SRC_X) or one spatial kernel's smoothed cube (SRC_P).
constexpr int kMultiMax = 8;
constexpr int kMultiStage = 256;     // captured keys staged per wave and width (MAD)
enum MultiOp { MOP_STATS = 0, MOP_CLIP = 1, MOP_SELECT = 2 };
struct MultiArgs {
    const float *src;
    const uint64_t *blank;           // blank bits (SRC_P)
    const uint64_t *det_in;          // CLIP: detection bits so far (null: none; may equal det_out)
    uint64_t *det_out;               // CLIP: detection bits out
    int64_t wpp;                     // 64-bit words per plane of the bit planes
    DevState *st;
    double *part_sum;                // [nw][nparts]
    unsigned long long *part_cnt;    // [nw][nparts]
    int64_t ncol, nz;
    int32_t ncb, zchunk, nparts;
    int32_t nw, hmax, range, zstride;
    double t;
    int32_t w[kMultiMax], h[kMultiMax], k[kMultiMax];
    // MOP_SELECT (MAD): every width's own state (its predicted key window),
    // capture list and count, and per-block counts [nparts][2]
    DevState *sti[kMultiMax];
    uint32_t *cap[kMultiMax];
    unsigned long long *cap_count[kMultiMax];
    unsigned long long cap_capacity;
    unsigned long long *sel_part[kMultiMax];
};

hipError_t launch_multi(int src, int mop, const MultiArgs &a, int nblocks, hipStream_t s);
hipError_t launch_multi_finalize(const MultiArgs &a, hipStream_t s);
// Every width's noise (and status, fallback bits) from its own state into st.
hipError_t launch_multi_gather(const MultiArgs &a, hipStream_t s);

// Arguments of the sampled-Gaussian spatial kernel (sc_gauss.h): strips of
// kGaussCols output columns, chunks of `rows` rows. tf / td hold the taps at
// distance 0..R (the kernel is symmetric) in FP32 (x pass) and FP64 (y pass).
constexpr int kGaussMaxR = SOFIA_SC_GAUSS_MAX_RADIUS;
constexpr int kGaussCols = 256;      // output columns per strip = threads per workgroup
struct GaussArgs {
    const float *x;              // raw cube (ST_F32)
    const uint16_t *xq;          // raw cube stored as 16 bits (ST_F16 / ST_BF16)
    const uint64_t *det;         // packed detection bits (replacement only)
    int64_t wpp;                 // 64-bit words per plane of det
    float *p;                    // output: spatially smoothed cube
    int64_t nx, ny, nz;
    int32_t nstrips, rows, nchunks, pad;
    int64_t tiles;               // workgroups: nstrips * nchunks * nz
    double repl_n;               // n of +-n sigma_0
    const DevState *st;
    float tf[kGaussMaxR + 1];
    double td[kGaussMaxR + 1];
};

// Taps (distance 0..R, normalised over -R..R) and grid of a sampled Gaussian.
int gauss_radius(double fwhm);
void gauss_setup(GaussArgs &a, double fwhm, int rows_max);
hipError_t launch_gauss(int radius, int xtype, bool repl, const GaussArgs &a, hipStream_t s);
template <int R>
hipError_t launch_gauss_r(const GaussArgs &a, int xtype, bool repl, hipStream_t s);

// Arguments of the local noise normalisation (sc_norm.hip). The noise is
// measured per block of a grid (gxy x gxy x gz voxels) in a window of
// wxy x wxy x wz voxels around the block's centre; every voxel of a block is
// then divided by that noise.
struct NormArgs {
    const float *x;              // input cube
    float *y;                    // normalised cube (may equal x)
    double *sigma;               // [nbz][nby][nbx] noise per block
    int64_t nx, ny, nz;
    int32_t wxy, wz;             // window sizes (odd)
    int32_t gxy, gz;             // grid steps
    int32_t nbx, nby, nbz;       // blocks per axis
    int32_t range;               // -1 negative, 0 all, +1 positive
};

// Threads of the windowed-noise kernel.
constexpr int kNormThreads = 512;
constexpr int kNormStage = 4096;     // keys of the median's level-1 bin staged in LDS

hipError_t launch_window_noise(int mode, const NormArgs &a, hipStream_t s);
hipError_t launch_norm_divide(const NormArgs &a, hipStream_t s);

// Arguments of the linker (sc_link.hip). L is the caller's int32 label cube,
// used as the union-find forest; off[] holds the forward half of the
// friends' offsets, each packed as (dx + 128) | (dy + 128) << 8 | (dz + 128) << 16.
constexpr int kLinkMaxOffsets = 160;
struct LinkArgs {
    const uint8_t *mask;
    int *L;
    int *list;                   // [m]: the detected voxels' indices, in raster order
    int64_t m;                   // detected voxels
    int *box;                    // [nc][8]: x0, x1, y0, y1, z0, z1, count, pad
    int *label_of;               // [nc]: label of each detection, 0 = dropped
    int64_t nx, ny, nz;
    int32_t min_xy, min_z, max_xy, max_z;
    int32_t n_off;
    int32_t off[kLinkMaxOffsets];
    int32_t delta[kLinkMaxOffsets];   // index difference of each offset
};

// Over the list of detected voxels (a.list, a.m entries).
hipError_t launch_link_init(const LinkArgs &a, hipStream_t s);
hipError_t launch_link_union(const LinkArgs &a, hipStream_t s);
hipError_t launch_link_flatten(const LinkArgs &a, hipStream_t s);
// Blocks of the count / assign steps over n items.
int64_t link_scan_blocks(int64_t n);
// Items of the count / assign steps: the cube's voxels (detected ones go to
// the list), the listed voxels (roots get their detection's number), or the
// detections (kept ones get their label).
enum LinkItems { LK_VOXELS = 0, LK_ROOTS = 1, LK_KEPT = 2 };
// Count flagged items per block and scan the counts in place; counts[blocks]
// receives the total.
hipError_t launch_link_number(int items, const LinkArgs &a, int64_t n, int *counts,
                              hipStream_t s);
hipError_t launch_link_assign(int items, const LinkArgs &a, int64_t n, const int *counts,
                              hipStream_t s);
hipError_t launch_link_resolve(const LinkArgs &a, int64_t nc, hipStream_t s);
hipError_t launch_link_label(const LinkArgs &a, hipStream_t s);
hipError_t launch_link_boxes_out(const LinkArgs &a, int64_t nc, long long *out, hipStream_t s);

// Parameterisation and reliability (sc_param.hip). Per-detection
// accumulators: voxel count, FP64 sums of the value and of value x position,
// and the order-keeping integer images of the largest and smallest value.
struct SrcAcc {
    unsigned long long count;
    double sum, sx, sy, sz;
    int peak, mn;
};
struct ParamArgs {
    const float *cube;
    const int *labels;
    int64_t nx, ny, nz;
    int64_t plane;                   // nx * ny
    int64_t n;                       // detections 1..n
    double channel_width, omega, sigma_rms;
    double scale, rel_threshold, snr_threshold;
    SrcAcc *acc;                     // [n]
    int *sign;                       // [n]: +1 / -1 / 0 by the sign of the sum
    double *vec;                     // [n][3]: log10 parameter vectors
    double *rel_state;               // [10]: inverse covariance, valid flag
    unsigned long long *n_kept;      // count of kept detections
    sofia_sc_source *out;            // [n]
    int vec4;                        // labels 16-byte aligned: 4 voxels per load
};

hipError_t launch_parameterise(const ParamArgs &a, hipStream_t s);
hipError_t launch_reliability(const ParamArgs &a, hipStream_t s);

// ---- launchers (sc_kernels.hip). Each returns the launch's hipError_t.
// Blank bits of the cube x (non-finite voxels) and, when mask_in is given,
// its nonzero finite voxels as detection bits (det may be null otherwise).
hipError_t launch_init_bits(const float *x, const uint8_t *mask_in, uint64_t *blank,
                            uint64_t *det, int64_t ncol, int64_t nz, int64_t wpp,
                            hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, hipStream_t s);
// The caller's mask from detection bits: mask = bit (keep = 0), mask |= bit
// (keep = 1), or, with a source mask src (not aliasing mask), mask = bit |
// (src != 0).
hipError_t launch_write_mask(const uint64_t *det, uint8_t *mask, int keep, const uint8_t *src,
                             int64_t ncol, int64_t nz, int64_t wpp, hipStream_t s);
// Spatial cascade of n_iter boxcars of radius r per axis into a.p.
hipError_t launch_spatial(int n_iter, int radius, int xtype, bool repl,
                          const StripArgs &a, hipStream_t s);
template <int R, int NIT>
hipError_t launch_strip(const StripArgs &a, int xtype, bool repl, hipStream_t s);
hipError_t launch_column(int src, int op, bool spectral, const ColArgs &a, int nblocks,
                         hipStream_t s);
hipError_t launch_finalize_std(DevState *st, const double *part_sum,
                               const unsigned long long *part_cnt, int nparts,
                               int k, double t, int also_sigma0, hipStream_t s);
hipError_t launch_finalize_mad1(DevState *st, const unsigned long long *hist1,
                                hipStream_t s);
hipError_t launch_finalize_select(DevState *st, const unsigned long long *sel_part, int nparts,
                                  const unsigned long long *cap_count,
                                  unsigned long long cap_capacity, int k,
                                  const unsigned long long *amb_count,
                                  unsigned long long amb_capacity, hipStream_t s);
// Walks over the captured keys run on `blocks` workgroups (grid-stride).
hipError_t launch_capture_l1(const DevState *st, const uint32_t *cap_buf,
                             const unsigned long long *cap_count,
                             unsigned long long *hist1, int blocks,
                             hipStream_t s);
hipError_t launch_finalize_predict(DevState *st, const unsigned long long *hist_s,
                                   double t, hipStream_t s);
// After sigma_k is exact: decide the voxels the fused selection pass left
// undecided (when st->fused_ok), into the detection bits.
hipError_t launch_clip_fixup(const DevState *st, const AmbEntry *amb,
                             const unsigned long long *amb_count,
                             unsigned long long amb_capacity, uint64_t *det_out, int64_t ncol,
                             int64_t wpp, hipStream_t s);
hipError_t launch_capture_coarse(const DevState *st, const uint32_t *cap_buf,
                                 const unsigned long long *cap_count,
                                 unsigned long long *hist2c, int blocks,
                             hipStream_t s);
hipError_t launch_capture_fine(const DevState *st, const uint32_t *cap_buf,
                               const unsigned long long *cap_count,
                               unsigned long long *hist2, int blocks,
                             hipStream_t s);
hipError_t launch_finalize_mad2a(DevState *st, const unsigned long long *hist2c,
                                 hipStream_t s);
hipError_t launch_finalize_mad2b(DevState *st, const unsigned long long *hist2, int k,
                                 double t, int also_sigma0, hipStream_t s);
hipError_t launch_set_sigma0(DevState *st, double sigma0, hipStream_t s);
// 16-bit noise-scaled copy; scale = st->sigma0 when st != null, else `scale`.
hipError_t launch_quantize(const float *x, const DevState *st, double scale, int type,
                           uint16_t *out, int64_t n, hipStream_t s);
// After quantisation: keep sigma_0 as the scale and continue in scaled units.
hipError_t launch_enter_scaled(DevState *st, hipStream_t s);

// Threads per block of the column kernel, and its dynamic LDS size.
constexpr int kColThreads = 256;
size_t column_lds_bytes(int src, int op, bool spectral, int w);

// The spatial kernel's wave covers a strip of kStripCols columns (two per
// lane); a workgroup holds the waves of up to kStripWaves adjacent strips of
// the same rows, which stage each row's span once in LDS.
constexpr int kStripCols = 128;
constexpr int kStripWaves = 4;

// Launch shapes of a run: the column kernel's grid aims at col_blocks
// blocks (z split into chunks of at least col_min_planes planes); the spatial
// kernel's row chunks hold at most strip_rows rows, and its workgroups hold
// up to strip_waves adjacent strips (1 .. kStripWaves).
struct Shapes {
    int col_blocks = 6144;
    int strip_rows = 256;
    int strip_waves = kStripWaves;
    int col_min_planes = 64;
};

// Strip geometry of the spatial kernel for a cube of width nx and halo H:
// strips of kStripCols - 2H output columns, up to waves_max adjacent strips
// per workgroup (spread evenly over the groups a row needs), rows in chunks
// of at most rows_max (>= 32).
inline void spatial_strips(StripArgs &a, int n_iter, int radius, int rows_max,
                           int waves_max = kStripWaves) {
    const int64_t H = (int64_t)n_iter * radius, W = kStripCols - 2 * H;
    const int64_t wmax = waves_max < 1 ? 1 : (waves_max > kStripWaves ? kStripWaves : waves_max);
    a.nstrips = (int32_t)((a.nx + W - 1) / W);
    const int64_t groups = (a.nstrips + wmax - 1) / wmax;
    a.wpb = (int32_t)((a.nstrips + groups - 1) / groups);
    a.ngroups = (int32_t)((a.nstrips + a.wpb - 1) / a.wpb);
    // rows per chunk: long chunks keep the y halo small; shorter ones when
    // the cube is too small to give the chip enough waves otherwise
    int64_t rows = rows_max;
    while (rows > 32 && a.nstrips * ((a.ny + rows - 1) / rows) * a.nz < 16384) rows /= 2;
    if (rows > a.ny) rows = a.ny;
    a.rows = (int32_t)rows;
    a.nchunks = (int32_t)((a.ny + rows - 1) / rows);
    a.tiles = (int64_t)a.ngroups * a.nchunks * a.nz;
}

}  // namespace sc
