/*
 * sofia_sc.h -- C ABI of the MI355X smooth-and-clip (S+C) source finder.
 *
 * S+C is the default source finder of SoFiA 2 (Westmeier et al. 2021,
 * arXiv:2106.15789, Sect. 4.2): the cube is smoothed with a list of spatial x
 * spectral kernels; after each smoothing the noise of the smoothed cube is
 * measured and every voxel whose absolute value exceeds threshold x noise is
 * added to one binary mask (positive and negative excursions alike, Sect. 4.2).
 * Before each smoothing, voxels already in the mask are replaced by +-n times
 * the noise of the input, keeping their sign (Sect. 6.2.4, default n = 2).
 * Spatial kernels are Gaussians given by FWHM in pixels, spectral kernels are
 * boxcars given by width in channels (Fig. 9 caption; kernel sets in Sects. 5
 * and 6). The robust noise is 1.4826 x the median absolute value (the MAD
 * estimator of Sect. 4.1, taken about zero).
 *
 * Conventions for every entry point:
 *  - Cubes are float32 [nz][ny][nx] (x fastest, z = spectral axis slowest),
 *    dense and contiguous. Masks are uint8 of the same shape: 1 = detected,
 *    0 = not detected. Non-finite voxels are "blanked": they count as 0 in the
 *    smoothing, never enter the noise and are never detected.
 *  - Pointers named cube/mask/out are DEVICE pointers on the handle's device;
 *    pointers named noise/sigma0/stats are HOST pointers. The caller owns all
 *    of them; the library keeps none after the call returns.
 *  - Work is enqueued on the given stream (NULL = the null stream); calls
 *    return after the work has completed, since results land in host memory.
 *  - Return 0 on success or a negative SOFIA_SC_E* code. On error every
 *    host noise value is set to NaN, sofia_sc_last_error() describes the
 *    cause and the handle stays usable.
 *  - A handle is not thread-safe: use one handle per host thread.
 */
#ifndef SOFIA_SC_H
#define SOFIA_SC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sofia_sc sofia_sc;

/* One smoothing kernel. spatial_fwhm_px = 0 means no spatial smoothing.
 * Otherwise the spatial Gaussian (Fig. 9 caption, Sect. 5) is built as set
 * by spatial_kind:
 *  SOFIA_SC_SPATIAL_CASCADE (0): a cascade of n boxcars of width 2r+1 along
 *    x and then along y (see sofia_sc_plan), halo n r <= SOFIA_SC_MAX_HALO;
 *  SOFIA_SC_SPATIAL_GAUSS (1): the Gaussian sampled at integer offsets
 *    |k| <= R = floor(4 sigma + 1/2), sigma = FWHM / (2 sqrt(2 ln 2)),
 *    normalised to sum 1, along x and then along y, zero outside the cube;
 *    R <= SOFIA_SC_GAUSS_MAX_RADIUS (FWHM up to about 14 px); R = 0 means
 *    no spatial smoothing.
 * spectral_width_ch = 0 or 1 means no spectral smoothing; other widths must
 * be odd and >= 3. Zero-initialise the struct: spatial_kind must be 0 or 1. */
enum { SOFIA_SC_SPATIAL_CASCADE = 0, SOFIA_SC_SPATIAL_GAUSS = 1 };
#define SOFIA_SC_GAUSS_MAX_RADIUS 24
typedef struct {
    double spatial_fwhm_px;
    int32_t spectral_width_ch;
    int32_t spatial_kind;
} sofia_sc_kernel;

enum { SOFIA_SC_NOISE_STD = 0, SOFIA_SC_NOISE_MAD = 1 };

/* Storage of the cube inside a run. F32 reads the caller's cube directly.
 * F16 / BF16 first measure sigma_0 (or take opt->sigma0), then store the
 * noise-scaled cube q = x / sigma_0 once, rounded to the 16-bit format, and
 * run every pass on q: half the input bytes per pass; all arithmetic stays
 * FP32 (smoothing) and FP64 (sums, noise). See sofia_sc_quantize. */
enum { SOFIA_SC_STORE_F32 = 0, SOFIA_SC_STORE_F16 = 1, SOFIA_SC_STORE_BF16 = 2 };
enum { SOFIA_SC_FLUX_NEGATIVE = -1, SOFIA_SC_FLUX_ALL = 0, SOFIA_SC_FLUX_POSITIVE = 1 };

enum {
    SOFIA_SC_OK = 0,
    SOFIA_SC_EINVAL = -1,   /* bad argument (see each entry point) */
    SOFIA_SC_ENOMEM = -2,   /* device allocation failed */
    SOFIA_SC_EDEVICE = -3,  /* HIP error; text via sofia_sc_last_error */
    SOFIA_SC_ENOSTAT = -4   /* a noise had no finite voxel in its flux range:
                               that noise is NaN and the mask is undefined */
};

/* Limits of this build. */
#define SOFIA_SC_MAX_KERNELS 64
#define SOFIA_SC_MAX_HALO 16        /* n * r of the spatial cascade */
#define SOFIA_SC_MAX_WIDTH 63       /* spectral boxcar width */
#define SOFIA_SC_MAX_CUBES 4096     /* cubes of one batch */
#define SOFIA_SC_MAX_PLANE (1LL << 28)  /* nx * ny */

typedef struct {
    uint32_t struct_size;   /* = sizeof(sofia_sc_options) */
    double replacement;     /* n of +-n sigma_0 (Sect. 6.2.4); < 0 disables
                               replacement; default 2.0 */
    double sigma0;          /* noise of the unsmoothed input used for
                               replacement and 16-bit scaling: NaN = measure
                               it (default); finite > 0 = use as given */
    int32_t storage;        /* SOFIA_SC_STORE_*; default F32 */
    int32_t keep_input_mask;  /* 0: the mask is fully overwritten with 0/1
                               (default); 1: mask[i] |= 1 where the run
                               detects, every other byte keeps its value (the
                               caller's mask takes no part in the run) */
    int32_t noise_plane_stride; /* noise subsampling: every noise (sigma_0 and
                               each sigma_k) is measured on the planes
                               z = 0, s, 2s, ... only; every voxel is still
                               smoothed and clipped. 0 or 1 (default): every
                               plane, the whole cube */
    int32_t fuse_widths;    /* 1: with replacement off (replacement < 0) the
                               pairs are independent; the pairs that share a
                               spatial kernel then share their passes: one
                               pass computes every spectral width's smoothed
                               values and its RMS partials (or, for MAD, its
                               counts and captured keys around its predicted
                               median), then every width's noise, then one
                               pass clips every width (ORed into the mask).
                               Same results as 0 up to the last bits of the
                               smoothed values and the summation order of the
                               RMS. Needs FP32 storage (sofia_sc_run / _run_ex
                               only; EINVAL otherwise). 0 (default): one pair
                               at a time */
    void *stream;           /* hipStream_t to run on; NULL = null stream */
} sofia_sc_options;

/* Fill opt with defaults (replacement 2.0, sigma0 measured, F32 storage,
 * mask overwritten, null stream). */
void sofia_sc_default_options(sofia_sc_options *opt);

/* Create a handle on a HIP device. The handle owns all device workspace
 * (packed blank and detection bits, smoothed-plane buffer, histograms);
 * workspace grows on demand and is released by sofia_sc_destroy. EINVAL for
 * a bad ordinal. */
int sofia_sc_create(sofia_sc **out, int device_ordinal);

/* Release a handle and its workspace. NULL is a no-op. */
void sofia_sc_destroy(sofia_sc *h);

/* Whole S+C run (Sect. 4.2) over n_kernels kernels, in list order.
 *  cube       device, float32 [nz][ny][nx], read only.
 *  kernels    host array of n_kernels (1..SOFIA_SC_MAX_KERNELS).
 *  threshold  t > 0: a voxel is detected when |s| > t * noise_k.
 *  noise_mode SOFIA_SC_NOISE_STD (RMS about zero) or SOFIA_SC_NOISE_MAD.
 *  flux_range which smoothed voxels enter the noise: NEGATIVE (s < 0),
 *             ALL (every finite s) or POSITIVE (s > 0).
 *  mask       device, uint8 [nz][ny][nx], fully overwritten with 0/1.
 *  noise      host, double[n_kernels]: the noise of each smoothed cube.
 * Uses the default options. EINVAL: NULL pointer, a dimension < 1,
 * nx*ny*nz > 2^40, nx*ny > SOFIA_SC_MAX_PLANE, bad kernel (FWHM < 0 or non-finite, halo above
 * SOFIA_SC_MAX_HALO, even or too large width), bad threshold or enum. */
int sofia_sc_run(sofia_sc *h, const float *cube, int64_t nx, int64_t ny,
                 int64_t nz, const sofia_sc_kernel *kernels, int32_t n_kernels,
                 double threshold, int32_t noise_mode, int32_t flux_range,
                 uint8_t *mask, double *noise);

/* sofia_sc_run with options. sigma0 (host, may be NULL) receives the noise
 * of the unsmoothed input that replacement and 16-bit scaling use (NaN when
 * neither needs it). Noise values are always in the cube's own units.
 * EINVAL also for opt == NULL, a struct_size mismatch, an unknown storage,
 * keep_input_mask not 0 or 1, or a given sigma0 that is not finite and > 0. */
int sofia_sc_run_ex(sofia_sc *h, const float *cube, int64_t nx, int64_t ny,
                    int64_t nz, const sofia_sc_kernel *kernels,
                    int32_t n_kernels, double threshold, int32_t noise_mode,
                    int32_t flux_range, uint8_t *mask, double *noise,
                    const sofia_sc_options *opt, double *sigma0);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture of their own work around the call, tight serving loops, harnesses
 * that forbid hipMalloc. The same whole run as sofia_sc_run_ex (same
 * arguments, options, results and errors, bit for bit), but no device or
 * pinned-host allocation and no allocating library call: the workspace is a
 * fixed device array of SOFIA_SC_NOALLOC_SCRATCH_BYTES that the library holds
 * on every device it runs on until the process ends (its address is taken
 * once per device by sofia_sc_create). The result copy goes to the caller's
 * pageable host memory, and the call returns after the work has completed.
 * Every call on one GPU shares that GPU's array, whatever the handle: calls
 * that overlap on one GPU (two host threads, or two streams) race and must
 * not be made. Profiling (sofia_sc_profile) records nothing for these calls.
 * EINVAL as sofia_sc_run_ex, and for a cube of more than
 * SOFIA_SC_NOALLOC_MAX_VOXELS voxels or a shape whose workspace exceeds the
 * array (very tall, thin cubes): the message says which. */
#define SOFIA_SC_NOALLOC_MAX_VOXELS (1LL << 22)
#define SOFIA_SC_NOALLOC_SCRATCH_BYTES (64LL << 20)
int sofia_sc_run_noalloc(sofia_sc *h, const float *cube, int64_t nx, int64_t ny,
                         int64_t nz, const sofia_sc_kernel *kernels,
                         int32_t n_kernels, double threshold, int32_t noise_mode,
                         int32_t flux_range, uint8_t *mask, double *noise,
                         const sofia_sc_options *opt, double *sigma0);

/* One cube of a batch: device pointers, owned by the caller. */
typedef struct {
    const float *cube;      /* float32 [nz][ny][nx], read only */
    int64_t nx, ny, nz;
    uint8_t *mask;          /* uint8 [nz][ny][nx], fully overwritten with 0/1 */
} sofia_sc_cube;

/* Independent S+C runs (Sect. 4.2) of many cubes with one kernel list,
 * threshold, noise mode, flux range and options: the result for each cube is
 * the one sofia_sc_run_ex gives for it alone (every cube measures its own
 * sigma_0 and noise; a given opt->sigma0 applies to every cube). The cubes
 * are spread over a few workspaces whose launch chains run concurrently;
 * the whole batch is captured once into a HIP graph and launched as one
 * graph on opt->stream. An identical later call (same cube and mask
 * pointers, shapes, kernels and settings) launches the same graph again
 * without capturing. Inputs must be ready on opt->stream. The cached graph
 * refers to the cube and mask pointers of the call that captured it; it is
 * destroyed by the next batch call with other arguments and by
 * sofia_sc_destroy, and is never launched again with freed buffers.
 *  cubes    host array of n_cubes (1..SOFIA_SC_MAX_CUBES) descriptors; the
 *           masks must be distinct and must not overlap any cube.
 *  noise    host, double[n_cubes][n_kernels] (cube-major).
 *  sigma0   host, double[n_cubes] or NULL: as sofia_sc_run_ex per cube.
 * Returns after the work has completed. EINVAL as sofia_sc_run_ex (the
 * message names the cube), and for n_cubes out of range or two cubes with
 * one mask. ENOSTAT when any cube has a noise without voxels: every other
 * value is still filled in. */
int sofia_sc_run_batch(sofia_sc *h, const sofia_sc_cube *cubes, int32_t n_cubes,
                       const sofia_sc_kernel *kernels, int32_t n_kernels, double threshold,
                       int32_t noise_mode, int32_t flux_range, double *noise,
                       const sofia_sc_options *opt, double *sigma0);

/* Launch shapes of the runs of a handle (batched and single). */
typedef struct {
    int32_t lanes;          /* batches: workspaces whose launch chains run side
                               by side: 4, 8 or 16 (default 8) */
    int32_t col_blocks;     /* column passes: blocks a launch aims at, by
                               splitting z into chunks: 3072, 6144 or 12288
                               (default 6144); whatever it is, no chunk is
                               longer than 1024 planes */
    int32_t strip_rows;     /* spatial pass: most rows per chunk of a strip:
                               64, 128 or 256 (default 256) */
    int32_t strip_waves;    /* spatial pass: most adjacent 128-column strips
                               (waves) per workgroup, which stage their rows
                               once in LDS: 1, 2 or 4 (default 4) */
    int32_t col_min_planes; /* column passes: fewest planes per z chunk (the
                               spectral halo is re-read per chunk): 32, 64 or
                               128 (default 64) */
    int32_t reserved;
    double ms;              /* time of one batched run with these shapes as
                               measured by the tuning (NaN if not tuned) */
} sofia_sc_batch_tuning;

/* SWITCHED OFF IN THIS BUILD: returns SOFIA_SC_EDEVICE at once (best, if
 * not NULL, receives the handle's current shapes). Timing candidate shapes
 * through repeated graph captures crashed the process when it ran after
 * other batched calls in the same process, for a reason not established.
 * Batches use the handle's shapes, which sofia_sc_tune_run and
 * sofia_sc_set_shapes set. */
int sofia_sc_tune_batch(sofia_sc *h, const sofia_sc_cube *cubes, int32_t n_cubes,
                        const sofia_sc_kernel *kernels, int32_t n_kernels, double threshold,
                        int32_t noise_mode, int32_t flux_range, const sofia_sc_options *opt,
                        sofia_sc_batch_tuning *best);

/* Autotune the launch shapes of whole runs (Sect. 4.2) on the caller's cube:
 * candidate shapes are timed one parameter at a time (col_blocks,
 * strip_rows, strip_waves, then col_min_planes; each candidate as the faster
 * of two sofia_sc_run_ex calls after an untimed one; no graph is captured)
 * and the fastest are kept in the handle: every later sofia_sc_run*,
 * sofia_sc_step*, sofia_sc_smooth and sofia_sc_run_batch call of the handle
 * uses them (lanes are left as they are). Results do not depend on the
 * shapes except for the last bits of std noise (summation order of the
 * per-block partials). Arguments as sofia_sc_run_ex; mask is written with
 * the run's result for the chosen shapes; best (host, may be NULL) receives
 * the chosen shapes and their time. Returns as sofia_sc_run_ex; on error the
 * handle keeps its previous shapes. */
int sofia_sc_tune_run(sofia_sc *h, const float *cube, int64_t nx, int64_t ny, int64_t nz,
                      const sofia_sc_kernel *kernels, int32_t n_kernels, double threshold,
                      int32_t noise_mode, int32_t flux_range, uint8_t *mask,
                      const sofia_sc_options *opt, sofia_sc_batch_tuning *best);

/* Set the handle's launch shapes (each field one of the candidates listed in
 * sofia_sc_batch_tuning; ms is ignored), or the defaults for shapes == NULL.
 * EINVAL for a value outside the candidates. No device work. */
int sofia_sc_set_shapes(sofia_sc *h, const sofia_sc_batch_tuning *shapes);

/* The handle's current launch shapes. EINVAL for NULL. */
int sofia_sc_get_shapes(const sofia_sc *h, sofia_sc_batch_tuning *shapes);

/* One S+C iteration with the previous state given (Sect. 4.2 and 6.2.4):
 * smooth the cube after replacing the voxels set in mask_in by
 * copysign(replacement * sigma0, x) (skipped when replacement < 0), measure
 * the noise, and write mask_out = mask_in OR (|s| > t * noise).
 *  mask_in    device, uint8 0/1 (may be NULL: no previous detections).
 *  mask_out   device, uint8, fully overwritten; must not alias mask_in.
 *  noise      host, double[1].
 *  stream     hipStream_t or NULL. */
int sofia_sc_step(sofia_sc *h, const float *cube, int64_t nx, int64_t ny,
                  int64_t nz, sofia_sc_kernel kernel, double threshold,
                  int32_t noise_mode, int32_t flux_range, double replacement,
                  double sigma0, const uint8_t *mask_in, uint8_t *mask_out,
                  double *noise, void *stream);

/* sofia_sc_step with options: opt->replacement, opt->sigma0 and opt->stream
 * take the place of the replacement, sigma0 and stream arguments, and
 * opt->storage selects the storage as in sofia_sc_run_ex. With F16/BF16 the
 * cube is stored as a run stores it, scaled by opt->sigma0, which must then
 * be given (finite and > 0); the noise is returned in the cube's own units.
 * EINVAL as sofia_sc_step, and for opt == NULL, a struct_size mismatch, an
 * unknown storage or a nonzero keep_input_mask (mask_in / mask_out give a
 * step its state explicitly). */
int sofia_sc_step_ex(sofia_sc *h, const float *cube, int64_t nx, int64_t ny,
                     int64_t nz, sofia_sc_kernel kernel, double threshold,
                     int32_t noise_mode, int32_t flux_range, const uint8_t *mask_in,
                     uint8_t *mask_out, double *noise, const sofia_sc_options *opt);

/* The smoothed cube s of one kernel, as float32 (NaN at blanked voxels),
 * with replacement applied as in sofia_sc_step. out: device, float32
 * [nz][ny][nx]. For inspection and tests; S+C itself never stores s. */
int sofia_sc_smooth(sofia_sc *h, const float *cube, int64_t nx, int64_t ny,
                    int64_t nz, sofia_sc_kernel kernel, double replacement,
                    double sigma0, const uint8_t *mask_in, float *out,
                    void *stream);

/* Noise-scaled 16-bit copy of a cube, exactly as a F16/BF16 run stores it:
 * q = RN_T( RN_f32( x * RN_f64(1 / scale) ) ), RN = round to nearest even,
 * T = binary16 (SOFIA_SC_STORE_F16) or bfloat16 (SOFIA_SC_STORE_BF16); finite
 * values beyond T's range saturate to its largest finite value; NaN and Inf
 * stay non-finite (blanked). cube: device float32[n]; out: device
 * uint16[n] (bit patterns). EINVAL: NULL, n < 1, scale not finite and > 0,
 * storage not F16/BF16. */
int sofia_sc_quantize(sofia_sc *h, const float *cube, int64_t n, double scale,
                      int32_t storage, uint16_t *out, void *stream);

/* Local noise normalisation (Sect. 4.1, last paragraph: where the noise
 * level is not constant, the cube is divided by the noise measured in a
 * running window before a constant threshold is applied; the speed test of
 * Sect. 5 uses a window of 31 pixels and 31 channels). The noise is measured
 * on a grid: each axis is cut into blocks of grid voxels (the last block may
 * be shorter); the window of a block is window voxels centred on the block's
 * middle voxel (the lower middle for an even block length), clipped to the
 * cube, spatial windows square (window_xy in x and y) and window_z long; its
 * noise uses the smooth-and-clip estimators over the finite voxels of the
 * flux range (RMS about zero, or 1.4826 x the median of |v| with the mean of
 * the two central order statistics for an even count). Every voxel of a
 * block is then divided by that noise in FP64 and rounded to float32;
 * non-finite voxels, and every voxel of a block whose noise is not finite
 * and > 0 (no voxel selected, or zero noise), become NaN (blanked).
 *  cube        device, float32 [nz][ny][nx], read only (unless out == cube).
 *  window_xy, window_z  odd window sizes, 1..SOFIA_SC_NORM_MAX_WINDOW.
 *  grid_xy, grid_z  block sizes; 0 = (window + 1) / 2 (windows of adjacent
 *              blocks then overlap by about half).
 *  out         device, float32 [nz][ny][nx] or NULL (noise grid only); may
 *              equal cube (in place).
 *  noise_grid  host, double [nbz][nby][nbx] (sofia_sc_normalise_grid gives
 *              the counts) or NULL.
 * Returns after the work has completed. EINVAL for NULL cube, both outputs
 * NULL, bad dimensions, windows, grid steps or enums. */
#define SOFIA_SC_NORM_MAX_WINDOW 255
int sofia_sc_normalise(sofia_sc *h, const float *cube, int64_t nx, int64_t ny, int64_t nz,
                       int32_t window_xy, int32_t window_z, int32_t grid_xy, int32_t grid_z,
                       int32_t noise_mode, int32_t flux_range, float *out, double *noise_grid,
                       void *stream);

/* Blocks per axis of the noise grid of sofia_sc_normalise for a cube and
 * window / grid settings (grid 0 = default). No device work. */
int sofia_sc_normalise_grid(int64_t nx, int64_t ny, int64_t nz, int32_t window_xy,
                            int32_t window_z, int32_t grid_xy, int32_t grid_z, int64_t *nbx,
                            int64_t *nby, int64_t *nbz);

/* Linker (Sect. 4.3): merges the detected voxels (mask != 0) into
 * detections by friends-of-friends: two detected voxels are friends when
 * their offset lies in the ellipsoid (dx^2 + dy^2) / radius_xy^2 +
 * dz^2 / radius_z^2 <= 1 (an axis of radius 0 admits offset 0 only), and a
 * detection is a connected set of friends, spatially and spectrally alike.
 * A detection is dropped when its bounding-box extent along x or y is below
 * min_size_xy or along z below min_size_z, or, for max_size_xy > 0 /
 * max_size_z > 0, above those. Kept detections are numbered 1, 2, ... in the
 * raster order (z, y, x) of their first voxel. The mock-galaxy run of
 * Sect. 6 uses radius 2 and minimum sizes of 8 pixels and 5 channels.
 *  mask        device, uint8 [nz][ny][nx], read only.
 *  labels      device, int32 [nz][ny][nx]: the detection number of every
 *              voxel, 0 where none (also for dropped detections); used as
 *              workspace during the call.
 *  n_sources   host: number of kept detections.
 *  boxes       host, int64 [box_capacity][7] or NULL: per kept detection in
 *              label order x_min, x_max, y_min, y_max, z_min, z_max, voxel
 *              count (the first box_capacity of them).
 * The handle's workspace holds the list of the detected voxels (4 bytes
 * each) and per detection 36 bytes. Returns after the work has completed.
 * EINVAL for NULL pointers, bad dimensions, nx*ny*nz >= 2^31, radii outside
 * 0..SOFIA_SC_LINK_MAX_RADIUS or negative sizes; ENOMEM when the workspace
 * cannot grow. */
#define SOFIA_SC_LINK_MAX_RADIUS 4
int sofia_sc_link(sofia_sc *h, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz,
                  int32_t radius_xy, int32_t radius_z, int32_t min_size_xy, int32_t min_size_z,
                  int32_t max_size_xy, int32_t max_size_z, int32_t *labels, int64_t *n_sources,
                  int64_t *boxes, int64_t box_capacity, void *stream);

/* Parameters of one detection (Sect. 4.5; Eq. 4 and 5) and its reliability
 * (Sect. 4.4). */
typedef struct {
    int64_t n_vox;        /* finite voxels carrying the detection's label */
    double sum;           /* sum of their values */
    double peak;          /* largest value */
    double min;           /* smallest value */
    double mean;          /* sum / n_vox */
    double x, y, z;       /* value-weighted centroid in pixels (NaN for sum 0) */
    double flux;          /* channel_width / Omega x sum (Eq. 4) */
    double flux_err;      /* sqrt(n_vox) x channel_width x sigma_rms / sqrt(Omega) (Eq. 5) */
    double snr;           /* flux / flux_err */
    double reliability;   /* max(0, (P - N) / P) for a positive sum, else 0 */
    int32_t kept;         /* 1: positive, reliability and SNR at their thresholds */
    int32_t pad;
} sofia_sc_source;

typedef struct {
    int32_t struct_size;      /* sizeof(sofia_sc_param_options) */
    int32_t pad;
    double channel_width;     /* of Eq. 4 and 5 (default 1) */
    double beam_major_px;     /* Gaussian beam FWHM in pixels; both > 0 give */
    double beam_minor_px;     /* Omega = pi a b / (4 ln 2), else Omega = 1 */
    double sigma_rms;         /* noise of Eq. 5 (default 1) */
    double rel_scale;         /* kernel scale factor of the density (0.4) */
    double rel_threshold;     /* reliability threshold (0.9) */
    double snr_threshold;     /* integrated-SNR threshold (2.8) */
} sofia_sc_param_options;

/* Defaults of the mock-galaxy run of Sect. 6 (no beam, unit channel width
 * and noise). */
void sofia_sc_param_defaults(sofia_sc_param_options *opt);

/* Parameterisation and reliability of detections 1..n_sources of a label
 * cube (e.g. the linker's).
 * Parameters: every voxel whose label l is in 1..n_sources and whose value
 * is finite counts toward detection l. Reliability: the parameter vector of
 * a detection with a positive sum is log10 (peak, sum, mean), with a
 * negative sum log10 (-min, -sum, -mean); the densities P and N at a
 * positive detection are sums over the positive and the negative detections
 * (itself included) of exp(-d^T C^-1 d / 2), C the sample covariance
 * (divisor n - 1) of the negative detections' vectors times rel_scale^2.
 * With fewer than three negative detections or a C that is not positive
 * definite, every positive detection has reliability 1. Detections with a
 * zero sum take part in neither density.
 *  cube      device, float [nz][ny][nx].
 *  labels    device, int32 [nz][ny][nx]; other labels are ignored.
 *  out       device, sofia_sc_source [n_sources], written.
 *  n_kept    host: number of detections with kept = 1.
 * The density costs n_sources^2 kernel evaluations. Returns after the work
 * has completed. EINVAL for NULL pointers, bad dimensions, n_sources < 0 or
 * >= 2^31, non-positive channel width, negative sigma_rms or scale <= 0. */
int sofia_sc_parameterise(sofia_sc *h, const float *cube, const int32_t *labels, int64_t nx,
                          int64_t ny, int64_t nz, int64_t n_sources,
                          const sofia_sc_param_options *opt, sofia_sc_source *out,
                          int64_t *n_kept, void *stream);

/* The argument checks of sofia_sc_run_ex (the same code, run before any
 * device work) for a cube of nx x ny x nz voxels, a kernel list, threshold,
 * modes and options: SOFIA_SC_OK or the code the run would return (EINVAL).
 * Needs no handle, no device and no buffers. */
int sofia_sc_check_run(int64_t nx, int64_t ny, int64_t nz, const sofia_sc_kernel *kernels,
                       int32_t n_kernels, double threshold, int32_t noise_mode,
                       int32_t flux_range, const sofia_sc_options *opt);

/* Spatial cascade for a FWHM: n_iter boxcars of radius r per axis, chosen to
 * match the Gaussian variance, sigma_g^2 = (FWHM / 2 sqrt(2 ln 2))^2, with
 * n_iter r (r+1) / 3 (n_iter in 3..6, r >= 1; ties go to the larger n_iter).
 * FWHM 0 gives (0, 0). EINVAL for FWHM < 0 or non-finite. No device work. */
int sofia_sc_plan(double spatial_fwhm_px, int32_t *n_iter, int32_t *radius);

/* Per-kernel timing of the GPU launches, collected with HIP events on the
 * launch stream while profiling is enabled. */
typedef struct {
    char name[40];          /* kernel family, e.g. "spatial_cascade" */
    int64_t launches;
    double total_ms;        /* sum of event-measured launch durations */
    double bytes;           /* algorithmic HBM bytes summed over launches */
    double voxels;          /* voxels processed, summed over launches */
} sofia_sc_kernel_stat;

/* enable = 1 starts collecting (and clears previous figures), 0 stops. */
int sofia_sc_profile(sofia_sc *h, int enable);

/* Copy up to cap entries into stats; *n_out gets the number of families. */
int sofia_sc_profile_read(const sofia_sc *h, sofia_sc_kernel_stat *stats,
                          int32_t cap, int32_t *n_out);

/* Last error text of this handle ("" if none). Valid until the next call. */
const char *sofia_sc_last_error(const sofia_sc *h);

/* Static text for an error code. */
const char *sofia_sc_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* SOFIA_SC_H */
