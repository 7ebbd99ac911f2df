/*
 * TEST INFRASTRUCTURE: plain FP64 CPU oracle of SoFiA 2's local noise
 * normalisation (Westmeier et al. 2021, arXiv:2106.15789).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this library. It shares no code, header, table or helper with the GPU
 * library, nor with the smooth-and-clip oracle, and neither side calls the
 * other.
 *
 * What the paper fixes: when the noise level of the cube is not constant,
 * the noise is measured in a running window and the cube is divided by that
 * local noise before a constant threshold is applied (Sect. 4.1, last
 * paragraph); the speed test uses a window of 31 pixels spatially and 31
 * channels spectrally (Sect. 5).
 *
 * Readings where the paper is silent (each listed with its reason in the
 * design notes):
 *  N1 the noise is measured on a grid: each axis is cut into blocks of g
 *     voxels (the last block may be shorter); block b spans
 *     [b g, min(n, (b+1) g) - 1] and its centre is b g + (len_b - 1) / 2
 *     (integer division);
 *  N2 the window of a block is the w voxels centred on the block's centre
 *     (w odd), clipped to the cube; spatial windows are square (w_xy in x
 *     and y), the spectral window w_z long;
 *  N3 the noise of a window uses the smooth-and-clip estimators: RMS about
 *     zero, or 1.4826 x the median of |v| (mean of the two central order
 *     statistics for an even count), over finite voxels of the flux range
 *     (negative: v < 0, positive: v > 0, all: every finite v);
 *  N4 every voxel of a block is divided by its block's noise in FP64 and
 *     rounded to float32; non-finite voxels stay NaN, and a block whose noise
 *     is not finite and > 0 (no voxel selected, or zero noise) is blanked.
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace {

constexpr int kNoiseStd = 0;
constexpr int kNoiseMad = 1;
constexpr int kRangeNeg = -1;
constexpr int kRangeAll = 0;
constexpr int kRangePos = 1;
constexpr double kMadToSigma = 1.4826;

bool selected(double v, int range) {
    if (!std::isfinite(v)) return false;
    if (range == kRangeNeg) return v < 0.0;
    if (range == kRangePos) return v > 0.0;
    return true;
}

// N1: block b of an axis of n voxels cut into blocks of g.
struct Block {
    int64_t lo, hi, centre;   // [lo, hi] inclusive
};

Block block_of(int64_t b, int64_t n, int64_t g) {
    Block k;
    k.lo = b * g;
    k.hi = std::min(n, (b + 1) * g) - 1;
    k.centre = k.lo + (k.hi - k.lo) / 2;
    return k;
}

// N2: window of half-width r around the centre, clipped to [0, n - 1].
void window_of(int64_t centre, int64_t r, int64_t n, int64_t *a, int64_t *b) {
    *a = std::max<int64_t>(0, centre - r);
    *b = std::min<int64_t>(n - 1, centre + r);
}

// N3: noise of the selected values of one window (NaN if none).
double window_noise(const std::vector<double> &v, int mode) {
    const int64_t m = (int64_t)v.size();
    if (m == 0) return NAN;
    if (mode == kNoiseStd) {
        double sum = 0.0;
        for (double x : v) sum += x * x;
        return std::sqrt(sum / (double)m);
    }
    std::vector<double> a(v.size());
    for (size_t i = 0; i < v.size(); ++i) a[i] = std::fabs(v[i]);
    const int64_t lo = (m - 1) / 2, hi = m / 2;
    std::nth_element(a.begin(), a.begin() + lo, a.end());
    const double v_lo = a[(size_t)lo];
    double v_hi = v_lo;
    if (hi != lo) v_hi = *std::min_element(a.begin() + hi, a.end());
    return kMadToSigma * (hi == lo ? v_lo : 0.5 * (v_lo + v_hi));
}

}  // namespace

extern "C" {

// Number of blocks along an axis of n voxels cut into blocks of g (N1).
int64_t nno_blocks(int64_t n, int64_t g) { return g < 1 || n < 1 ? 0 : (n + g - 1) / g; }

// Local noise normalisation of X [nz][ny][nx] (float32):
//  sigma [nbz][nby][nbx] receives the noise of every block's window,
//  Y [nz][ny][nx] (float32, may be null) the normalised cube.
// Returns 0, or -1 for bad arguments.
int nno_normalise(const float *X, int64_t nx, int64_t ny, int64_t nz, int32_t w_xy,
                  int32_t w_z, int32_t g_xy, int32_t g_z, int32_t mode, int32_t range,
                  double *sigma, float *Y) {
    if (!X || !sigma || nx < 1 || ny < 1 || nz < 1) return -1;
    if (w_xy < 1 || w_z < 1 || !(w_xy & 1) || !(w_z & 1) || g_xy < 1 || g_z < 1) return -1;
    if (mode != kNoiseStd && mode != kNoiseMad) return -1;
    if (range != kRangeNeg && range != kRangeAll && range != kRangePos) return -1;
    const int64_t nbx = nno_blocks(nx, g_xy), nby = nno_blocks(ny, g_xy);
    const int64_t nbz = nno_blocks(nz, g_z);
    const int64_t rxy = (w_xy - 1) / 2, rz = (w_z - 1) / 2;
    const int64_t nblocks = nbx * nby * nbz;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t bi = 0; bi < nblocks; ++bi) {
        const int64_t bx = bi % nbx, by = (bi / nbx) % nby, bz = bi / (nbx * nby);
        const Block kx = block_of(bx, nx, g_xy), ky = block_of(by, ny, g_xy);
        const Block kz = block_of(bz, nz, g_z);
        int64_t x0, x1, y0, y1, z0, z1;
        window_of(kx.centre, rxy, nx, &x0, &x1);
        window_of(ky.centre, rxy, ny, &y0, &y1);
        window_of(kz.centre, rz, nz, &z0, &z1);
        std::vector<double> v;
        for (int64_t z = z0; z <= z1; ++z)
            for (int64_t y = y0; y <= y1; ++y)
                for (int64_t x = x0; x <= x1; ++x) {
                    const double d = (double)X[(z * ny + y) * nx + x];
                    if (selected(d, range)) v.push_back(d);
                }
        const double s = window_noise(v, mode);
        sigma[bi] = s;
        if (!Y) continue;
        const bool usable = std::isfinite(s) && s > 0.0;
        for (int64_t z = kz.lo; z <= kz.hi; ++z)
            for (int64_t y = ky.lo; y <= ky.hi; ++y)
                for (int64_t x = kx.lo; x <= kx.hi; ++x) {
                    const int64_t i = (z * ny + y) * nx + x;
                    const double d = (double)X[i];
                    Y[i] = (usable && std::isfinite(d)) ? (float)(d / s) : NAN;
                }
    }
    return 0;
}

}  // extern "C"
