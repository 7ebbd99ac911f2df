/*
 * Seeded synthetic H I data cubes: Gaussian noise plus injected mock galaxies.
 *
 * This module only produces inputs. It holds none of the smooth-and-clip
 * arithmetic and is shared, unchanged, by the oracle tests, the GPU tests and
 * the benchmark.
 *
 * Noise: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11, "Parallel random
 * numbers: as easy as 1, 2, 3") keyed by (seed, cube id, stream), with the
 * voxel index as the counter, followed by the Box-Muller transform. One Philox
 * block per voxel, so every voxel is independent of the thread layout.
 *
 * Galaxies: 3D Gaussian blobs (positive only, like H I emission), with the
 * peak given in units of the local noise sigma. The paper injects model
 * galaxies into real noise (Sect. 6); those models are not available, so
 * blobs of comparable spatial and spectral extent stand in for them.
 *
 * Layout: float32 [nz][ny][nx], x fastest, z (spectral) slowest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

/* Philox4x32 with 10 rounds, as published (round function: two 32x32->64
 * multiplies, xor with the other counter words and the key; key bumped by the
 * Weyl constants between rounds). */
static void philox4x32_10(const uint32_t in[4], uint32_t k0, uint32_t k1,
                          uint32_t out[4]) {
    uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Public for the known-answer test of the generator itself. */
void synth_philox4x32_10(const uint32_t in[4], uint32_t k0, uint32_t k1,
                         uint32_t out[4]) {
    philox4x32_10(in, k0, k1, out);
}

/* Uniform double in the open interval (0, 1) from two 32-bit words. */
static double u01_open(uint32_t a, uint32_t b) {
    uint64_t m = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6); /* 53 bits */
    return ((double)m + 0.5) * (1.0 / 9007199254740992.0);
}

static void draw(uint64_t seed, uint32_t cube_id, uint32_t stream,
                 uint64_t index, uint32_t out[4]) {
    uint32_t ctr[4] = {(uint32_t)index, (uint32_t)(index >> 32), stream,
                       cube_id};
    philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), out);
}

/* One standard normal deviate per counter value (Box-Muller, first branch). */
static double normal_at(uint64_t seed, uint32_t cube_id, uint32_t stream,
                        uint64_t index) {
    uint32_t w[4];
    draw(seed, cube_id, stream, index, w);
    double u1 = u01_open(w[0], w[1]);
    double u2 = u01_open(w[2], w[3]);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

typedef struct {
    int64_t nx, ny, nz;
    uint64_t seed;
    uint32_t cube_id;
    int32_t field_kind;   /* 0: constant sigma_lo; 1: radial sigma_lo..sigma_hi */
    double sigma_lo, sigma_hi;
    int64_t n_gal;
    int64_t nan_border;   /* spatial border (px) blanked in every channel */
    double peak_lo, peak_hi;         /* galaxy peak in units of local sigma */
    double fwhm_z_lo, fwhm_z_hi;     /* spectral FWHM range (channels) */
    double fwhm_xy_lo, fwhm_xy_hi;   /* spatial FWHM range (pixels) */
    int64_t z0, z1;       /* generate only planes [z0, z1) into out (slab) */
} synth_params;

/* Noise sigma at spatial pixel (x, y). The radial field grows with the squared
 * distance from the field centre, normalised to 1 at the corners. */
static double sigma_at(const synth_params *p, int64_t x, int64_t y) {
    if (p->field_kind == 0) return p->sigma_lo;
    double cx = 0.5 * (double)(p->nx - 1), cy = 0.5 * (double)(p->ny - 1);
    double dx = (double)x - cx, dy = (double)y - cy;
    double rmax2 = cx * cx + cy * cy;
    double rho2 = rmax2 > 0.0 ? (dx * dx + dy * dy) / rmax2 : 0.0;
    return p->sigma_lo + (p->sigma_hi - p->sigma_lo) * rho2;
}

typedef struct {
    double cx, cy, cz, peak, sxy, sz;
} blob;

static double uniform_in(double lo, double hi, uint32_t a, uint32_t b) {
    return lo + (hi - lo) * u01_open(a, b);
}

static double centre_in(int64_t n, double margin, uint32_t a, uint32_t b) {
    double lo = margin, hi = (double)(n - 1) - margin;
    if (hi < lo) return 0.5 * (double)(n - 1);
    return uniform_in(lo, hi, a, b);
}

static void make_blobs(const synth_params *p, blob *g) {
    const double k = 2.3548200450309493; /* FWHM / sigma of a Gaussian */
    for (int64_t i = 0; i < p->n_gal; ++i) {
        uint32_t w0[4], w1[4];
        draw(p->seed, p->cube_id, 1u, (uint64_t)(2 * i), w0);
        draw(p->seed, p->cube_id, 1u, (uint64_t)(2 * i + 1), w1);
        double fxy = uniform_in(p->fwhm_xy_lo, p->fwhm_xy_hi, w0[0], w0[1]);
        double fz = uniform_in(p->fwhm_z_lo, p->fwhm_z_hi, w0[2], w0[3]);
        g[i].sxy = fxy / k;
        g[i].sz = fz / k;
        g[i].cx = centre_in(p->nx, 1.5 * fxy, w1[0], w1[1]);
        g[i].cy = centre_in(p->ny, 1.5 * fxy, w1[2], w1[3]);
        uint32_t w2[4];
        draw(p->seed, p->cube_id, 2u, (uint64_t)i, w2);
        g[i].cz = centre_in(p->nz, 1.5 * fz, w2[0], w2[1]);
        double s_loc = sigma_at(p, (int64_t)llround(g[i].cx),
                                (int64_t)llround(g[i].cy));
        g[i].peak = uniform_in(p->peak_lo, p->peak_hi, w2[2], w2[3]) * s_loc;
    }
}

/* Fill planes [z0, z1) of the cube. out holds (z1 - z0) * ny * nx floats.
 * Returns 0, or -1 on bad arguments / allocation failure. */
int synth_cube(const synth_params *p, float *out) {
    if (!p || !out || p->nx < 1 || p->ny < 1 || p->nz < 1 || p->n_gal < 0)
        return -1;
    int64_t z0 = p->z0, z1 = p->z1;
    if (z1 <= 0 && z0 == 0) z1 = p->nz;
    if (z0 < 0 || z1 > p->nz || z0 >= z1) return -1;
    const int64_t nx = p->nx, ny = p->ny, plane = nx * ny;

    double *sig = (double *)malloc((size_t)plane * sizeof(double));
    blob *g = p->n_gal ? (blob *)malloc((size_t)p->n_gal * sizeof(blob)) : NULL;
    if (!sig || (p->n_gal && !g)) { free(sig); free(g); return -1; }
    for (int64_t y = 0; y < ny; ++y)
        for (int64_t x = 0; x < nx; ++x) sig[y * nx + x] = sigma_at(p, x, y);
    if (p->n_gal) make_blobs(p, g);

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t z = z0; z < z1; ++z) {
        float *pl = out + (z - z0) * plane;
        for (int64_t i = 0; i < plane; ++i) {
            uint64_t idx = (uint64_t)(z * plane + i);
            pl[i] = (float)(sig[i] * normal_at(p->seed, p->cube_id, 0u, idx));
        }
        /* Galaxies are added in index order, so the result does not depend
         * on the number of threads. */
        for (int64_t gi = 0; gi < p->n_gal; ++gi) {
            const blob *b = &g[gi];
            double dz = ((double)z - b->cz) / b->sz;
            if (fabs(dz) > 4.0) continue;
            double ez = exp(-0.5 * dz * dz);
            int64_t xa = (int64_t)ceil(b->cx - 4.0 * b->sxy);
            int64_t xb = (int64_t)floor(b->cx + 4.0 * b->sxy);
            int64_t ya = (int64_t)ceil(b->cy - 4.0 * b->sxy);
            int64_t yb = (int64_t)floor(b->cy + 4.0 * b->sxy);
            if (xa < 0) xa = 0;
            if (ya < 0) ya = 0;
            if (xb > nx - 1) xb = nx - 1;
            if (yb > ny - 1) yb = ny - 1;
            for (int64_t y = ya; y <= yb; ++y) {
                double dy = ((double)y - b->cy) / b->sxy;
                double ey = exp(-0.5 * dy * dy);
                for (int64_t x = xa; x <= xb; ++x) {
                    double dx = ((double)x - b->cx) / b->sxy;
                    double v = b->peak * ez * ey * exp(-0.5 * dx * dx);
                    pl[y * nx + x] = (float)((double)pl[y * nx + x] + v);
                }
            }
        }
        if (p->nan_border > 0) {
            const int64_t bw = p->nan_border;
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x)
                    if (x < bw || y < bw || x >= nx - bw || y >= ny - bw)
                        pl[y * nx + x] = NAN;
        }
    }
    free(sig);
    free(g);
    return 0;
}

/* Voxel-wise noise sigma (no galaxies, no blanking): used by tests that need
 * the generating sigma field. out holds ny * nx doubles. */
int synth_sigma_field(const synth_params *p, double *out) {
    if (!p || !out) return -1;
    for (int64_t y = 0; y < p->ny; ++y)
        for (int64_t x = 0; x < p->nx; ++x)
            out[y * p->nx + x] = sigma_at(p, x, y);
    return 0;
}
