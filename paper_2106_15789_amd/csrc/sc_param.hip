// Source parameterisation and reliability (Westmeier et al. 2021, Sect. 4.4
// and 4.5; Eq. 4 and 5).
//
// For the detections of a label cube (the linker's output):
//  * k_param_accum: one pass over the cube; every labelled finite voxel adds
//    its value, its value times its position, and its voxel count to its
//    detection's accumulators (FP64 and 64-bit integer atomics), and moves
//    the detection's peak and minimum (integer atomics on an order-keeping
//    map of the float's bits);
//  * k_param_finalize: per detection: mean, flux-weighted centroid,
//    F = channel width / Omega x sum (Eq. 4), sigma_F = sqrt(N) x channel
//    width x sigma_rms / sqrt(Omega) (Eq. 5), SNR = F / sigma_F, and the
//    reliability parameter vector: log10 of (peak, sum, mean), or of
//    (-min, -sum, -mean) for a detection of negative total flux;
//  * k_rel_stats (one workgroup): mean and covariance (divisor n - 1) of
//    the negative detections' vectors, times the kernel scale squared, and
//    its inverse;
//  * k_rel_density: per positive detection, the sums of Gaussian kernels of
//    the positive (P) and negative (N) detections around it, tiled through
//    LDS; R = max(0, (P - N) / P); a detection is kept when positive with
//    R >= the reliability threshold and SNR >= the SNR threshold.
#include <climits>
#include <math.h>

#include "sc_internal.h"

namespace sc {

namespace {

// Floats to ints of the same order (for integer max / min atomics).
__device__ __forceinline__ int order_key(float f) {
    const int i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7fffffff;
}
__device__ __forceinline__ float order_value(int k) {
    return __int_as_float(k >= 0 ? k : k ^ 0x7fffffff);
}

}  // namespace

__global__ __launch_bounds__(256) void k_param_init(SrcAcc *acc, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        SrcAcc a;
        a.count = 0;
        a.sum = a.sx = a.sy = a.sz = 0.0;
        a.peak = order_key(-INFINITY);
        a.mn = order_key(INFINITY);
        acc[i] = a;
    }
}

__device__ __forceinline__ void add_voxel(const ParamArgs &a, int64_t i, int l) {
    const float v = a.cube[i];
    if (!isfinite(v)) return;
    const int64_t x = i % a.nx, y = (i / a.nx) % a.ny, z = i / (a.nx * a.ny);
    SrcAcc *s = a.acc + (l - 1);
    const double d = (double)v;
    atomicAdd(&s->count, 1ull);
    atomicAdd(&s->sum, d);
    atomicAdd(&s->sx, d * (double)x);
    atomicAdd(&s->sy, d * (double)y);
    atomicAdd(&s->sz, d * (double)z);
    const int k = order_key(v);
    atomicMax(&s->peak, k);
    atomicMin(&s->mn, k);
}

// Wave-wide reductions (every lane of the wave takes part).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

// One record per lane (valid: it holds voxels of detection l in 1..n): its
// voxel count, sums of v, v x, v y, v z and the order keys of its largest
// and smallest value. The lanes that share a label are reduced across the
// wave first, and one lane per label updates that detection's
// accumulators: neighbouring voxels mostly carry the same label, so this
// replaces up to 64 contended atomics by one.
struct Rec {
    int cnt;
    double s, sx, sy, sz;
    int kmax, kmin;
};

__device__ __forceinline__ void rec_add(Rec &r, float v, int64_t x, int64_t y, int64_t z) {
    const double d = (double)v;
    r.cnt += 1;
    r.s += d;
    r.sx += d * (double)x;
    r.sy += d * (double)y;
    r.sz += d * (double)z;
    const int k = order_key(v);
    r.kmax = max(r.kmax, k);
    r.kmin = min(r.kmin, k);
}

__device__ __forceinline__ Rec rec_empty() {
    Rec r;
    r.cnt = 0;
    r.s = r.sx = r.sy = r.sz = 0.0;
    r.kmax = INT_MIN;
    r.kmin = INT_MAX;
    return r;
}

__device__ __forceinline__ void add_records_wave(const ParamArgs &a, bool valid, int l,
                                                 const Rec &r) {
    uint64_t pending = __ballot(valid);
    const int lane = threadIdx.x & 63;
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int lab = __shfl(l, leader);
        const bool mine = valid && l == lab;
        const uint64_t m = __ballot(mine);
        const double s = wave_sum(mine ? r.s : 0.0);
        const double sx = wave_sum(mine ? r.sx : 0.0);
        const double sy = wave_sum(mine ? r.sy : 0.0);
        const double sz = wave_sum(mine ? r.sz : 0.0);
        int c = mine ? r.cnt : 0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
        const int pk = wave_max(mine ? r.kmax : INT_MIN);
        const int mn = wave_min(mine ? r.kmin : INT_MAX);
        if (lane == leader) {
            SrcAcc *p = a.acc + (lab - 1);
            atomicAdd(&p->count, (unsigned long long)c);
            atomicAdd(&p->sum, s);
            atomicAdd(&p->sx, sx);
            atomicAdd(&p->sy, sy);
            atomicAdd(&p->sz, sz);
            atomicMax(&p->peak, pk);
            atomicMin(&p->mn, mn);
        }
        pending &= ~m;
    }
}

// The label cube is read whole (four labels per load when aligned); the
// cube's values only where a label is set. Waves step through the cube
// together, so the wave-wide reductions see every lane.
template <int V>
__global__ __launch_bounds__(256) void k_param_accum(ParamArgs a) {
    const int64_t N = a.nx * a.ny * a.nz;
    const int64_t nq = N / V;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t wbase = t - (threadIdx.x & 63);
    for (int64_t qb = wbase; qb < nq; qb += stride) {
        const int64_t q = qb + (threadIdx.x & 63);
        int lab[V];
        if (q < nq) {
            if constexpr (V == 4) {
                const int4 l4 = reinterpret_cast<const int4 *>(a.labels)[q];
                lab[0] = l4.x; lab[1] = l4.y; lab[2] = l4.z; lab[3] = l4.w;
            } else {
                lab[0] = a.labels[q];
            }
        } else {
#pragma unroll
            for (int k = 0; k < V; ++k) lab[k] = 0;
        }
        // position of voxel q V (only for lanes holding a label): one
        // division by the plane size, then 32-bit arithmetic (planes hold
        // < 2^28 voxels)
        bool any = false;
#pragma unroll
        for (int k = 0; k < V; ++k) any |= lab[k] > 0 && lab[k] <= a.n;
        int64_t x0 = 0, y0 = 0, z0 = 0;
        if (any) {
            const int64_t i0 = q * V;
            z0 = i0 / a.plane;
            const uint32_t rem = (uint32_t)(i0 - z0 * a.plane);
            y0 = rem / (uint32_t)a.nx;
            x0 = rem - (uint32_t)y0 * (uint32_t)a.nx;
        }
        // the lane's voxels as one record when they all carry one label
        // (the usual case), else one record per voxel
        int L = 0;
        bool mixed = false;
        float v[V];
        int64_t px[V], py[V], pz[V];
        {
            int64_t x = x0, y = y0, z = z0;
#pragma unroll
            for (int k = 0; k < V; ++k) {
                px[k] = x; py[k] = y; pz[k] = z;
                const bool in = lab[k] > 0 && lab[k] <= a.n;
                v[k] = in ? a.cube[q * V + k] : 0.f;
                if (!(in && isfinite(v[k]))) lab[k] = 0;
                if (lab[k]) {
                    if (L == 0) L = lab[k];
                    else if (lab[k] != L) mixed = true;
                }
                if (++x == a.nx) {
                    x = 0;
                    if (++y == a.ny) { y = 0; ++z; }
                }
            }
        }
        Rec r = rec_empty();
        if (L && !mixed) {
#pragma unroll
            for (int k = 0; k < V; ++k)
                if (lab[k]) rec_add(r, v[k], px[k], py[k], pz[k]);
        }
        add_records_wave(a, L != 0 && !mixed, L, r);
        if (__ballot(mixed)) {
#pragma unroll
            for (int k = 0; k < V; ++k) {
                Rec rk = rec_empty();
                if (mixed && lab[k]) rec_add(rk, v[k], px[k], py[k], pz[k]);
                add_records_wave(a, mixed && lab[k] != 0, lab[k], rk);
            }
        }
    }
    // the last N mod V voxels, one thread each
    for (int64_t i = nq * V + t; i < N; i += stride) {
        const int l = a.labels[i];
        if (l > 0 && l <= a.n) add_voxel(a, i, l);
    }
}

__global__ __launch_bounds__(256) void k_param_finalize(ParamArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        const SrcAcc s = a.acc[i];
        sofia_sc_source o;
        o.n_vox = (int64_t)s.count;
        o.sum = s.sum;
        o.peak = (double)order_value(s.peak);
        o.min = (double)order_value(s.mn);
        o.mean = s.sum / (double)s.count;
        const bool nz = s.sum != 0.0;
        o.x = nz ? s.sx / s.sum : NAN;
        o.y = nz ? s.sy / s.sum : NAN;
        o.z = nz ? s.sz / s.sum : NAN;
        o.flux = a.channel_width / a.omega * s.sum;
        o.flux_err = sqrt((double)s.count) * a.channel_width * a.sigma_rms / sqrt(a.omega);
        o.snr = o.flux / o.flux_err;
        o.reliability = 0.0;
        o.kept = 0;
        o.pad = 0;
        a.out[i] = o;
        // reliability parameters: sign of the total flux, log10 of the
        // vector (peak, sum, mean) or (-min, -sum, -mean)
        const int sg = s.sum > 0.0 ? 1 : (s.sum < 0.0 ? -1 : 0);
        a.sign[i] = sg;
        double v0 = 0.0, v1 = 0.0, v2 = 0.0;
        if (sg > 0) { v0 = log10(o.peak); v1 = log10(o.sum); v2 = log10(o.mean); }
        if (sg < 0) { v0 = log10(-o.min); v1 = log10(-o.sum); v2 = log10(-o.mean); }
        a.vec[3 * i] = v0;
        a.vec[3 * i + 1] = v1;
        a.vec[3 * i + 2] = v2;
    }
}

// One workgroup: statistics of the negative detections' vectors. rs[0..8]
// receives the inverse covariance (row-major), rs[9] 1 when it exists.
__global__ __launch_bounds__(1024) void k_rel_stats(ParamArgs a) {
    __shared__ double red[1024];
    __shared__ double mu[3];
    __shared__ double cov[6];
    __shared__ unsigned long long cnt;
    const int tid = threadIdx.x;
    auto reduce = [&](double v) -> double {
        red[tid] = v;
        __syncthreads();
        for (int off = 512; off > 0; off >>= 1) {
            if (tid < off) red[tid] += red[tid + off];
            __syncthreads();
        }
        const double r = red[0];
        __syncthreads();
        return r;
    };
    // count and mean
    double m = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t i = tid; i < a.n; i += 1024)
        if (a.sign[i] < 0) {
            m += 1.0;
            s0 += a.vec[3 * i];
            s1 += a.vec[3 * i + 1];
            s2 += a.vec[3 * i + 2];
        }
    const double M = reduce(m);
    const double t0 = reduce(s0), t1 = reduce(s1), t2 = reduce(s2);
    if (tid == 0) {
        cnt = (unsigned long long)M;
        mu[0] = M > 0 ? t0 / M : 0.0;
        mu[1] = M > 0 ? t1 / M : 0.0;
        mu[2] = M > 0 ? t2 / M : 0.0;
    }
    __syncthreads();
    // centred second moments
    double c[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = tid; i < a.n; i += 1024)
        if (a.sign[i] < 0) {
            const double d0 = a.vec[3 * i] - mu[0], d1 = a.vec[3 * i + 1] - mu[1],
                         d2 = a.vec[3 * i + 2] - mu[2];
            c[0] += d0 * d0; c[1] += d0 * d1; c[2] += d0 * d2;
            c[3] += d1 * d1; c[4] += d1 * d2; c[5] += d2 * d2;
        }
    for (int k = 0; k < 6; ++k) {
        const double r = reduce(c[k]);
        if (tid == 0) cov[k] = r;
    }
    if (tid != 0) return;
    *a.n_kept = 0;
    double *rs = a.rel_state;
    rs[9] = 0.0;
    if (cnt < 3) return;
    const double f = a.scale * a.scale / (double)(cnt - 1);
    const double A = cov[0] * f, B = cov[1] * f, C = cov[2] * f;
    const double D = cov[3] * f, E = cov[4] * f, F = cov[5] * f;
    // symmetric [[A B C] [B D E] [C E F]]: inverse by cofactors
    const double c00 = D * F - E * E, c01 = C * E - B * F, c02 = B * E - C * D;
    const double det = A * c00 + B * c01 + C * c02;
    if (!(isfinite(det) && det > 0.0)) return;
    const double c11 = A * F - C * C, c12 = B * C - A * E, c22 = A * D - B * B;
    rs[0] = c00 / det; rs[1] = c01 / det; rs[2] = c02 / det;
    rs[3] = c01 / det; rs[4] = c11 / det; rs[5] = c12 / det;
    rs[6] = c02 / det; rs[7] = c12 / det; rs[8] = c22 / det;
    rs[9] = 1.0;
}

// One thread per detection; the other detections' vectors pass through LDS
// in tiles of 256.
__global__ __launch_bounds__(256) void k_rel_density(ParamArgs a) {
    __shared__ double tv[256][3];
    __shared__ int ts[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool mine = i < a.n;
    const int sg = mine ? a.sign[i] : 0;
    double v0 = 0, v1 = 0, v2 = 0;
    if (mine) { v0 = a.vec[3 * i]; v1 = a.vec[3 * i + 1]; v2 = a.vec[3 * i + 2]; }
    double inv[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) inv[k] = a.rel_state[k];
    const bool stats = a.rel_state[9] != 0.0;
    double P = 0.0, Nn = 0.0;
    for (int64_t t0 = 0; t0 < a.n; t0 += 256) {
        const int64_t j = t0 + threadIdx.x;
        if (j < a.n) {
            tv[threadIdx.x][0] = a.vec[3 * j];
            tv[threadIdx.x][1] = a.vec[3 * j + 1];
            tv[threadIdx.x][2] = a.vec[3 * j + 2];
            ts[threadIdx.x] = a.sign[j];
        } else {
            ts[threadIdx.x] = 0;
        }
        __syncthreads();
        if (sg > 0 && stats) {
            const int m = (int)(a.n - t0 < 256 ? a.n - t0 : 256);
            for (int k = 0; k < m; ++k) {
                const int sk = ts[k];
                if (sk == 0) continue;
                const double d0 = v0 - tv[k][0], d1 = v1 - tv[k][1], d2 = v2 - tv[k][2];
                const double q = d0 * (inv[0] * d0 + inv[1] * d1 + inv[2] * d2) +
                                 d1 * (inv[3] * d0 + inv[4] * d1 + inv[5] * d2) +
                                 d2 * (inv[6] * d0 + inv[7] * d1 + inv[8] * d2);
                const double e = exp(-0.5 * q);
                if (sk > 0) P += e; else Nn += e;
            }
        }
        __syncthreads();
    }
    if (!mine) return;
    double R = 0.0;
    if (sg > 0) R = stats ? fmax(0.0, (P - Nn) / P) : 1.0;
    sofia_sc_source &o = a.out[i];
    o.reliability = R;
    o.kept = (sg > 0 && R >= a.rel_threshold && o.snr >= a.snr_threshold) ? 1 : 0;
    if (o.kept) atomicAdd(a.n_kept, 1ull);
}

namespace {
unsigned blocks_for(int64_t n, int per, int64_t cap) {
    int64_t g = (n + per - 1) / per;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}
}  // namespace

hipError_t launch_parameterise(const ParamArgs &a, hipStream_t s) {
    const int64_t N = a.nx * a.ny * a.nz;
    hipLaunchKernelGGL(k_param_init, dim3(blocks_for(a.n, 256, 65536)), dim3(256), 0, s, a.acc,
                       a.n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned g = blocks_for(N / (a.vec4 ? 4 : 1), 256, 65536);
    if (a.vec4)
        hipLaunchKernelGGL(k_param_accum<4>, dim3(g), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_param_accum<1>, dim3(g), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_param_finalize, dim3(blocks_for(a.n, 256, 65536)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reliability(const ParamArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_rel_stats, dim3(1), dim3(1024), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t blocks = (a.n + 255) / 256;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rel_density, dim3((unsigned)(blocks < 1 ? 1 : blocks)), dim3(256), 0, s,
                       a);
    return hipGetLastError();
}

}  // namespace sc
