// Linker (Westmeier et al. 2021, Sect. 4.3): the detected voxels of the mask
// are merged into detections by friends-of-friends over a merging radius,
// spatially and spectrally alike, each detection gets a unique identifier,
// and detections outside the spatial and spectral size limits are dropped.
// Friends are the voxels whose offset lies in the ellipsoid
// (dx^2 + dy^2) / r_xy^2 + dz^2 / r_z^2 <= 1 (an axis of radius 0 admits
// offset 0 only); a detection's size is its bounding-box extent; kept
// detections are numbered 1, 2, ... in the raster order of their first voxel.
//
// Work split (the label cube itself is the union-find forest, int32 voxel
// indices). The mask is sparse, so after one pass over the cube the work
// runs over a list of the detected voxels, in raster order, one per lane:
//  * per-block counts, a scan and a block-local scan write the detected
//    voxels' indices to the list; k_link_init makes every listed voxel its
//    own root (the other voxels' links are never read);
//  * k_link_union: one thread per listed voxel unites it with its detected
//    friends at the forward half of the offsets (the other half is the
//    friends' own forward half). Unions hook the larger root under the
//    smaller one with a compare-and-swap, so every tree's root ends as the
//    smallest index of its detection: the canonical label, independent of
//    the order in which the threads ran;
//  * k_link_flatten: every listed voxel points straight at its root;
//  * the same count/scan/assign steps over the list number the roots in
//    raster order; k_link_resolve then gives every listed voxel its
//    detection's number and accumulates the bounding boxes with atomics;
//  * the same steps number the kept detections, and k_link_label writes the
//    final labels of the whole cube (reading links only where detected).
// Forest links are read with agent-scope atomic loads: a CU's vector cache is
// not coherent with the other CUs' writes.
#include <limits.h>

#include "sc_device.h"

namespace sc {

namespace {

__device__ __forceinline__ int ld_link(const int *L, int i) {
    return __hip_atomic_load(L + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of voxel x, halving the path on the way (every link only ever moves
// to a smaller index, so a halving write never breaks a tree; writes are
// minima, so concurrent halvings and flattening never raise a link).
__device__ int find_root(int *L, int x) {
    while (true) {
        const int p = ld_link(L, x);
        if (p == x) return x;
        const int g = ld_link(L, p);
        // a minimum, not a store: another thread may already have linked x
        // closer to the root, and a link must never move away from it
        if (g != p) atomicMin(L + x, g);
        x = p;
    }
}

__device__ void unite(int *L, int a, int b) {
    while (true) {
        a = find_root(L, a);
        b = find_root(L, b);
        if (a == b) return;
        if (a > b) { const int t = a; a = b; b = t; }
        // hook root b under the smaller root a
        const int old = atomicCAS(L + b, b, a);
        if (old == b) return;
        b = old;
    }
}

__device__ __forceinline__ void decode_off(int code, int &dx, int &dy, int &dz) {
    dx = (code & 255) - 128;
    dy = ((code >> 8) & 255) - 128;
    dz = ((code >> 16) & 255) - 128;
}

constexpr int kScanItems = 4096;    // items per block of the count / assign steps
constexpr int kScanThreads = 1024;  // 4 consecutive items per thread

// Exclusive block scan of one value per thread (kScanThreads values);
// returns the exclusive prefix; *total gets the block's sum.
__device__ int block_excl_scan(int v, int *buf, int *total) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(x, off);
        if (lane >= off) x += t;
    }
    if (lane == 63) buf[wave] = x;
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) {
            const int t = buf[w];
            buf[w] = acc;
            acc += t;
        }
        buf[kScanThreads / 64] = acc;
    }
    __syncthreads();
    const int ex = x - v + buf[wave];
    *total = buf[kScanThreads / 64];
    __syncthreads();
    return ex;
}

}  // namespace

__global__ __launch_bounds__(256) void k_link_init(LinkArgs a) {
    const int m = (int)a.m;
    const int stride = (int)(gridDim.x * blockDim.x);
    for (int t = (int)(blockIdx.x * blockDim.x + threadIdx.x); t < m; t += stride) {
        const int i = a.list[t];
        a.L[i] = i;
    }
}

// Position of voxel i (the linker's cubes hold fewer than 2^31 voxels, so
// 32-bit divisions suffice).
__device__ __forceinline__ void pos_of(const LinkArgs &a, uint32_t i, int &x, int &y, int &z) {
    const uint32_t nx = (uint32_t)a.nx, ny = (uint32_t)a.ny;
    const uint32_t r = i / nx;
    x = (int)(i - r * nx);
    z = (int)(r / ny);
    y = (int)(r - (uint32_t)z * ny);
}

__global__ __launch_bounds__(256) void k_link_union(LinkArgs a) {
    const int m = (int)a.m;
    const int stride = (int)(gridDim.x * blockDim.x);
    for (int t = (int)(blockIdx.x * blockDim.x + threadIdx.x); t < m; t += stride) {
        const int i = a.list[t];
        int x, y, z;
        pos_of(a, (uint32_t)i, x, y, z);
        for (int k = 0; k < a.n_off; ++k) {
            int dx, dy, dz;
            decode_off(a.off[k], dx, dy, dz);
            const int xx = x + dx, yy = y + dy, zz = z + dz;
            if (xx < 0 || xx >= a.nx || yy < 0 || yy >= a.ny || zz < 0 || zz >= a.nz) continue;
            const int j = i + a.delta[k];
            if (!a.mask[j]) continue;
            // already in one tree when both link to the same voxel
            if (ld_link(a.L, i) == ld_link(a.L, j)) continue;
            unite(a.L, i, j);
        }
    }
}

__global__ __launch_bounds__(256) void k_link_flatten(LinkArgs a) {
    const int m = (int)a.m;
    const int stride = (int)(gridDim.x * blockDim.x);
    for (int t = (int)(blockIdx.x * blockDim.x + threadIdx.x); t < m; t += stride) {
        const int i = a.list[t];
        const int r = find_root(a.L, i);
        // the root is the smallest index on the path: after every thread's
        // minimum, each detected voxel links straight to its root
        atomicMin(a.L + i, r);
    }
}

// Flags of the count / assign steps: voxel i is detected (LK_VOXELS), listed
// voxel i is a root (LK_ROOTS), detection i is kept (LK_KEPT).
template <int ITEMS>
__device__ __forceinline__ bool link_flag(const LinkArgs &a, int64_t i) {
    if (ITEMS == LK_VOXELS) return a.mask[i] != 0;
    if (ITEMS == LK_ROOTS) {
        const int v = a.list[i];
        return a.L[v] == v;
    }
    const int *b = a.box + 8 * i;
    const int ex = b[1] - b[0] + 1, ey = b[3] - b[2] + 1, ez = b[5] - b[4] + 1;
    bool keep = ex >= a.min_xy && ey >= a.min_xy && ez >= a.min_z;
    if (a.max_xy > 0 && (ex > a.max_xy || ey > a.max_xy)) keep = false;
    if (a.max_z > 0 && ez > a.max_z) keep = false;
    return keep;
}

template <int ITEMS>
__global__ __launch_bounds__(kScanThreads) void k_link_count(LinkArgs a, int64_t n,
                                                             int *counts) {
    __shared__ int buf[kScanThreads / 64 + 1];
    const int64_t i0 = (int64_t)blockIdx.x * kScanItems + 4 * threadIdx.x;
    int c = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (i0 + k < n && link_flag<ITEMS>(a, i0 + k)) ++c;
    int total;
    block_excl_scan(c, buf, &total);
    if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

// Exclusive scan of nb block counts in place (one workgroup); counts[nb]
// receives the total.
__global__ __launch_bounds__(kScanThreads) void k_link_scan(int *counts, int64_t nb) {
    __shared__ int buf[kScanThreads / 64 + 1];
    const int64_t per = (nb + kScanThreads - 1) / kScanThreads;
    const int64_t b0 = threadIdx.x * per, b1 = b0 + per < nb ? b0 + per : nb;
    int s = 0;
    for (int64_t b = b0; b < b1; ++b) s += counts[b];
    int total;
    int ex = block_excl_scan(s, buf, &total);
    for (int64_t b = b0; b < b1; ++b) {
        const int c = counts[b];
        counts[b] = ex;
        ex += c;
    }
    if (threadIdx.x == 0) counts[nb] = total;
}

// Detected voxels: list[rank] = index. Roots: the detection number (raster
// order) into the root's own link, encoded as -2 - number. Kept detections:
// label_of[c] = 1 + rank or 0.
template <int ITEMS>
__global__ __launch_bounds__(kScanThreads) void k_link_assign(LinkArgs a, int64_t n,
                                                              const int *offsets) {
    __shared__ int buf[kScanThreads / 64 + 1];
    const int64_t i0 = (int64_t)blockIdx.x * kScanItems + 4 * threadIdx.x;
    bool f[4];
    int c = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        f[k] = i0 + k < n && link_flag<ITEMS>(a, i0 + k);
        c += f[k] ? 1 : 0;
    }
    int total;
    int rank = offsets[blockIdx.x] + block_excl_scan(c, buf, &total);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (i0 + k >= n) break;
        if (ITEMS == LK_VOXELS) {
            if (f[k]) a.list[rank++] = (int)(i0 + k);
        } else if (ITEMS == LK_ROOTS) {
            if (f[k]) a.L[a.list[i0 + k]] = -2 - rank++;
        } else {
            a.label_of[i0 + k] = f[k] ? 1 + rank++ : 0;
        }
    }
}

__global__ __launch_bounds__(256) void k_link_box_init(int *box, int64_t nc) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += stride) {
        int *b = box + 8 * c;
        b[0] = INT_MAX; b[1] = -1; b[2] = INT_MAX; b[3] = -1; b[4] = INT_MAX; b[5] = -1;
        b[6] = 0; b[7] = 0;
    }
}

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// Every listed voxel: its detection's number (from its root) and its share
// of the detection's bounding box and voxel count. The lanes of a wave that
// belong to one detection are reduced first, and one of them updates the
// box: consecutive listed voxels mostly share a detection. Waves step
// through the list together, so every lane takes part in the reductions.
__global__ __launch_bounds__(256) void k_link_resolve(LinkArgs a) {
    const int m = (int)a.m;
    const int stride = (int)(gridDim.x * blockDim.x);
    const int lane = threadIdx.x & 63;
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    for (int tb = t - lane; tb < m; tb += stride) {
        const int tt = tb + lane;
        int c = -1, x = 0, y = 0, z = 0;
        if (tt < m) {
            const int i = a.list[tt];
            const int p = a.L[i];
            const int code = p >= 0 ? a.L[p] : p;   // a non-root points at its root
            c = -2 - code;
            if (p >= 0) a.L[i] = code;
            pos_of(a, (uint32_t)i, x, y, z);
        }
        unsigned long long pending = __ballot(c >= 0);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int cl = __shfl(c, leader);
            const bool mine = c == cl;
            const unsigned long long m = __ballot(mine);
            const int x0 = wave_min_i(mine ? x : INT_MAX), x1 = wave_max_i(mine ? x : -1);
            const int y0 = wave_min_i(mine ? y : INT_MAX), y1 = wave_max_i(mine ? y : -1);
            const int z0 = wave_min_i(mine ? z : INT_MAX), z1 = wave_max_i(mine ? z : -1);
            if (lane == leader) {
                int *b = a.box + 8 * (int64_t)cl;
                atomicMin(b + 0, x0); atomicMax(b + 1, x1);
                atomicMin(b + 2, y0); atomicMax(b + 3, y1);
                atomicMin(b + 4, z0); atomicMax(b + 5, z1);
                atomicAdd(b + 6, __popcll(m));
            }
            pending &= ~m;
        }
    }
}

__global__ __launch_bounds__(256) void k_link_label(LinkArgs a) {
    const int64_t n = a.nx * a.ny * a.nz;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        // a detected voxel's link holds its detection's code (-2 - number)
        const int p = a.mask[i] ? a.L[i] : 0;
        a.L[i] = p <= -2 ? a.label_of[-2 - p] : 0;
    }
}

// Boxes of the kept detections in label order: x0, x1, y0, y1, z0, z1, count.
__global__ __launch_bounds__(256) void k_link_boxes_out(LinkArgs a, int64_t nc,
                                                        long long *out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += stride) {
        const int l = a.label_of[c];
        if (!l) continue;
        const int *b = a.box + 8 * c;
        long long *o = out + 7 * (int64_t)(l - 1);
        for (int k = 0; k < 7; ++k) o[k] = b[k];
    }
}

namespace {
unsigned grid_of(int64_t n, int per) {
    const int64_t g = (n + per - 1) / per;
    return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}
}  // namespace

hipError_t launch_link_init(const LinkArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_link_init, dim3(grid_of(a.m, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_link_union(const LinkArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_link_union, dim3(grid_of(a.m, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_link_flatten(const LinkArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_link_flatten, dim3(grid_of(a.m, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

int64_t link_scan_blocks(int64_t n) { return (n + kScanItems - 1) / kScanItems; }

hipError_t launch_link_number(int items, const LinkArgs &a, int64_t n, int *counts,
                              hipStream_t s) {
    const int64_t nb = link_scan_blocks(n);
    if (nb < 1 || nb > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 g((unsigned)nb), b(kScanThreads);
    if (items == LK_VOXELS)
        hipLaunchKernelGGL(k_link_count<LK_VOXELS>, g, b, 0, s, a, n, counts);
    else if (items == LK_ROOTS)
        hipLaunchKernelGGL(k_link_count<LK_ROOTS>, g, b, 0, s, a, n, counts);
    else
        hipLaunchKernelGGL(k_link_count<LK_KEPT>, g, b, 0, s, a, n, counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_link_scan, dim3(1), dim3(kScanThreads), 0, s, counts, nb);
    return hipGetLastError();
}

hipError_t launch_link_assign(int items, const LinkArgs &a, int64_t n, const int *counts,
                              hipStream_t s) {
    const int64_t nb = link_scan_blocks(n);
    const dim3 g((unsigned)nb), b(kScanThreads);
    if (items == LK_VOXELS)
        hipLaunchKernelGGL(k_link_assign<LK_VOXELS>, g, b, 0, s, a, n, counts);
    else if (items == LK_ROOTS)
        hipLaunchKernelGGL(k_link_assign<LK_ROOTS>, g, b, 0, s, a, n, counts);
    else
        hipLaunchKernelGGL(k_link_assign<LK_KEPT>, g, b, 0, s, a, n, counts);
    return hipGetLastError();
}

hipError_t launch_link_resolve(const LinkArgs &a, int64_t nc, hipStream_t s) {
    hipLaunchKernelGGL(k_link_box_init, dim3(grid_of(nc, 256)), dim3(256), 0, s, a.box, nc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_link_resolve, dim3(grid_of(a.m, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_link_label(const LinkArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_link_label, dim3(grid_of(a.nx * a.ny * a.nz, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_link_boxes_out(const LinkArgs &a, int64_t nc, long long *out, hipStream_t s) {
    hipLaunchKernelGGL(k_link_boxes_out, dim3(grid_of(nc, 256)), dim3(256), 0, s, a, nc, out);
    return hipGetLastError();
}

}  // namespace sc
