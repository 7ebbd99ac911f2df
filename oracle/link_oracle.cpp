/*
 * TEST INFRASTRUCTURE: plain CPU oracle of SoFiA 2's linker (Westmeier et
 * al. 2021, arXiv:2106.15789, Sect. 4.3).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this library. It shares no code with the GPU library or the other oracles.
 *
 * What the paper fixes: the linker merges the detected voxels of the binary
 * mask into individual detections with a friends-of-friends rule that links
 * every pair of voxels within a merging radius, in the spatial plane and
 * along the spectral axis alike (3-D sources), gives each detection a unique
 * identifier, and can drop detections smaller or larger than given spatial
 * and spectral sizes (Sect. 4.3). The mock-galaxy run uses a radius of 2
 * pixels/channels and minimum sizes of 8 pixels and 5 channels (Sect. 6).
 *
 * Readings where the paper is silent (each listed with its reason in the
 * design notes):
 *  L1 two detected voxels are friends when their offset (dx, dy, dz) lies in
 *     the ellipsoid (dx^2 + dy^2) / r_xy^2 + dz^2 / r_z^2 <= 1; an axis with
 *     radius 0 admits only offset 0 along it;
 *  L2 a detection is a connected component of the friendship graph;
 *  L3 its size is its bounding-box extent (max - min + 1) along x, y and z;
 *     it is dropped when the extent along x or y is below min_xy, or along z
 *     below min_z, or (for max_xy > 0, max_z > 0) above those maxima;
 *  L4 kept detections are numbered 1, 2, ... in the raster order (z, then y,
 *     then x) of their first voxel; every other voxel gets 0.
 *
 * The oracle is a breadth-first flood fill from every unvisited detected
 * voxel, taken in raster order, over every offset of the ellipsoid.
 */
#include <cstddef>
#include <cstdint>
#include <deque>
#include <vector>

namespace {

struct Off {
    int dx, dy, dz;
};

// L1: every offset of the ellipsoid except (0, 0, 0).
std::vector<Off> ellipsoid(int rxy, int rz) {
    std::vector<Off> v;
    const int64_t a = (int64_t)rxy * rxy, c = (int64_t)rz * rz;
    for (int dz = -rz; dz <= rz; ++dz)
        for (int dy = -rxy; dy <= rxy; ++dy)
            for (int dx = -rxy; dx <= rxy; ++dx) {
                if (dx == 0 && dy == 0 && dz == 0) continue;
                const int64_t sxy = (int64_t)dx * dx + (int64_t)dy * dy;
                const int64_t sz = (int64_t)dz * dz;
                bool in;
                if (rxy > 0 && rz > 0) in = sxy * c + sz * a <= a * c;
                else if (rxy > 0) in = sz == 0 && sxy <= a;
                else if (rz > 0) in = sxy == 0 && sz <= c;
                else in = false;
                if (in) v.push_back({dx, dy, dz});
            }
    return v;
}

}  // namespace

extern "C" {

// Link the detected voxels (mask != 0) of a [nz][ny][nx] mask. labels
// [nz][ny][nx] (int32) receives 1..n for kept detections and 0 elsewhere;
// *n_out the number of kept detections. When bbox is not null it receives,
// per kept detection in label order, x_min, x_max, y_min, y_max, z_min,
// z_max and the voxel count (7 int64 each, at most cap detections).
// Returns 0, or -1 for bad arguments.
int lko_link(const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz, int32_t rxy,
             int32_t rz, int32_t min_xy, int32_t min_z, int32_t max_xy, int32_t max_z,
             int32_t *labels, int64_t *n_out, int64_t *bbox, int64_t cap) {
    if (!mask || !labels || !n_out || nx < 1 || ny < 1 || nz < 1) return -1;
    if (rxy < 0 || rz < 0 || min_xy < 0 || min_z < 0 || max_xy < 0 || max_z < 0) return -1;
    const int64_t N = nx * ny * nz;
    const std::vector<Off> offs = ellipsoid(rxy, rz);
    // provisional component of every voxel (-1: not detected or not yet seen)
    std::vector<int64_t> comp((size_t)N, -1);
    struct Box {
        int64_t x0, x1, y0, y1, z0, z1, count;
    };
    std::vector<Box> boxes;
    std::deque<int64_t> queue;
    for (int64_t start = 0; start < N; ++start) {
        if (!mask[start] || comp[(size_t)start] >= 0) continue;
        const int64_t id = (int64_t)boxes.size();
        Box b{nx, -1, ny, -1, nz, -1, 0};
        comp[(size_t)start] = id;
        queue.push_back(start);
        while (!queue.empty()) {
            const int64_t i = queue.front();
            queue.pop_front();
            const int64_t x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
            if (x < b.x0) b.x0 = x;
            if (x > b.x1) b.x1 = x;
            if (y < b.y0) b.y0 = y;
            if (y > b.y1) b.y1 = y;
            if (z < b.z0) b.z0 = z;
            if (z > b.z1) b.z1 = z;
            b.count += 1;
            for (const Off &o : offs) {
                const int64_t xx = x + o.dx, yy = y + o.dy, zz = z + o.dz;
                if (xx < 0 || xx >= nx || yy < 0 || yy >= ny || zz < 0 || zz >= nz) continue;
                const int64_t j = (zz * ny + yy) * nx + xx;
                if (mask[j] && comp[(size_t)j] < 0) {
                    comp[(size_t)j] = id;
                    queue.push_back(j);
                }
            }
        }
        boxes.push_back(b);
    }
    // L3, L4: keep or drop, and number the kept ones in discovery order,
    // which is the raster order of their first voxel
    std::vector<int32_t> label_of(boxes.size(), 0);
    int64_t n = 0;
    for (size_t k = 0; k < boxes.size(); ++k) {
        const Box &b = boxes[k];
        const int64_t ex = b.x1 - b.x0 + 1, ey = b.y1 - b.y0 + 1, ez = b.z1 - b.z0 + 1;
        bool keep = ex >= min_xy && ey >= min_xy && ez >= min_z;
        if (max_xy > 0 && (ex > max_xy || ey > max_xy)) keep = false;
        if (max_z > 0 && ez > max_z) keep = false;
        if (!keep) continue;
        if (bbox && n < cap) {
            int64_t *o = bbox + 7 * n;
            o[0] = b.x0; o[1] = b.x1; o[2] = b.y0; o[3] = b.y1; o[4] = b.z0; o[5] = b.z1;
            o[6] = b.count;
        }
        label_of[k] = (int32_t)(++n);
    }
    for (int64_t i = 0; i < N; ++i)
        labels[i] = comp[(size_t)i] >= 0 ? label_of[(size_t)comp[(size_t)i]] : 0;
    *n_out = n;
    return 0;
}

}  // extern "C"
