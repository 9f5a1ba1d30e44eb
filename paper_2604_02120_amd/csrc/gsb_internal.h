// Internal declarations shared by the HIP translation units of libgsblend (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gsblend.h"

namespace gsb {

constexpr int kTile = 16;             // screen tile edge, pixels
constexpr int kTilePixels = kTile * kTile;
constexpr int kBlock = 256;           // threads per tile block = 4 wavefronts of 64

// Status helpers (capi.hip): record a message for gsb_last_error() and return the code.
gsb_status fail(gsb_status code, const char *fmt, ...);
gsb_status check_launch(const char *what);

// Tile grid of a W x H image.
inline int64_t grid_x(int32_t W) { return (W + kTile - 1) / kTile; }
inline int64_t grid_y(int32_t H) { return (H + kTile - 1) / kTile; }

// Blocks of a tile launch are spread over the 8 XCDs of the MI355X round-robin by the hardware
// dispatcher (block b runs on XCD b % 8). Block b takes rank (b % 8) * chunk + b / 8 of the tile
// order, so every XCD walks one contiguous range of ranks, and the Gaussians shared by the tiles
// it renders at the same time are reused from that XCD's own L2. The order (strip_tile) walks the
// image in strips of kStrip tile rows, column by column within a strip: the few hundred blocks an
// XCD holds at once then cover a compact kStrip-row region instead of one long row of tiles (the
// forward 2-5% and the backward 1-3% faster than plain row-major ranks at 1080p and 4K).
// Blocks past the last tile exit at once.
constexpr int kXcds = 8;
constexpr int kStrip = 8;
inline int64_t xcd_grid(int64_t n_tiles) {
    const int64_t chunk = (n_tiles + kXcds - 1) / kXcds;
    return chunk * kXcds;
}
// Tile of rank r (< n_tiles) of the strip order on a grid gx tiles wide.
__device__ inline int64_t strip_tile(int64_t r, int64_t n_tiles, int64_t gx) {
    const int64_t gy = n_tiles / gx;
    const int64_t s = r / (kStrip * gx), r0 = s * kStrip;
    const int64_t hs = gy - r0 < kStrip ? gy - r0 : kStrip;   // rows of this strip
    const int64_t j = r - s * kStrip * gx;
    return (r0 + j % hs) * gx + j / hs;
}
// Tile of block `block` (>= n_tiles: past the end).
__device__ inline int64_t xcd_tile(int64_t block, int64_t n_tiles, int64_t gx) {
    const int64_t chunk = (n_tiles + kXcds - 1) / kXcds;
    const int64_t r = (block % kXcds) * chunk + block / kXcds;
    return r < n_tiles ? strip_tile(r, n_tiles, gx) : r;
}

// Covered tiles [tx0, tx1) x [ty0, ty1) of a Gaussian at (x, y) with radius r: tx in
// [floor((x - r)/16), floor((x + r + 15)/16)) clamped to [0, gx], same for y. With x = ix + f,
// 0 <= f < 1, and r an integer, floor((x - r)/16) = floor((ix - r)/16) = (ix - r) >> 4 exactly.
// Used by binning (the pairs to emit) and by preprocessing (a Gaussian whose rectangle is empty
// is culled).
struct Rect { int32_t tx0, tx1, ty0, ty1; };

__device__ inline int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ inline Rect tile_rect(float x, float y, int32_t r, int32_t gx, int32_t gy) {
    Rect R{0, 0, 0, 0};
    if (r <= 0) return R;
    // |x|, |y| < 2^24 by contract; the clamp only keeps the integer conversion defined otherwise
    const int64_t ix = int64_t(floorf(fminf(fmaxf(x, -16777216.f), 16777216.f)));
    const int64_t iy = int64_t(floorf(fminf(fmaxf(y, -16777216.f), 16777216.f)));
    R.tx0 = int32_t(clampi((ix - r) >> 4, 0, gx));
    R.tx1 = int32_t(clampi((ix + r + kTile - 1) >> 4, 0, gx));
    R.ty0 = int32_t(clampi((iy - r) >> 4, 0, gy));
    R.ty1 = int32_t(clampi((iy + r + kTile - 1) >> 4, 0, gy));
    return R;
}

// ---- binning (bin.hip)
size_t bin_workspace_bytes(int64_t n, int64_t pair_capacity, int64_t n_tiles);
gsb_status bin_noalloc(const float *means2d, const int32_t *radii, const float *conics,
                       const float *opacity, int32_t mode, const float *depths, int64_t n,
                       int32_t W, int32_t H, uint32_t *point_list, int64_t cap, uint32_t *ranges,
                       int64_t *n_pairs_dev, int32_t *status_dev, hipStream_t s);
gsb_status bin_count(const float *means2d, const int32_t *radii, const float *conics,
                     const float *opacity, int32_t mode, int64_t n, int32_t W, int32_t H, void *ws,
                     int64_t *n_pairs_dev, hipStream_t s);
gsb_status bin_fill(const float *means2d, const int32_t *radii, const float *conics,
                    const float *opacity, int32_t mode, const float *depths, int64_t n, int32_t W,
                    int32_t H, void *ws, uint32_t *point_list, int64_t pair_capacity,
                    uint32_t *ranges, int32_t *status_dev, hipStream_t s);

// ---- preprocessing (project.hip)
struct ProjectCam {
    float R[9], t[3];        // world to camera: p = R m + t (R row-major)
    float fx, fy, cx, cy;
    float limx, limy;        // clamp of x/z and y/z in the Jacobian: 1.3 W / (2 fx), 1.3 H / (2 fy)
    float near;
    float o[3];              // camera centre -R^T t (world)
    int32_t gx, gy;          // tile grid
};
struct ProjectArgs {
    const float *means3d, *scales, *quats, *sh;
    int64_t n;
    int32_t deg, pad;
    ProjectCam cam;
    float *means2d, *conics, *depths;
    int32_t *radii;
    float *colors;
};
gsb_status project(const ProjectArgs &a, int32_t sh_coeffs, hipStream_t s);

// ---- blending (blend.hip)
// Everything one tile launch needs about one view (image): geometry, inputs, outputs. Built on the
// host; passed by value to the single-view kernels and stored in device memory for batches.
struct ViewDesc {
    int32_t W, H, gx;
    int32_t reach;           // plain form, 1: each wavefront skips the staged Gaussians that cannot
                             // reach its quadrant of the tile (0: every Gaussian is evaluated)
    int64_t n_tiles;
    const uint32_t *ranges;
    const uint32_t *point_list;
    int64_t n;
    const float *means2d, *conics, *opacity, *colors;
    const float4 *records;   // packed attributes (gsb_pack_gaussians), read instead of the four
                             // arrays above by the record kernels
    float bg[3];
    float pad1;
    float *image, *final_T;
    int32_t *last_contrib;
    const float *dL_dimage;
    float *dL_dmeans2d, *dL_dconics, *dL_dopacity, *dL_dcolors;
    float *det_partial;       // deterministic backward: per list position, its nine sums
    int64_t det_pairs;        // ... for positions [0, det_pairs)
};

ViewDesc make_view(int32_t W, int32_t H, const uint32_t *ranges, const uint32_t *point_list,
                   const float *means2d, const float *conics, const float *opacity,
                   const float *colors, int64_t n, const float bg[3]);
// Packed per-Gaussian records: 3 float4 per Gaussian, (x, y, A, B), (C, o, r, g), (b, 0, 0, 0).
constexpr int kRecordFloats = 12;
gsb_status pack_gaussians(const float *means2d, const float *conics, const float *opacity,
                          const float *colors, int64_t n, float *records, hipStream_t s);
// Single-view blends that read the packed records (v.records) instead of the four arrays.
gsb_status blend_forward_packed(const ViewDesc &v, gsb_precision prec, hipStream_t s);
gsb_status blend_backward_packed(const ViewDesc &v, gsb_precision prec, hipStream_t s);
// Deterministic backward (records): workspace size for n Gaussians and `pairs` list entries, and
// the call (gradients bit-reproducible run to run).
size_t backward_det_workspace_bytes(int64_t n, int64_t pairs);
gsb_status blend_backward_det(const ViewDesc &v, gsb_precision prec, int64_t pairs, void *ws,
                              hipStream_t s);
// The binning's stable pair sort (bin.hip), for grouping (key, value) pairs by key.
size_t pair_sort_scratch_bytes(int64_t cap);
int pair_sort(uint32_t *ka, uint32_t *kb, uint32_t *va, uint32_t *vb,
              const unsigned long long *count, int64_t cap, int bits, void *scratch,
              hipStream_t s);
void key_ranges(const uint32_t *sorted_keys, const unsigned long long *count, int64_t cap,
                uint32_t *ranges, hipStream_t s);

// Launch shape choices (all have defaults).
struct Tuning {
    int batch_fwd;       // Gaussians per LDS batch in the forward: 64, 128 or 256
    int batch_bwd;       // same for the backward
    int blocks_per_cu;   // persistent batched launches: resident blocks per compute unit
    int launch;          // batched: kLaunchPersistent or kLaunchGrid
    int bwd_mm;          // backward: geometric gradient sums on the matrix cores (1) or VALU (0)
};
constexpr int kLaunchPersistent = 0;
constexpr int kLaunchGrid = 1;
constexpr int kDefaultBatchFwd = 128;
constexpr int kDefaultBatchBwd = 128;

gsb_status blend_forward(const ViewDesc &v, gsb_precision prec, int batch, hipStream_t s);
gsb_status blend_backward(const ViewDesc &v, gsb_precision prec, int batch, bool mm, hipStream_t s);

// Batched (multi-view) persistent launches.
struct Plan;
gsb_status plan_create(const ViewDesc *views, int n_views, gsb_precision prec, const Tuning &t,
                       Plan **out);
hipError_t plan_destroy(Plan *p);   // frees everything; returns the first hipFree error
gsb_status plan_forward(Plan *p, hipStream_t s);
gsb_status plan_backward(Plan *p, hipStream_t s);

}  // namespace gsb
