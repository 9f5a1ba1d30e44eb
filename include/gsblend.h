/*
 * gsblend — tile-based front-to-back blending of depth-sorted projected 2D Gaussians on
 * AMD Instinct MI355X (gfx950), with the exponent evaluated either per pixel in FP32 (the
 * classic form) or as a GEMM on the matrix cores (GEMM-GS, DAC'26, arXiv 2604.02120).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Array pointers are DEVICE pointers to contiguous, caller-owned memory (e.g. PyTorch tensors);
 *    `bg` is a HOST pointer to 3 floats. Nothing here allocates or frees device memory and no call
 *    synchronises: work is enqueued on `stream` (a hipStream_t; NULL = the default stream).
 *  - Arguments are validated on the host before anything is enqueued; a call that returns an
 *    error has enqueued nothing and written nothing. The message of the last error of the calling
 *    thread is returned by gsb_last_error().
 *  - Screen tiles are 16x16 pixels; the grid is gx = ceil(W/16) by gy = ceil(H/16) tiles, tile
 *    index t = ty * gx + tx. Pixel (px, py) sits at integer coordinates. Images are planar
 *    [3][H][W] FP32; per-pixel maps are [H][W].
 *  - Gaussian attributes (the data fetched per Gaussian in Alg. 1 of the paper):
 *      means2d  f32[n][2]  projected centre (x, y), pixels
 *      conics   f32[n][3]  (A, B, C) of the inverse 2D covariance [[A, B], [B, C]], Eq. (alpha)
 *      opacity  f32[n]     o in [0, 1]
 *      colors   f32[n][3]  RGB
 *      depths   f32[n]     view depth > 0
 *      radii    i32[n]     screen radius in pixels; 0 = not rendered
 *    Inputs must be finite, conics positive definite, n < 2^32, |x|, |y| < 2^24. Inputs outside
 *    that contract give unspecified values but never an out-of-bounds access.
 *  - Thresholds (FP32): a Gaussian is skipped for a pixel when alpha < 1/255; a pixel stops at the
 *    first Gaussian whose blend would take its transmittance below 1e-4 (that Gaussian is not
 *    blended); alpha = min(0.99, o * exp(min(power, 0))).
 *  - Calls are reentrant; concurrent calls on different streams are allowed.
 */
#ifndef GSBLEND_H
#define GSBLEND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gsb_status;
#define GSB_OK 0
#define GSB_ERR_INVALID 1      /* bad argument (null pointer, size out of range, bad enum) */
#define GSB_ERR_CAPACITY 2     /* pair list larger than the caller's capacity */
#define GSB_ERR_UNSUPPORTED 3  /* device is not gfx950 */
#define GSB_ERR_HIP 4          /* HIP runtime error (message from hipGetErrorString) */
#define GSB_ERR_INTERNAL 5     /* a device-side consistency check failed (a bounded wait of the
                                  pair sort expired); the outputs are unspecified */

typedef int32_t gsb_precision;
#define GSB_FP32_PLAIN 0  /* exponent per pixel in FP32 on the vector ALUs (Alg. 1, Eq. (power)) */
#define GSB_FP16_GEMM 1   /* exponent as an MFMA product, FP16 hi+lo operands, FP32 accumulate */
#define GSB_BF16_GEMM 2   /* same with BF16 hi+lo operands */
/* Flag that may be OR'ed into any precision argument below. Without it, the plain form skips,
 * for each 8x8 quadrant of a tile, the staged Gaussians whose alpha cannot reach 1/255 at any of
 * its pixels (a conservative ellipse test made once per staged Gaussian, Eq. (power) and the
 * 1/255 skip of Alg. 1), so that their exponent is never evaluated there; the outputs are the
 * same bit for bit. GSB_FULL_SCAN evaluates every staged Gaussian at every pixel, the per-pixel
 * loop of Alg. 1 as written. The GEMM forms always evaluate the whole group (one MFMA product
 * gives every exponent of 16 Gaussians), so the flag changes nothing for them. */
#define GSB_FULL_SCAN 0x100

#define GSB_ABI_VERSION 8

/* Version of this interface (GSB_ABI_VERSION of the library that was loaded). */
int32_t gsb_abi_version(void);

/* Message of the last failed call on this thread ("" if none). Valid until the next call made by
 * the same thread. */
const char *gsb_last_error(void);

/* ---------------------------------------------------------------------------------------------
 * Preprocessing (paper Sec. 2.1(a)): 3D Gaussians seen by a pinhole camera become the 2D Gaussians
 * of the blend, with their depth, extent radius and view-dependent colour. The paper names this
 * step and its outputs; the rule is the EWA splatting projection of 3D Gaussian splatting, the
 * renderer whose blend the paper replaces. Per Gaussian i:
 *   p = R m_i + t (camera coordinates); culled if p.z <= near;
 *   means2d = (fx p.x / p.z + cx, fy p.y / p.z + cy), depth = p.z;
 *   Sigma3 = Rq diag(s_i^2) Rq^T, Rq the rotation of the normalised quaternion q_i = (w, x, y, z);
 *   J = d(means2d)/dp = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]] with x/z and y/z clamped to
 *       +-1.3 W / (2 fx) and +-1.3 H / (2 fy);
 *   Sigma2 = J R Sigma3 R^T J^T + 0.3 I = [[a, b], [b, c]]; culled unless det > 0;
 *   conic = (c, -b, a) / det (the (A, B, C) of the blend);
 *   radius = ceil(3 sqrt(lmax)), lmax = mid + sqrt(max(0.1, mid^2 - det)), mid = (a + c) / 2;
 *   culled if the radius square covers no tile of the W x H image (binning rule below);
 *   colour_c = max(0, 0.5 + sum_{k < (deg+1)^2} Y_k(d) sh_i[k][c]), d the unit direction from
 *       the camera centre -R^T t to m_i, Y_k the real spherical harmonics of degree <= 3 in the
 *       order (l, m = -l..l) with the Condon-Shortley phase kept (band 1 is
 *       sqrt(3/(4 pi)) (-y, z, -x)).
 * A culled Gaussian gets radius 0 and zeros in every other output. Opacity needs no
 * preprocessing and is passed to binning and blending as it is.
 * ------------------------------------------------------------------------------------------- */
typedef struct gsb_camera {
    float R[9];               /* world-to-camera rotation, row-major */
    float t[3];               /* world-to-camera translation: p = R m + t */
    float fx, fy;             /* focal lengths, pixels (> 0) */
    float cx, cy;             /* principal point, pixels (pixel (i, j) sits at (i, j)) */
    int32_t width, height;    /* image size, [1, 65536] */
    float near;               /* near plane (>= 0): Gaussians with p.z <= near are culled */
} gsb_camera;

/* means3d f32[n][3], scales f32[n][3] (per-axis standard deviations), quats f32[n][4] (w, x, y,
 * z; 16-byte aligned; non-zero), sh f32[n][sh_coeffs][3] (16-byte aligned), all device.
 * sh_degree in [0, 3] with (sh_degree + 1)^2 <= sh_coeffs <= 16: the first (sh_degree + 1)^2
 * coefficients of each row are used (the whole row is read).
 * camera: host pointer. Outputs (device, overwritten): means2d f32[n][2] (8-byte aligned),
 * conics f32[n][3], depths f32[n], radii i32[n], colors f32[n][3].
 * Computed in FP32. Errors: INVALID (null pointers when n > 0, n outside [0, 2^31), bad degree
 * or coefficient count, a camera with non-positive or non-finite focal lengths, a negative or
 * non-finite near plane, an image size outside [1, 65536], misaligned pointers), UNSUPPORTED,
 * HIP. */
gsb_status gsb_project(const float *means3d, const float *scales, const float *quats,
                       const float *sh, int32_t sh_coeffs, int32_t sh_degree, int64_t n,
                       const gsb_camera *camera, float *means2d, float *conics, float *depths,
                       int32_t *radii, float *colors, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Binning: duplication with tile|depth keys, depth sort and per-tile ranges (paper §2.1(b)-(c);
 * the ranges are the per-tile sorted index lists that Alg. 1 and Alg. 2 take as input).
 *
 * A Gaussian with radius r > 0 at (x, y) covers the tiles tx in [floor((x - r)/16),
 * floor((x + r + 15)/16)) and ty likewise, clamped to the grid. Each covered tile gets one pair
 * with the 64-bit key (t << 32) | bits(depth) and the Gaussian's index as value. Pairs are sorted
 * by key with a stable sort from Gaussian-major emission order, i.e. by (tile, depth, index), so
 * the result is unique and reproducible bit for bit.
 *
 * Use: gsb_bin_workspace_bytes -> gsb_bin_count -> (read *n_pairs, or use a known bound as the
 * capacity) -> gsb_bin_fill, with the same workspace (it carries the per-Gaussian offsets).
 * ------------------------------------------------------------------------------------------- */

/* Workspace size in bytes for n Gaussians, up to pair_capacity pairs, on a W x H image.
 * Errors: INVALID if n < 0 or > 2^24, pair_capacity < 0 or > 2^28, W or H not in [1, 2^16],
 * or bytes == NULL. */
gsb_status gsb_bin_workspace_bytes(int64_t n, int64_t pair_capacity, int32_t W, int32_t H,
                                   size_t *bytes);

/* Binning modes.
 * GSB_BIN_RECT:    every tile of the 3-sigma square above (the method's rule).
 * GSB_BIN_VISIBLE: only the tiles of that square on which the Gaussian can reach alpha >= 1/255
 *   at a pixel inside the image (an opacity-aware extent: the tighter binning that the paper
 *   combines its blend with, Sec. 2.1(c) and the orthogonality study of Sec. 4). A pair is kept
 *   iff o >= fp32(1/255) and the minimum of Q = d^T Sigma^-1 d over the tile's pixel rectangle is
 *   <= 2 (e ln2 + m - 1) + 0.1 with 255 o = m 2^e, m in [1, 2) (an upper bound of 2 ln(255 o),
 *   plus a margin), decided by division-free double-precision tests, reproducibly. A dropped pair
 *   has alpha < (1/255) e^-0.05 on every pixel of its tile, so the blend would skip it: images
 *   and final T are those of GSB_BIN_RECT; last_contrib positions refer to the shorter lists.
 *   Needs conics and opacity (same layouts as for the blend). */
typedef int32_t gsb_bin_mode;
#define GSB_BIN_RECT 0
#define GSB_BIN_VISIBLE 1

/* Counts the pairs each Gaussian emits (kept in `ws`) and writes the total to the device int64
 * *n_pairs_dev. Asynchronous on `stream`.
 * conics, opacity: device f32[n][3], f32[n], read in GSB_BIN_VISIBLE only (may be NULL in
 *            GSB_BIN_RECT). gsb_bin_fill must then be called with the same mode and arrays.
 * ws: device workspace of ws_bytes >= gsb_bin_workspace_bytes(n, 0, W, H) bytes.
 * Errors: INVALID for null pointers (means2d/radii may be null only when n == 0), an unknown mode,
 * bad sizes or a too-small workspace; HIP for launch failures. */
gsb_status gsb_bin_count(const float *means2d, const int32_t *radii, const float *conics,
                         const float *opacity, gsb_bin_mode mode, int64_t n, int32_t W,
                         int32_t H, void *ws, size_t ws_bytes, int64_t *n_pairs_dev,
                         void *stream);

/* Emits, sorts and ranges the pairs counted by the preceding gsb_bin_count on the same `ws`
 * (a workspace at least as large, whose leading gsb_bin_workspace_bytes(n, 0, W, H) bytes are the
 * ones gsb_bin_count wrote). Implementation: the Gaussians are sorted by depth, pairs are emitted
 * in that order and stably sorted on the tile id alone, which yields the same (tile, depth, index)
 * order as sorting the 64-bit keys.
 * point_list: device u32[pair_capacity], receives the Gaussian index of each sorted pair.
 * ranges:     device u32[gx*gy][2], receives [start, end) of each tile in point_list, [0, 0) for
 *             an empty tile.
 * status_dev: device int32, receives GSB_OK, or GSB_ERR_CAPACITY when the pair count exceeds
 *             pair_capacity (then nothing past pair_capacity is written and the contents of
 *             point_list/ranges are unspecified), or GSB_ERR_INTERNAL (see above).
 * ws_bytes must be >= gsb_bin_workspace_bytes(n, pair_capacity, W, H).
 * Errors: INVALID for null pointers, bad sizes, too-small workspace; HIP for launch failures. */
gsb_status gsb_bin_fill(const float *means2d, const int32_t *radii, const float *conics,
                        const float *opacity, gsb_bin_mode mode, const float *depths, int64_t n,
                        int32_t W, int32_t H, void *ws, size_t ws_bytes, uint32_t *point_list,
                        int64_t pair_capacity, uint32_t *ranges, int32_t *status_dev,
                        void *stream);

/* For callers that cannot allocate device memory (code under hipGraph capture, tight serving
 * loops, harnesses that forbid hipMalloc): gsb_bin_count followed by gsb_bin_fill in one call, with
 * the workspace taken from an array that the library holds in device memory instead of a caller
 * buffer. Nothing is allocated or freed, by the library or on its behalf.
 * The array is GSB_NOALLOC_SCRATCH_BYTES (64 MiB) on every GPU the library runs on, held until the
 * process ends; the call fails with INVALID when gsb_bin_workspace_bytes(n, pair_capacity, W, H)
 * exceeds it (e.g. 300,000 Gaussians with 3M pairs fit; a 1080p frame of 1M Gaussians does not).
 * Arguments and results are those of gsb_bin_count + gsb_bin_fill: *n_pairs_dev receives the total
 * pair count; point_list / ranges / status_dev as in gsb_bin_fill (status GSB_ERR_CAPACITY when
 * the count exceeds pair_capacity, which the caller therefore chooses as a bound beforehand).
 * All calls on one GPU share the array: two calls in flight at once on that GPU (on different
 * streams, or from different threads) race and give unspecified results; serialise them.
 * Errors: INVALID (as the two calls, or a workspace larger than the array), UNSUPPORTED, HIP. */
#define GSB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
gsb_status gsb_bin_noalloc(const float *means2d, const int32_t *radii, const float *conics,
                           const float *opacity, gsb_bin_mode mode, const float *depths,
                           int64_t n, int32_t W, int32_t H, uint32_t *point_list,
                           int64_t pair_capacity, uint32_t *ranges, int64_t *n_pairs_dev,
                           int32_t *status_dev, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Forward blend (Eq. (volume-render) with the per-pixel loop of Alg. 1; in the GEMM precisions
 * the exponent comes from M_power = M_g . M_p, Eq. (power rewritten) and Eq. (matrix
 * multiplication), Alg. 2).
 *
 * ranges/point_list: output of binning (u32[gx*gy][2], u32[>= max end]).
 * bg:        host float[3], background added as T_final * bg.
 * prec:      GSB_FP32_PLAIN, GSB_FP16_GEMM or GSB_BF16_GEMM.
 * image:     device f32[3][H][W]  = sum_i alpha_i T_i c_i + T_final * bg.
 * final_T:   device f32[H][W]     transmittance after the last blended Gaussian.
 * last_contrib: device i32[H][W]  1-based position, within the tile's list, of the last blended
 *            Gaussian (0 = none).
 * Every pixel of the image is written. Errors: INVALID (null pointers, sizes, prec), HIP.
 * ------------------------------------------------------------------------------------------- */
gsb_status gsb_blend_forward(int32_t W, int32_t H, const uint32_t *ranges,
                             const uint32_t *point_list, const float *means2d,
                             const float *conics, const float *opacity, const float *colors,
                             int64_t n, const float *bg, gsb_precision prec, float *image,
                             float *final_T, int32_t *last_contrib, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Backward blend: gradient of L = sum(dL_dimage * image) with respect to the stored inputs, for
 * fixed binning. The forward's decisions are replayed exactly (same precision `prec`, same
 * kernels for the exponent), and transmittance is recovered in reverse from final_T:
 * T_i = T_{i+1} / (1 - alpha_i).
 *
 * final_T, last_contrib: the forward's outputs for the same inputs and `prec`.
 * dL_dimage: device f32[3][H][W].
 * Outputs (device, overwritten, not accumulated into):
 *   dL_dmeans2d f32[n][2], dL_dconics f32[n][3] (d/dA, d/dB, d/dC of the stored scalars),
 *   dL_dopacity f32[n], dL_dcolors f32[n][3].
 * A clamp that is active for a pair (alpha at 0.99, or a positive exponent) passes no gradient to
 * the exponent or opacity. Gradient sums use FP32 atomics, so their rounding is not bit-stable
 * from run to run. Errors: INVALID, HIP.
 * ------------------------------------------------------------------------------------------- */
gsb_status gsb_blend_backward(int32_t W, int32_t H, const uint32_t *ranges,
                              const uint32_t *point_list, const float *means2d,
                              const float *conics, const float *opacity, const float *colors,
                              int64_t n, const float *bg, gsb_precision prec,
                              const float *final_T, const int32_t *last_contrib,
                              const float *dL_dimage, float *dL_dmeans2d, float *dL_dconics,
                              float *dL_dopacity, float *dL_dcolors, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Packed attributes. The blend fetches, per list entry, the 9 attributes of one Gaussian (the
 * fetch step of Alg. 1 and Alg. 2). Read from the four input arrays that is four scattered loads,
 * each touching a cache line of its own; gsb_pack_gaussians writes them once per frame as one
 * 48-byte record per Gaussian, which the _packed blends read with three 16-byte loads.
 *
 * records: device f32[n][GSB_RECORD_FLOATS], 16-byte aligned; record i is
 *   (x, y, A, B), (C, o, r, g), (b, 0, 0, 0) of Gaussian i.
 * gsb_blend_forward_packed / gsb_blend_backward_packed compute exactly what gsb_blend_forward /
 * gsb_blend_backward compute from the arrays the records were packed from (same arithmetic, same
 * outputs; the gradients up to the order of their FP32 atomic sums), with the default launch shape.
 * Errors: INVALID (null or misaligned pointers, sizes, prec), UNSUPPORTED, HIP.
 * ------------------------------------------------------------------------------------------- */
#define GSB_RECORD_FLOATS 12
gsb_status gsb_pack_gaussians(const float *means2d, const float *conics, const float *opacity,
                              const float *colors, int64_t n, float *records, void *stream);

gsb_status gsb_blend_forward_packed(int32_t W, int32_t H, const uint32_t *ranges,
                                    const uint32_t *point_list, const float *records, int64_t n,
                                    const float *bg, gsb_precision prec, float *image,
                                    float *final_T, int32_t *last_contrib, void *stream);

gsb_status gsb_blend_backward_packed(int32_t W, int32_t H, const uint32_t *ranges,
                                     const uint32_t *point_list, const float *records, int64_t n,
                                     const float *bg, gsb_precision prec, const float *final_T,
                                     const int32_t *last_contrib, const float *dL_dimage,
                                     float *dL_dmeans2d, float *dL_dconics, float *dL_dopacity,
                                     float *dL_dcolors, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Deterministic backward. gsb_blend_backward sums each Gaussian's gradient over the tiles that
 * list it with FP32 atomics, whose order (and so whose rounding) changes from run to run. This
 * call computes the same gradient (the product rule of Eq. (volume-render) and Eq. (alpha), as
 * gsb_blend_backward) with every sum in a fixed order, so that its result is identical bit for bit
 * on every run with the same inputs: per list entry, the wavefronts' sums over the tile's pixels
 * are added in wavefront order and stored at the entry's position; the positions are then grouped
 * by Gaussian with a stable sort and each Gaussian's entries are added in a fixed order (lane l of
 * a wavefront takes entries l, l + 64, ... in list order; the lane sums are combined by a fixed
 * reduction tree).
 *
 * pairs:   number of entries of point_list; every range must lie in [0, pairs) (the binning's
 *          pair count). Entries outside are neither read nor written.
 * records: the packed attributes (gsb_pack_gaussians).
 * ws:      device workspace of ws_bytes >= gsb_backward_det_workspace_bytes(n, pairs) bytes,
 *          256-byte aligned (about 80 bytes per list entry).
 * Other arguments and the outputs as gsb_blend_backward_packed. Errors: INVALID, UNSUPPORTED, HIP.
 * ------------------------------------------------------------------------------------------- */
gsb_status gsb_backward_det_workspace_bytes(int64_t n, int64_t pairs, size_t *bytes);

gsb_status gsb_blend_backward_deterministic(
    int32_t W, int32_t H, const uint32_t *ranges, const uint32_t *point_list, int64_t pairs,
    const float *records, int64_t n, const float *bg, gsb_precision prec, const float *final_T,
    const int32_t *last_contrib, const float *dL_dimage, void *ws, size_t ws_bytes,
    float *dL_dmeans2d, float *dL_dconics, float *dL_dopacity, float *dL_dcolors, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Batched views: many images (views) of uneven size, each with its own Gaussians and binning,
 * blended by ONE launch per direction. The (view, tile) items form 8 queues, one per XCD of the
 * MI355X (each XCD takes a contiguous band of every view), views in order of decreasing Gaussians
 * per tile (heaviest first). By default the launch is persistent: resident blocks pull items from
 * their own XCD's queue and take items from the others once it runs dry; GSB_LAUNCH_GRID instead
 * launches one block per item in the same order. The per-tile computation is exactly gsb_blend_forward /
 * gsb_blend_backward's, so each view's results equal the single-view calls'.
 *
 * A plan holds the view table (device copy), the queue counters and the launch shape. Those are
 * the only device memory the library allocates; gsb_plan_destroy frees them. The pointers in the
 * views are captured at creation: the buffers must stay allocated and in place while the plan is
 * used. Plan calls enqueue only kernels (no memset, no allocation, no synchronisation), so they
 * can be captured into a hipGraph and replayed. Two plan calls in flight at once on different
 * streams would share the queue counters: serialise calls on one plan.
 * ------------------------------------------------------------------------------------------- */
typedef struct gsb_view {
    int32_t width, height;             /* image size W x H */
    int64_t n;                         /* Gaussians of this view */
    const uint32_t *ranges;            /* device u32[gx*gy][2] (from binning) */
    const uint32_t *point_list;        /* device u32[pairs] */
    const float *means2d, *conics, *opacity, *colors;   /* device, shapes as above */
    float bg[3];                       /* background (by value) */
    float *image, *final_T;            /* forward outputs: f32[3][H][W], f32[H][W] */
    int32_t *last_contrib;             /* forward output: i32[H][W] */
    const float *dL_dimage;            /* backward input f32[3][H][W] */
    float *dL_dmeans2d, *dL_dconics, *dL_dopacity, *dL_dcolors;   /* backward outputs */
} gsb_view;

/* Launch shape. Zero fields take the defaults. */
#define GSB_LAUNCH_PERSISTENT 0   /* resident blocks pull items from the per-XCD queues */
#define GSB_LAUNCH_GRID 1         /* one block per item: block b takes item b/8 of queue b%8 */
/* How the backward sums each Gaussian's per-pixel gradient terms over a wavefront's 64 pixels:
 * GSB_REDUCE_VALU: all nine sums by cross-lane adds on the vector ALUs (default);
 * GSB_REDUCE_MFMA: the five geometric sums (of dL/dpower times dx^2, dx dy, dy^2, dx, dy) as a
 *   matrix product of dL/dpower (8 Gaussians x 64 pixels, FP16 hi + lo) with the pixel basis
 *   [1, xb, yb, xb^2, xb yb, yb^2] on the matrix cores, i.e. Eq. (power rewritten) applied in
 *   reverse: dL/dM_g = dL/dM_power . M_p^T; the other four sums stay on the vector ALUs. */
#define GSB_REDUCE_VALU 0
#define GSB_REDUCE_MFMA 1
typedef struct gsb_tuning {
    int32_t batch_fwd;       /* Gaussians staged in LDS per batch, forward: 64, 128, 256 (128) */
    int32_t batch_bwd;       /* same, backward (128) */
    int32_t blocks_per_cu;   /* persistent: resident blocks per compute unit; 0 = as many as fit */
    int32_t launch;          /* GSB_LAUNCH_PERSISTENT (default) or GSB_LAUNCH_GRID */
    int32_t bwd_reduce;      /* GSB_REDUCE_VALU (default) or GSB_REDUCE_MFMA */
} gsb_tuning;

typedef struct gsb_plan_s *gsb_plan;

/* Validates every view as gsb_blend_forward / gsb_blend_backward would (all outputs, including
 * the gradients, must be given), uploads the view table and sizes the persistent grids.
 * tuning may be NULL. On error *plan is NULL and nothing is allocated.
 * Errors: INVALID, UNSUPPORTED, HIP. */
gsb_status gsb_plan_create(const gsb_view *views, int32_t n_views, gsb_precision prec,
                           const gsb_tuning *tuning, gsb_plan *plan);

/* Frees the plan (NULL is allowed). Call once the stream work that uses it has completed. */
gsb_status gsb_plan_destroy(gsb_plan plan);

/* Forward of every view of the plan (as gsb_blend_forward per view). */
gsb_status gsb_blend_batched_forward(gsb_plan plan, void *stream);

/* Backward of every view (as gsb_blend_backward per view); the views' final_T and last_contrib
 * must hold the forward's outputs. */
gsb_status gsb_blend_batched_backward(gsb_plan plan, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GSBLEND_H */
