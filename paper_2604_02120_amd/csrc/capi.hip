// The C ABI of libgsblend (declared in include/gsblend.h): host-side validation, device check,
// error strings, and dispatch to the binning and blending launchers.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "gsb_internal.h"

namespace gsb {

int64_t bin_max_gaussians();
int64_t bin_max_pairs();

namespace {
thread_local char g_err[512] = "";

constexpr int32_t kMaxDim = 65536;
constexpr int32_t kMaxViews = 4096;
constexpr int kMaxDevices = 64;
int g_arch_ok[kMaxDevices];   // 0 = unknown, 1 = gfx950, 2 = other

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

gsb_status check_device() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(GSB_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(GSB_ERR_UNSUPPORTED, "device id %d out of range", dev);
    if (g_arch_ok[dev] == 0) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return fail(GSB_ERR_HIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
        g_arch_ok[dev] = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
    }
    if (g_arch_ok[dev] != 1) return fail(GSB_ERR_UNSUPPORTED, "device %d is not gfx950", dev);
    return GSB_OK;
}

gsb_status check_dims(int32_t W, int32_t H) {
    if (W < 1 || H < 1 || W > kMaxDim || H > kMaxDim)
        return fail(GSB_ERR_INVALID, "image size %d x %d outside [1, %d]", W, H, kMaxDim);
    return GSB_OK;
}

#define GSB_TRY(expr)                      \
    do {                                   \
        gsb_status _st = (expr);           \
        if (_st != GSB_OK) return _st;     \
    } while (0)

#define GSB_REQUIRE(cond, ...)                                   \
    do {                                                         \
        if (!(cond)) return fail(GSB_ERR_INVALID, __VA_ARGS__);  \
    } while (0)

gsb_status check_blend_common(int32_t W, int32_t H, const uint32_t *ranges,
                              const uint32_t *point_list, const float *means2d,
                              const float *conics, const float *opacity, const float *colors,
                              int64_t n, const float *bg, gsb_precision prec) {
    GSB_TRY(check_dims(W, H));
    GSB_REQUIRE(n >= 0 && n <= int64_t(0xffffffffll), "n = %lld out of range", (long long)n);
    GSB_REQUIRE(ranges != nullptr && point_list != nullptr, "ranges and point_list must be non-null");
    GSB_REQUIRE(aligned(ranges, 8), "ranges must be 8-byte aligned");
    GSB_REQUIRE(n == 0 || (means2d && conics && opacity && colors),
                "Gaussian attribute pointers must be non-null");
    GSB_REQUIRE(aligned(means2d, 8), "means2d must be 8-byte aligned");
    GSB_REQUIRE(bg != nullptr, "bg must be a host pointer to 3 floats");
    const gsb_precision base = prec & ~GSB_FULL_SCAN;
    GSB_REQUIRE(base == GSB_FP32_PLAIN || base == GSB_FP16_GEMM || base == GSB_BF16_GEMM,
                "unknown precision %d", int(prec));
    return GSB_OK;
}

// The precision of a (validated) precision argument, and the view's reach setting from its flag.
gsb_precision prec_base(gsb_precision prec) { return prec & ~GSB_FULL_SCAN; }
void set_reach(ViewDesc &v, gsb_precision prec) {
    v.reach = prec_base(prec) == GSB_FP32_PLAIN && (prec & GSB_FULL_SCAN) == 0 ? 1 : 0;
}

}  // namespace

gsb_status fail(gsb_status code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

gsb_status check_launch(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(GSB_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return GSB_OK;
}

}  // namespace gsb

using namespace gsb;

extern "C" {

int32_t gsb_abi_version(void) { return GSB_ABI_VERSION; }

const char *gsb_last_error(void) { return g_err; }

gsb_status gsb_project(const float *means3d, const float *scales, const float *quats,
                       const float *sh, int32_t sh_coeffs, int32_t sh_degree, int64_t n,
                       const gsb_camera *camera, float *means2d, float *conics, float *depths,
                       int32_t *radii, float *colors, void *stream) {
    g_err[0] = '\0';
    GSB_REQUIRE(n >= 0 && n < (int64_t(1) << 31), "n = %lld outside [0, 2^31)", (long long)n);
    GSB_REQUIRE(sh_degree >= 0 && sh_degree <= 3, "sh_degree = %d outside [0, 3]", int(sh_degree));
    GSB_REQUIRE(sh_coeffs >= (sh_degree + 1) * (sh_degree + 1) && sh_coeffs <= 16,
                "sh_coeffs = %d outside [%d, 16]", int(sh_coeffs), (sh_degree + 1) * (sh_degree + 1));
    GSB_REQUIRE(camera != nullptr, "camera must be a non-null host pointer");
    const gsb_camera &c = *camera;
    GSB_TRY(check_dims(c.width, c.height));
    GSB_REQUIRE(isfinite(c.fx) && isfinite(c.fy) && c.fx > 0.0f && c.fy > 0.0f,
                "focal lengths must be finite and positive");
    GSB_REQUIRE(isfinite(c.near) && c.near >= 0.0f, "near plane must be finite and >= 0");
    GSB_REQUIRE(n == 0 || (means3d && scales && quats && sh && means2d && conics && depths &&
                           radii && colors),
                "array pointers must be non-null");
    GSB_REQUIRE(aligned(quats, 16) && aligned(sh, 16), "quats and sh must be 16-byte aligned");
    GSB_REQUIRE(aligned(means2d, 8), "means2d must be 8-byte aligned");
    GSB_REQUIRE(aligned(means3d, 4) && aligned(scales, 4) && aligned(conics, 4) &&
                    aligned(depths, 4) && aligned(radii, 4) && aligned(colors, 4),
                "arrays must be 4-byte aligned");
    GSB_TRY(check_device());
    ProjectArgs a{};
    a.means3d = means3d;
    a.scales = scales;
    a.quats = quats;
    a.sh = sh;
    a.n = n;
    a.deg = sh_degree;
    for (int k = 0; k < 9; ++k) a.cam.R[k] = c.R[k];
    for (int k = 0; k < 3; ++k) a.cam.t[k] = c.t[k];
    a.cam.fx = c.fx;
    a.cam.fy = c.fy;
    a.cam.cx = c.cx;
    a.cam.cy = c.cy;
    a.cam.limx = float(1.3 * (double(c.width) / (2.0 * double(c.fx))));
    a.cam.limy = float(1.3 * (double(c.height) / (2.0 * double(c.fy))));
    a.cam.near = c.near;
    for (int k = 0; k < 3; ++k)
        a.cam.o[k] = float(-(double(c.R[k]) * c.t[0] + double(c.R[3 + k]) * c.t[1] +
                             double(c.R[6 + k]) * c.t[2]));
    a.cam.gx = int32_t(grid_x(c.width));
    a.cam.gy = int32_t(grid_y(c.height));
    a.means2d = means2d;
    a.conics = conics;
    a.depths = depths;
    a.radii = radii;
    a.colors = colors;
    return project(a, sh_coeffs, static_cast<hipStream_t>(stream));
}

gsb_status gsb_bin_workspace_bytes(int64_t n, int64_t pair_capacity, int32_t W, int32_t H,
                                   size_t *bytes) {
    g_err[0] = '\0';
    GSB_TRY(check_dims(W, H));
    GSB_REQUIRE(bytes != nullptr, "bytes must be non-null");
    GSB_REQUIRE(n >= 0 && n <= bin_max_gaussians(), "n = %lld outside [0, %lld]", (long long)n,
                (long long)bin_max_gaussians());
    GSB_REQUIRE(pair_capacity >= 0 && pair_capacity <= bin_max_pairs() &&
                    pair_capacity <= int64_t(0x7fffffff),
                "pair_capacity = %lld outside [0, %lld]", (long long)pair_capacity,
                (long long)(bin_max_pairs() < 0x7fffffff ? bin_max_pairs() : 0x7fffffff));
    *bytes = bin_workspace_bytes(n, pair_capacity, grid_x(W) * grid_y(H));
    return GSB_OK;
}

namespace {
gsb_status check_bin_mode(gsb_bin_mode mode, int64_t n, const float *conics, const float *opacity) {
    GSB_REQUIRE(mode == GSB_BIN_RECT || mode == GSB_BIN_VISIBLE, "unknown binning mode %d", int(mode));
    if (mode == GSB_BIN_VISIBLE && n > 0) {
        GSB_REQUIRE(conics && opacity, "binning mode 1 needs non-null conics and opacity");
        GSB_REQUIRE(aligned(conics, 4) && aligned(opacity, 4), "conics and opacity must be 4-byte aligned");
    }
    return GSB_OK;
}
}  // namespace

gsb_status gsb_bin_count(const float *means2d, const int32_t *radii, const float *conics,
                         const float *opacity, gsb_bin_mode mode, int64_t n, int32_t W,
                         int32_t H, void *ws, size_t ws_bytes, int64_t *n_pairs_dev,
                         void *stream) {
    size_t need = 0;
    GSB_TRY(gsb_bin_workspace_bytes(n, 0, W, H, &need));
    GSB_REQUIRE(n == 0 || (means2d && radii), "means2d and radii must be non-null");
    GSB_REQUIRE(aligned(means2d, 8), "means2d must be 8-byte aligned");
    GSB_TRY(check_bin_mode(mode, n, conics, opacity));
    GSB_REQUIRE(ws != nullptr && aligned(ws, 256), "workspace must be non-null and 256-byte aligned");
    GSB_REQUIRE(ws_bytes >= need, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    GSB_REQUIRE(n_pairs_dev != nullptr && aligned(n_pairs_dev, 8), "n_pairs_dev must be a non-null, 8-byte aligned device pointer");
    GSB_TRY(check_device());
    return bin_count(means2d, radii, conics, opacity, mode, n, W, H, ws, n_pairs_dev,
                     static_cast<hipStream_t>(stream));
}

gsb_status gsb_bin_fill(const float *means2d, const int32_t *radii, const float *conics,
                        const float *opacity, gsb_bin_mode mode, const float *depths, int64_t n,
                        int32_t W, int32_t H, void *ws, size_t ws_bytes, uint32_t *point_list,
                        int64_t pair_capacity, uint32_t *ranges, int32_t *status_dev,
                        void *stream) {
    size_t need = 0;
    GSB_TRY(gsb_bin_workspace_bytes(n, pair_capacity, W, H, &need));
    GSB_REQUIRE(n == 0 || (means2d && radii && depths), "means2d, radii and depths must be non-null");
    GSB_REQUIRE(aligned(means2d, 8), "means2d must be 8-byte aligned");
    GSB_TRY(check_bin_mode(mode, n, conics, opacity));
    GSB_REQUIRE(ws != nullptr && aligned(ws, 256), "workspace must be non-null and 256-byte aligned");
    GSB_REQUIRE(ws_bytes >= need, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    GSB_REQUIRE(pair_capacity == 0 || point_list != nullptr, "point_list must be non-null");
    GSB_REQUIRE(ranges != nullptr && status_dev != nullptr, "ranges and status_dev must be non-null");
    GSB_TRY(check_device());
    return bin_fill(means2d, radii, conics, opacity, mode, depths, n, W, H, ws, point_list,
                    pair_capacity, ranges, status_dev, static_cast<hipStream_t>(stream));
}

gsb_status gsb_bin_noalloc(const float *means2d, const int32_t *radii, const float *conics,
                           const float *opacity, gsb_bin_mode mode, const float *depths,
                           int64_t n, int32_t W, int32_t H, uint32_t *point_list,
                           int64_t pair_capacity, uint32_t *ranges, int64_t *n_pairs_dev,
                           int32_t *status_dev, void *stream) {
    size_t need = 0;
    GSB_TRY(gsb_bin_workspace_bytes(n, pair_capacity, W, H, &need));
    GSB_REQUIRE(need <= GSB_NOALLOC_SCRATCH_BYTES,
                "binning %lld Gaussians into at most %lld pairs needs a %zu-byte workspace, more "
                "than the %zu bytes the library holds", (long long)n, (long long)pair_capacity,
                need, size_t(GSB_NOALLOC_SCRATCH_BYTES));
    GSB_REQUIRE(n == 0 || (means2d && radii && depths), "means2d, radii and depths must be non-null");
    GSB_REQUIRE(aligned(means2d, 8), "means2d must be 8-byte aligned");
    GSB_TRY(check_bin_mode(mode, n, conics, opacity));
    GSB_REQUIRE(pair_capacity == 0 || point_list != nullptr, "point_list must be non-null");
    GSB_REQUIRE(ranges != nullptr && status_dev != nullptr, "ranges and status_dev must be non-null");
    GSB_REQUIRE(n_pairs_dev != nullptr && aligned(n_pairs_dev, 8),
                "n_pairs_dev must be a non-null, 8-byte aligned device pointer");
    GSB_TRY(check_device());
    return bin_noalloc(means2d, radii, conics, opacity, mode, depths, n, W, H, point_list,
                       pair_capacity, ranges, n_pairs_dev, status_dev,
                       static_cast<hipStream_t>(stream));
}

gsb_status gsb_blend_forward(int32_t W, int32_t H, const uint32_t *ranges,
                             const uint32_t *point_list, const float *means2d,
                             const float *conics, const float *opacity, const float *colors,
                             int64_t n, const float *bg, gsb_precision prec, float *image,
                             float *final_T, int32_t *last_contrib, void *stream) {
    g_err[0] = '\0';
    GSB_TRY(check_blend_common(W, H, ranges, point_list, means2d, conics, opacity, colors, n, bg, prec));
    GSB_REQUIRE(image && final_T && last_contrib, "output pointers must be non-null");
    GSB_TRY(check_device());
    ViewDesc v = make_view(W, H, ranges, point_list, means2d, conics, opacity, colors, n, bg);
    v.image = image;
    v.final_T = final_T;
    v.last_contrib = last_contrib;
    set_reach(v, prec);
    return blend_forward(v, prec_base(prec), kDefaultBatchFwd, static_cast<hipStream_t>(stream));
}

gsb_status gsb_blend_backward(int32_t W, int32_t H, const uint32_t *ranges,
                              const uint32_t *point_list, const float *means2d,
                              const float *conics, const float *opacity, const float *colors,
                              int64_t n, const float *bg, gsb_precision prec,
                              const float *final_T, const int32_t *last_contrib,
                              const float *dL_dimage, float *dL_dmeans2d, float *dL_dconics,
                              float *dL_dopacity, float *dL_dcolors, void *stream) {
    g_err[0] = '\0';
    GSB_TRY(check_blend_common(W, H, ranges, point_list, means2d, conics, opacity, colors, n, bg, prec));
    GSB_REQUIRE(final_T && last_contrib && dL_dimage, "final_T, last_contrib and dL_dimage must be non-null");
    GSB_REQUIRE(n == 0 || (dL_dmeans2d && dL_dconics && dL_dopacity && dL_dcolors),
                "gradient pointers must be non-null");
    GSB_REQUIRE(aligned(dL_dmeans2d, 8), "dL_dmeans2d must be 8-byte aligned");
    GSB_TRY(check_device());
    ViewDesc v = make_view(W, H, ranges, point_list, means2d, conics, opacity, colors, n, bg);
    v.final_T = const_cast<float *>(final_T);
    v.last_contrib = const_cast<int32_t *>(last_contrib);
    v.dL_dimage = dL_dimage;
    v.dL_dmeans2d = dL_dmeans2d;
    v.dL_dconics = dL_dconics;
    v.dL_dopacity = dL_dopacity;
    v.dL_dcolors = dL_dcolors;
    set_reach(v, prec);
    return blend_backward(v, prec_base(prec), kDefaultBatchBwd, false, static_cast<hipStream_t>(stream));
}

gsb_status gsb_pack_gaussians(const float *means2d, const float *conics, const float *opacity,
                              const float *colors, int64_t n, float *records, void *stream) {
    g_err[0] = '\0';
    GSB_REQUIRE(n >= 0 && n <= int64_t(0xffffffffll), "n = %lld out of range", (long long)n);
    GSB_REQUIRE(n == 0 || (means2d && conics && opacity && colors && records),
                "array pointers must be non-null");
    GSB_REQUIRE(aligned(means2d, 8) && aligned(records, 16),
                "means2d must be 8-byte and records 16-byte aligned");
    GSB_TRY(check_device());
    return pack_gaussians(means2d, conics, opacity, colors, n, records,
                          static_cast<hipStream_t>(stream));
}

gsb_status gsb_blend_forward_packed(int32_t W, int32_t H, const uint32_t *ranges,
                                    const uint32_t *point_list, const float *records, int64_t n,
                                    const float *bg, gsb_precision prec, float *image,
                                    float *final_T, int32_t *last_contrib, void *stream) {
    g_err[0] = '\0';
    GSB_REQUIRE(aligned(records, 16), "records must be 16-byte aligned");
    GSB_TRY(check_blend_common(W, H, ranges, point_list, records, records, records, records, n,
                               bg, prec));
    GSB_REQUIRE(image && final_T && last_contrib, "output pointers must be non-null");
    GSB_TRY(check_device());
    ViewDesc v = make_view(W, H, ranges, point_list, nullptr, nullptr, nullptr, nullptr, n, bg);
    v.records = reinterpret_cast<const float4 *>(records);
    v.image = image;
    v.final_T = final_T;
    v.last_contrib = last_contrib;
    set_reach(v, prec);
    return blend_forward_packed(v, prec_base(prec), static_cast<hipStream_t>(stream));
}

gsb_status gsb_blend_backward_packed(int32_t W, int32_t H, const uint32_t *ranges,
                                     const uint32_t *point_list, const float *records, int64_t n,
                                     const float *bg, gsb_precision prec, const float *final_T,
                                     const int32_t *last_contrib, const float *dL_dimage,
                                     float *dL_dmeans2d, float *dL_dconics, float *dL_dopacity,
                                     float *dL_dcolors, void *stream) {
    g_err[0] = '\0';
    GSB_REQUIRE(aligned(records, 16), "records must be 16-byte aligned");
    GSB_TRY(check_blend_common(W, H, ranges, point_list, records, records, records, records, n,
                               bg, prec));
    GSB_REQUIRE(final_T && last_contrib && dL_dimage, "final_T, last_contrib and dL_dimage must be non-null");
    GSB_REQUIRE(n == 0 || (dL_dmeans2d && dL_dconics && dL_dopacity && dL_dcolors),
                "gradient pointers must be non-null");
    GSB_REQUIRE(aligned(dL_dmeans2d, 8), "dL_dmeans2d must be 8-byte aligned");
    GSB_TRY(check_device());
    ViewDesc v = make_view(W, H, ranges, point_list, nullptr, nullptr, nullptr, nullptr, n, bg);
    v.records = reinterpret_cast<const float4 *>(records);
    v.final_T = const_cast<float *>(final_T);
    v.last_contrib = const_cast<int32_t *>(last_contrib);
    v.dL_dimage = dL_dimage;
    v.dL_dmeans2d = dL_dmeans2d;
    v.dL_dconics = dL_dconics;
    v.dL_dopacity = dL_dopacity;
    v.dL_dcolors = dL_dcolors;
    set_reach(v, prec);
    return blend_backward_packed(v, prec_base(prec), static_cast<hipStream_t>(stream));
}

gsb_status gsb_backward_det_workspace_bytes(int64_t n, int64_t pairs, size_t *bytes) {
    g_err[0] = '\0';
    GSB_REQUIRE(bytes != nullptr, "bytes must be non-null");
    GSB_REQUIRE(n >= 0 && n <= int64_t(0xffffffffll), "n = %lld out of range", (long long)n);
    GSB_REQUIRE(pairs >= 0 && pairs <= bin_max_pairs() && pairs <= int64_t(0x7fffffff),
                "pairs = %lld outside [0, %lld]", (long long)pairs,
                (long long)(bin_max_pairs() < 0x7fffffff ? bin_max_pairs() : 0x7fffffff));
    *bytes = backward_det_workspace_bytes(n, pairs);
    return GSB_OK;
}

gsb_status gsb_blend_backward_deterministic(
    int32_t W, int32_t H, const uint32_t *ranges, const uint32_t *point_list, int64_t pairs,
    const float *records, int64_t n, const float *bg, gsb_precision prec, const float *final_T,
    const int32_t *last_contrib, const float *dL_dimage, void *ws, size_t ws_bytes,
    float *dL_dmeans2d, float *dL_dconics, float *dL_dopacity, float *dL_dcolors, void *stream) {
    size_t need = 0;
    GSB_TRY(gsb_backward_det_workspace_bytes(n, pairs, &need));
    GSB_REQUIRE(aligned(records, 16), "records must be 16-byte aligned");
    GSB_TRY(check_blend_common(W, H, ranges, point_list, records, records, records, records, n,
                               bg, prec));
    GSB_REQUIRE(final_T && last_contrib && dL_dimage, "final_T, last_contrib and dL_dimage must be non-null");
    GSB_REQUIRE(n == 0 || (dL_dmeans2d && dL_dconics && dL_dopacity && dL_dcolors),
                "gradient pointers must be non-null");
    GSB_REQUIRE(aligned(dL_dmeans2d, 8), "dL_dmeans2d must be 8-byte aligned");
    GSB_REQUIRE(ws != nullptr && aligned(ws, 256), "workspace must be non-null and 256-byte aligned");
    GSB_REQUIRE(ws_bytes >= need, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    GSB_TRY(check_device());
    ViewDesc v = make_view(W, H, ranges, point_list, nullptr, nullptr, nullptr, nullptr, n, bg);
    v.records = reinterpret_cast<const float4 *>(records);
    v.final_T = const_cast<float *>(final_T);
    v.last_contrib = const_cast<int32_t *>(last_contrib);
    v.dL_dimage = dL_dimage;
    v.dL_dmeans2d = dL_dmeans2d;
    v.dL_dconics = dL_dconics;
    v.dL_dopacity = dL_dopacity;
    v.dL_dcolors = dL_dcolors;
    set_reach(v, prec);
    return blend_backward_det(v, prec_base(prec), pairs, ws, static_cast<hipStream_t>(stream));
}

gsb_status gsb_plan_create(const gsb_view *views, int32_t n_views, gsb_precision prec,
                           const gsb_tuning *tuning, gsb_plan *plan) {
    g_err[0] = '\0';
    GSB_REQUIRE(plan != nullptr, "plan must be non-null");
    *plan = nullptr;
    GSB_REQUIRE(n_views >= 1 && n_views <= kMaxViews, "n_views = %d outside [1, %d]", int(n_views), kMaxViews);
    GSB_REQUIRE(views != nullptr, "views must be non-null");
    GSB_REQUIRE(prec_base(prec) == GSB_FP32_PLAIN || prec_base(prec) == GSB_FP16_GEMM ||
                    prec_base(prec) == GSB_BF16_GEMM,
                "unknown precision %d", int(prec));
    Tuning t{kDefaultBatchFwd, kDefaultBatchBwd, 0, kLaunchPersistent, 0};
    if (tuning) {
        if (tuning->batch_fwd) t.batch_fwd = tuning->batch_fwd;
        if (tuning->batch_bwd) t.batch_bwd = tuning->batch_bwd;
        t.blocks_per_cu = tuning->blocks_per_cu;
        t.launch = tuning->launch;
        t.bwd_mm = tuning->bwd_reduce;
        GSB_REQUIRE(t.bwd_mm == GSB_REDUCE_VALU || t.bwd_mm == GSB_REDUCE_MFMA,
                    "backward reduction %d unknown", int(t.bwd_mm));
        GSB_REQUIRE(t.blocks_per_cu >= 0, "blocks_per_cu must be >= 0");
        GSB_REQUIRE(t.launch == GSB_LAUNCH_PERSISTENT || t.launch == GSB_LAUNCH_GRID,
                    "launch mode %d unknown", int(t.launch));
    }
    std::vector<ViewDesc> vd(static_cast<size_t>(n_views));
    for (int i = 0; i < n_views; ++i) {
        const gsb_view &u = views[i];
        gsb_status st = check_blend_common(u.width, u.height, u.ranges, u.point_list, u.means2d,
                                           u.conics, u.opacity, u.colors, u.n, u.bg, prec);
        if (st != GSB_OK) return fail(st, "view %d: %s", i, std::string(g_err).c_str());
        GSB_REQUIRE(u.image && u.final_T && u.last_contrib, "view %d: forward outputs must be non-null", i);
        GSB_REQUIRE(u.dL_dimage != nullptr, "view %d: dL_dimage must be non-null", i);
        GSB_REQUIRE(u.n == 0 || (u.dL_dmeans2d && u.dL_dconics && u.dL_dopacity && u.dL_dcolors),
                    "view %d: gradient pointers must be non-null", i);
        GSB_REQUIRE(aligned(u.dL_dmeans2d, 8), "view %d: dL_dmeans2d must be 8-byte aligned", i);
        ViewDesc v = make_view(u.width, u.height, u.ranges, u.point_list, u.means2d, u.conics,
                               u.opacity, u.colors, u.n, u.bg);
        v.image = u.image;
        v.final_T = u.final_T;
        v.last_contrib = u.last_contrib;
        v.dL_dimage = u.dL_dimage;
        v.dL_dmeans2d = u.dL_dmeans2d;
        v.dL_dconics = u.dL_dconics;
        v.dL_dopacity = u.dL_dopacity;
        v.dL_dcolors = u.dL_dcolors;
        set_reach(v, prec);
        vd[size_t(i)] = v;
    }
    GSB_TRY(check_device());
    Plan *p = nullptr;
    GSB_TRY(plan_create(vd.data(), n_views, prec_base(prec), t, &p));
    *plan = reinterpret_cast<gsb_plan>(p);
    return GSB_OK;
}

gsb_status gsb_plan_destroy(gsb_plan plan) {
    g_err[0] = '\0';
    const hipError_t e = plan_destroy(reinterpret_cast<Plan *>(plan));
    if (e != hipSuccess) return fail(GSB_ERR_HIP, "gsb_plan_destroy: %s", hipGetErrorString(e));
    return GSB_OK;
}

gsb_status gsb_blend_batched_forward(gsb_plan plan, void *stream) {
    g_err[0] = '\0';
    GSB_REQUIRE(plan != nullptr, "plan must be non-null");
    GSB_TRY(check_device());
    return plan_forward(reinterpret_cast<Plan *>(plan), static_cast<hipStream_t>(stream));
}

gsb_status gsb_blend_batched_backward(gsb_plan plan, void *stream) {
    g_err[0] = '\0';
    GSB_REQUIRE(plan != nullptr, "plan must be non-null");
    GSB_TRY(check_device());
    return plan_backward(reinterpret_cast<Plan *>(plan), static_cast<hipStream_t>(stream));
}

}  // extern "C"
