// Preprocessing (Sec. 2.1(a)): 3D Gaussians seen by a pinhole camera become the 2D Gaussians the
// blend consumes (mean, conic, depth, radius) and get their colour for this view from
// spherical-harmonic coefficients. This is the EWA splatting projection of 3D Gaussian splatting,
// the renderer whose blend the paper replaces.
//
// One lane per Gaussian, 64 consecutive Gaussians per wavefront. The step is bound by HBM: per
// Gaussian it reads 40 bytes of geometry and 12 K bytes of coefficients (K stored per Gaussian,
// 16 for degree 3) and writes 40 bytes. The coefficient rows are long (192 bytes at K = 16), so a
// lane reading its own row would touch a different cache line on every lane of every load; the
// wavefront instead streams its 64 rows as one contiguous block with float4 loads (8 cache lines
// per instruction) into LDS, then each lane reads its row from there. Rows sit in LDS at a stride
// of an odd number of float4s (or of dwords, when a row is not a whole number of float4s), so the
// lanes' reads fall on distinct banks.
#include <type_traits>

#include "gsb_internal.h"

namespace gsb {
namespace {

constexpr int kProjBlock = 256;                      // 4 wavefronts
constexpr int kWave = 64;
constexpr int kWavesPerBlock = kProjBlock / kWave;

template <int K>
struct ShLayout {
    static constexpr int kDw = 3 * K;                 // dwords of one stored row
    static constexpr bool kVec = (kDw % 4) == 0;      // rows are whole float4s
    static constexpr int kQuads = kDw / 4;
    static constexpr int kStride = kVec ? 4 * (kQuads | 1) : (kDw | 1);   // LDS dwords per row
    // elements each lane moves: float4s (vector path) or dwords
    static constexpr int kIt = kVec ? kQuads : kDw;
    // rows go through LDS in two passes of 32 when 64 of them would take more than 8 KB, which
    // halves the LDS of a block (K = 16: 26 KB instead of 53 KB, 6 instead of 3 blocks per CU).
    // With kIt even, the first kIt / 2 elements of every lane are exactly rows 0..31.
    static constexpr int kPasses = (kWave * kStride * 4 > 8192 && kIt % 2 == 0) ? 2 : 1;
    static constexpr int kRowsPerPass = kWave / kPasses;
};

// Real spherical harmonics up to degree 3 at a unit direction (polar axis z), order
// (l, m = -l..l), Condon-Shortley phase kept: the Cartesian polynomials of
//   Y_l^m = sqrt(2) K_l^|m| {cos, sin}(|m| phi) P_l^|m|(cos theta),  K_l^m = sqrt((2l+1)/(4 pi)
//   (l-m)!/(l+m)!),
// whose constants are 1/(2 sqrt(pi)); sqrt(3/(4 pi)); sqrt(15/pi)/2, sqrt(5/pi)/4, sqrt(15/pi)/4;
// sqrt(35/(2 pi))/4, sqrt(105/pi)/2, sqrt(21/(2 pi))/4, sqrt(7/pi)/4, sqrt(105/pi)/4.
__device__ inline void sh_basis(float x, float y, float z, int deg, float (&Y)[16]) {
#pragma unroll
    for (int k = 1; k < 16; ++k) Y[k] = 0.0f;          // bands above deg contribute nothing
    Y[0] = 0.28209479177387814f;
    if (deg < 1) return;
    const float c1 = 0.4886025119029199f;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    const float xy = x * y, yz = y * z, xz = x * z;
    Y[4] = 1.0925484305920792f * xy;
    Y[5] = -1.0925484305920792f * yz;
    Y[6] = 0.31539156525252005f * (2.0f * zz - xx - yy);
    Y[7] = -1.0925484305920792f * xz;
    Y[8] = 0.5462742152960396f * (xx - yy);
    if (deg < 3) return;
    Y[9] = -0.5900435899266435f * y * (3.0f * xx - yy);
    Y[10] = 2.890611442640554f * xy * z;
    Y[11] = -0.4570457994644658f * y * (4.0f * zz - xx - yy);
    Y[12] = 0.3731763325901154f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -0.4570457994644658f * x * (4.0f * zz - xx - yy);
    Y[14] = 1.445305721320277f * z * (xx - yy);
    Y[15] = -0.5900435899266435f * x * (xx - 3.0f * yy);
}

// ab - cd with one rounding of the products' difference (Kahan's 2x2 determinant with FMA)
__device__ inline float diff_of_products(float a, float b, float c, float d) {
    const float w = c * d;
    const float e = fmaf(-c, d, w);
    const float f = fmaf(a, b, -w);
    return f + e;
}

// Wavefront-scope ordering of the LDS staging writes before the reads of other lanes
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Element e of a wavefront's block (float4s or dwords) into its row's LDS slot, for a pass that
// holds rows [r0, r0 + kRowsPerPass).
template <int K, typename T>
__device__ inline void put_elem(float *lds, int e, int r0, const T &v) {
    using L = ShLayout<K>;
    constexpr int kW = L::kVec ? 4 : 1;               // dwords per element
    constexpr int kPerRow = L::kDw / kW;              // elements per row
    const int r = e / kPerRow, c = e - r * kPerRow;
    *reinterpret_cast<T *>(lds + (r - r0) * L::kStride + kW * c) = v;
}

// The lane's row from its LDS slot into registers.
template <int K, typename T>
__device__ inline void get_row(const float *lds, int slot, float (&row)[3 * K]) {
    using L = ShLayout<K>;
    constexpr int kW = L::kVec ? 4 : 1;
    const T *own = reinterpret_cast<const T *>(__builtin_assume_aligned(lds + slot * L::kStride, kW * 4));
#pragma unroll
    for (int c = 0; c < L::kDw / kW; ++c) {
        const T v = own[c];
        if constexpr (L::kVec) {
            row[4 * c] = v.x;
            row[4 * c + 1] = v.y;
            row[4 * c + 2] = v.z;
            row[4 * c + 3] = v.w;
        } else {
            row[c] = v;
        }
    }
}

// Brings the coefficient row of Gaussian g0 + lane into registers (row), for the wavefront's
// Gaussians [g0, g0 + rows). The rows are streamed as one contiguous block and transposed
// through LDS, in kPasses passes of kRowsPerPass rows: a pass stores the elements of its rows
// (with kPasses = 2, the first half of every lane's elements are exactly rows 0..31), then the
// lanes of those rows read theirs back. Loads are unconditional, so that every one is in flight
// before the first wait: an index past the block re-reads the block's last element (inside the
// array) into a row >= rows, which belongs to a lane that has no Gaussian.
template <int K>
__device__ inline void fetch_row(const float *__restrict__ sh, int64_t g0, int rows, float *lds,
                                 int lane, float (&row)[3 * K]) {
    using L = ShLayout<K>;
    using T = typename std::conditional<L::kVec, float4, float>::type;
    constexpr int kW = L::kVec ? 4 : 1;
    constexpr int kHalf = L::kIt / L::kPasses;
    constexpr int kRp = L::kRowsPerPass;
    const T *src = reinterpret_cast<const T *>(sh) + g0 * (L::kDw / kW);
    const int ne = rows * (L::kDw / kW);
    // the two halves in separate arrays (one array indexed across both passes ends up on the
    // stack)
    T lo[kHalf], hi[L::kIt - kHalf > 0 ? L::kIt - kHalf : 1];
#pragma unroll
    for (int it = 0; it < L::kIt; ++it) {
        const int e = lane + kWave * it;
        const T v = src[e < ne ? e : ne - 1];
        if (it < kHalf) lo[it] = v;
        else hi[it - kHalf] = v;
    }
#pragma unroll
    for (int it = 0; it < kHalf; ++it) put_elem<K, T>(lds, lane + kWave * it, 0, lo[it]);
    wave_lds_sync();
    if (lane < kRp) get_row<K, T>(lds, lane, row);
    if constexpr (L::kPasses == 2) {
        wave_lds_sync();
#pragma unroll
        for (int it = kHalf; it < L::kIt; ++it)
            put_elem<K, T>(lds, lane + kWave * it, kRp, hi[it - kHalf]);
        wave_lds_sync();
        if (lane >= kRp) get_row<K, T>(lds, lane - kRp, row);
    }
}

template <int K>
__global__ __launch_bounds__(kProjBlock) void k_project(ProjectArgs a) {
    using L = ShLayout<K>;
    __shared__ __align__(16) float lds_all[kWavesPerBlock][L::kRowsPerPass * L::kStride];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int64_t g0 = (int64_t(blockIdx.x) * kWavesPerBlock + wave) * kWave;
    if (g0 >= a.n) return;                            // whole wavefront past the end
    const int rows = int(a.n - g0 < kWave ? a.n - g0 : kWave);
    const bool active = lane < rows;
    // lanes past the end work on the last Gaussian and store nothing
    const int64_t i = g0 + (active ? lane : rows - 1);

    // every load of the wavefront is issued before the first wait: geometry, then coefficients
    const float mx = a.means3d[3 * i], my = a.means3d[3 * i + 1], mz = a.means3d[3 * i + 2];
    const float sx = a.scales[3 * i], sy = a.scales[3 * i + 1], sz = a.scales[3 * i + 2];
    const float4 q4 = reinterpret_cast<const float4 *>(a.quats)[i];
    float row[L::kDw];
    fetch_row<K>(a.sh, g0, rows, lds_all[wave], lane, row);
    if (!active) return;

    const float *R = a.cam.R;
    const float px = fmaf(R[0], mx, fmaf(R[1], my, fmaf(R[2], mz, a.cam.t[0])));
    const float py = fmaf(R[3], mx, fmaf(R[4], my, fmaf(R[5], mz, a.cam.t[1])));
    const float pz = fmaf(R[6], mx, fmaf(R[7], my, fmaf(R[8], mz, a.cam.t[2])));

    float2 mean2{0.0f, 0.0f};
    float con[3] = {0.0f, 0.0f, 0.0f}, col[3] = {0.0f, 0.0f, 0.0f};
    float depth = 0.0f;
    int32_t radius = 0;
    if (pz > a.cam.near) {                            // false for NaN too
        const float xz = px / pz, yz = py / pz;
        const float u = fmaf(a.cam.fx, xz, a.cam.cx), v = fmaf(a.cam.fy, yz, a.cam.cy);

        // Sigma3 = M M^T with M = Rq diag(s), Rq the rotation of the normalised quaternion
        const float qinv = 1.0f / sqrtf(q4.x * q4.x + q4.y * q4.y + q4.z * q4.z + q4.w * q4.w);
        const float w = q4.x * qinv, x = q4.y * qinv, y = q4.z * qinv, z = q4.w * qinv;
        const float M[3][3] = {
            {(1.0f - 2.0f * (y * y + z * z)) * sx, 2.0f * (x * y - w * z) * sy, 2.0f * (x * z + w * y) * sz},
            {2.0f * (x * y + w * z) * sx, (1.0f - 2.0f * (x * x + z * z)) * sy, 2.0f * (y * z - w * x) * sz},
            {2.0f * (x * z - w * y) * sx, 2.0f * (y * z + w * x) * sy, (1.0f - 2.0f * (x * x + y * y)) * sz}};
        float S3[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = r; c < 3; ++c) {
                S3[r][c] = fmaf(M[r][0], M[c][0], fmaf(M[r][1], M[c][1], M[r][2] * M[c][2]));
                S3[c][r] = S3[r][c];
            }
        // T = J R, J the Jacobian of the pinhole map with x/z, y/z clamped to 1.3x the half field
        // of view (the linearisation stays bounded for Gaussians far outside the image)
        const float cxz = fminf(a.cam.limx, fmaxf(-a.cam.limx, xz));
        const float cyz = fminf(a.cam.limy, fmaxf(-a.cam.limy, yz));
        const float j00 = a.cam.fx / pz, j02 = -a.cam.fx * cxz / pz;
        const float j11 = a.cam.fy / pz, j12 = -a.cam.fy * cyz / pz;
        float T0[3], T1[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T0[c] = fmaf(j00, R[c], j02 * R[6 + c]);
            T1[c] = fmaf(j11, R[3 + c], j12 * R[6 + c]);
        }
        // Sigma2 = T Sigma3 T^T + 0.3 I
        float U0[3], U1[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            U0[c] = fmaf(T0[0], S3[0][c], fmaf(T0[1], S3[1][c], T0[2] * S3[2][c]));
            U1[c] = fmaf(T1[0], S3[0][c], fmaf(T1[1], S3[1][c], T1[2] * S3[2][c]));
        }
        const float sa = fmaf(U0[0], T0[0], fmaf(U0[1], T0[1], U0[2] * T0[2])) + 0.3f;
        const float sb = fmaf(U0[0], T1[0], fmaf(U0[1], T1[1], U0[2] * T1[2]));
        const float sc = fmaf(U1[0], T1[0], fmaf(U1[1], T1[1], U1[2] * T1[2])) + 0.3f;
        const float det = diff_of_products(sa, sc, sb, sb);
        if (det > 0.0f) {
            // mid^2 - det written as ((a - c) / 2)^2 + b^2, free of cancellation
            const float mid = 0.5f * (sa + sc), hd = 0.5f * (sa - sc);
            const float lmax = mid + sqrtf(fmaxf(0.1f, fmaf(hd, hd, sb * sb)));
            const int32_t r = int32_t(ceilf(3.0f * sqrtf(lmax)));
            const Rect box = tile_rect(u, v, r, a.cam.gx, a.cam.gy);
            if (box.tx1 > box.tx0 && box.ty1 > box.ty0) {
                const float idet = 1.0f / det;
                mean2 = make_float2(u, v);
                depth = pz;
                radius = r;
                con[0] = sc * idet;
                con[1] = -sb * idet;
                con[2] = sa * idet;
                // colour for the direction from the camera centre
                const float dx = mx - a.cam.o[0], dy = my - a.cam.o[1], dz = mz - a.cam.o[2];
                const float dinv = 1.0f / sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
                float Y[16];
                sh_basis(dx * dinv, dy * dinv, dz * dinv, a.deg, Y);
                float acc[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) acc[ch] = fmaf(Y[k], row[3 * k + ch], acc[ch]);
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) col[ch] = fmaxf(acc[ch], 0.0f);
            }
        }
    }
    reinterpret_cast<float2 *>(a.means2d)[i] = mean2;
    a.conics[3 * i] = con[0];
    a.conics[3 * i + 1] = con[1];
    a.conics[3 * i + 2] = con[2];
    a.depths[i] = depth;
    a.radii[i] = radius;
    a.colors[3 * i] = col[0];
    a.colors[3 * i + 1] = col[1];
    a.colors[3 * i + 2] = col[2];
}

template <int K>
gsb_status launch_k(const ProjectArgs &a, hipStream_t s) {
    const int64_t blocks = (a.n + kProjBlock - 1) / kProjBlock;
    hipLaunchKernelGGL(k_project<K>, dim3(unsigned(blocks)), dim3(kProjBlock), 0, s, a);
    return check_launch("k_project");
}

}  // namespace

gsb_status project(const ProjectArgs &a, int32_t sh_coeffs, hipStream_t s) {
    if (a.n == 0) return GSB_OK;
    switch (sh_coeffs) {
    case 1: return launch_k<1>(a, s);
    case 2: return launch_k<2>(a, s);
    case 3: return launch_k<3>(a, s);
    case 4: return launch_k<4>(a, s);
    case 5: return launch_k<5>(a, s);
    case 6: return launch_k<6>(a, s);
    case 7: return launch_k<7>(a, s);
    case 8: return launch_k<8>(a, s);
    case 9: return launch_k<9>(a, s);
    case 10: return launch_k<10>(a, s);
    case 11: return launch_k<11>(a, s);
    case 12: return launch_k<12>(a, s);
    case 13: return launch_k<13>(a, s);
    case 14: return launch_k<14>(a, s);
    case 15: return launch_k<15>(a, s);
    case 16: return launch_k<16>(a, s);
    default: return fail(GSB_ERR_INVALID, "sh_coeffs = %d outside [1, 16]", int(sh_coeffs));
    }
}

}  // namespace gsb
