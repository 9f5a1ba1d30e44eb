// Tile blending of depth-sorted projected 2D Gaussians on gfx950: forward (Eq. (volume-render)
// with the per-pixel loop of Alg. 1) and backward, with the Gaussian exponent evaluated either
//   PLAIN : per pixel on the vector ALUs in FP32 from Eq. (power), or
//   F16 / BF16 : as the product M_power = M_g . M_p of Eq. (power rewritten) / Eq. (matrix
//          multiplication) on the matrix cores (MFMA), FP16 or BF16 operands, FP32 accumulation.
//
// Launch shape: one 256-thread block (4 wavefronts) per 16x16 tile, one pixel per lane; wave w
// owns the 8x8 quadrant (w mod 2, w div 2) of the tile. The tile's sorted list is walked in
// batches of NB Gaussians (a template parameter: 64, 128 or 256): every thread below NB stages
// one Gaussian into LDS (double-buffered; the next batch's global loads are issued before the
// current batch is composited), then each wave composites the batch for its pixels, 16 Gaussians
// (one MFMA group) at a time.
//
// Exponent in log2 units. With L = log2(e), every path evaluates
//     q = L * power + log2(o),   alpha = min(0.99, 2^min(q, log2 o))  (= min(0.99, o e^min(power,0)))
// and skips a pair when q < log2(1/255) (alpha < 1/255), so culled pairs never reach exp2. A
// Gaussian with o < 1/255 can never pass and is staged as inert.
//
// GEMM form. Relative to the tile centre (x_c, y_c) = (x0 + 7.5, y0 + 7.5) (the reference pixel of
// Eq. 4), pixel basis v_p = [xb^2, yb^2, xb yb, xb, yb] with xb = x_c - px (quarter-integers, exact
// in FP16 and BF16) and Gaussian row v_g = L [-A/2, -C/2, -B, -(A xh + B yh), -(C yh + B xh)] with
// xh = x - x_c; the constant term L(-A xh^2/2 - C yh^2/2 - B xh yh) + log2 o is the FP32
// accumulator init. v_g is split into hi + lo terms in the 16-bit format (lo scaled by 2^12 to stay
// clear of FP16 subnormals, with the basis scaled by 2^-12 for that product, both exact), so the two
// MFMAs recover ~22 (FP16) / ~16 (BF16) significant bits of v_g.
//
// Conditioning. Needle-like Gaussians (axis ratio up to ~100) make the quadratic form a sum of
// terms ~1e5 that cancel to O(1); evaluated naively in FP32 the exponent is off by up to ~1e-2.
// Both paths therefore evaluate Q = d^T Sigma^-1 d as dx*gx + dy*gy with g = Sigma^-1 d, where each
// product A*dx's rounding error is recovered exactly with an FMA and added back, so g (small along
// the needle, where the cancellation happens) carries full FP32 relative accuracy. The plain path
// does this per pair; the GEMM path once per staged Gaussian, for v_g[3], v_g[4] and the constant.
//
// MFMA packing (v_mfma_f32_32x32x16_{f16,bf16}): lane l supplies A[l%32][8(l/32)..+7] and
// B[8(l/32)..+7][l%32]; accumulator register v of lane l holds D[8(v/4) + 4(l/32) + v%4][l%32].
// B is each lane's own pixel basis. A is block-diagonal: row i carries v_g of Gaussian
// 4(i/8) + i%4 in k-block (i/4)%2 and zeros in the other, so register v of lane l ends up holding
// q of Gaussian v of the group for pixel l: one MFMA pair yields 16 Gaussians x 64 pixels in
// exactly the "lane = pixel, register = next Gaussian in depth order" layout that compositing
// needs, with no shuffles.
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>
#include <cstddef>
#include <type_traits>
#include <vector>

#include "gsb_internal.h"

namespace gsb {
namespace {

enum class Mode { Plain, F16, BF16 };

constexpr int kGroup = 16;                  // Gaussians per MFMA group
constexpr float kLog2e = 0x1.715476p+0f;    // log2(e) rounded to FP32
constexpr float kQCull = -0x1.ffa37cp+2f;   // log2(fp32(1/255)) rounded to FP32
constexpr float kTauCull = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
// The 0.99 clamp applied before the exponential: v_exp_f32 is monotonic near log2(0.99) and
// returns exactly 0.99f for every input from -0x1.db1f6ep-7 to -0x1.db1eb8p-7 (checked over every
// FP32 input in [-0.03, -0.014]), so min(2^x, 0.99f) = 2^min(x, kQAlphaMax) bit for bit, one
// three-way min instead of two mins; 2^x >= 0.99f exactly when x >= kQAlphaMaxLo.
constexpr float kQAlphaMax = -0x1.db1f16p-7f;     // log2f(0.99f)
constexpr float kQAlphaMaxLo = -0x1.db1f6ep-7f;
constexpr float kTStop = 1e-4f;
constexpr float kLoScale = 4096.0f;         // 2^12
constexpr float kLoScaleInv = 1.0f / 4096.0f;
constexpr float kF16Max = 65504.0f;

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4x __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f16x __attribute__((ext_vector_type(16)));

template <Mode M> struct Op;
template <> struct Op<Mode::F16> {
    typedef h8 vec;
    static __device__ inline vec cvt(const float v[8]) {
        vec r;
#pragma unroll
        for (int k = 0; k < 8; ++k) r[k] = _Float16(fminf(fmaxf(v[k], -kF16Max), kF16Max));
        return r;
    }
    static __device__ inline float back(const vec &x, int k) { return float(x[k]); }
    static __device__ inline f16x mfma(vec a, vec b, f16x c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct Op<Mode::BF16> {
    typedef b8 vec;
    static __device__ inline vec cvt(const float v[8]) {
        vec r;
#pragma unroll
        for (int k = 0; k < 8; ++k) r[k] = __bf16(v[k]);
        return r;
    }
    static __device__ inline float back(const vec &x, int k) { return float(x[k]); }
    static __device__ inline f16x mfma(vec a, vec b, f16x c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Op<Mode::Plain> { typedef h8 vec; };

// ------------------------------------------------------------------------------- LDS staging
template <Mode M, int NB>
struct Stage {                 // GEMM form
    typedef typename Op<M>::vec vec;
    vec ahi[2][NB];            // v_g hi terms, 5 used of 8
    vec zero_hi;               // zeros: the A operand of the lanes off the block diagonal
    vec alo[2][NB];            // v_g lo terms * 2^12
    vec zero_lo;               // zeros, as far from zero_hi as alo[b][i] is from ahi[b][i]
    float kc[2][NB];           // accumulator init: constant term + log2 o (-inf = inert)
    float4 attr[2][NB];        // (log2 o, r, g, b)
    alignas(16) uint32_t live[2][4];   // forward: whether wavefront w still has a live pixel
};
template <int NB>
struct Stage<Mode::Plain, NB> {  // plain form
    float4 geo[2][NB];         // (x, y, A, B)
    float2 geo2[2][NB];        // (C, log2 o)
    float4 attr[2][NB];        // (log2 o, r, g, b)
    uint16_t reach[2][4][NB / kGroup];   // reach masks per quadrant and group (stage_reach)
    alignas(16) uint32_t live[2][4];   // forward: whether wavefront w still has a live pixel
};

template <int NB>
struct StageBwd {
    float2 bwd[2][NB];         // the mean (x, y)
    // The Gaussian index of each slot of batch b, in ids[b % 3]. The flush of batch
    // b + 1 reads other threads' slots while the next batch is staged; three buffers keep that
    // staging out of the ones being read.
    uint32_t ids[3][NB];
};

constexpr int kGrad = 9;   // per-Gaussian sums kept per batch
// Deterministic backward: each list position's nine sums sit in a 64-byte row of 16 words (the
// last seven zero), so that the per-Gaussian gather, which reads the rows of one Gaussian's
// positions scattered over the whole list, touches one aligned 64-byte segment per position.
constexpr int kDetStride = 16;

// dL/do from the sum of alpha dL/dalpha over the Gaussian's pairs (alpha = o e^power below the 0.99
// clamp): that sum over o. A Gaussian with o < 1/255 is never blended (its sum is zero).
__device__ inline float opacity_grad(float sum, float o) { return o >= kTauCull ? sum / o : 0.f; }

// Per-Gaussian gradient sums of a batch: 9 consecutive words per staged Gaussian, which the
// flush reads as consecutive words across lanes. Two buffers: batch b sums into buffer b & 1
// while batch b + 1's sums are flushed from the other.
template <int NB>
struct BwdAcc {
    float v[2][NB * kGrad];
    // each wavefront's list of the slots with a nonzero sum, built when it flushes
    uint16_t list[kBlock / 64][64];
    __device__ float *slot(int ab, int t) { return v[ab] + t * kGrad; }
};

// Deterministic backward: each wavefront stores its per-batch sums in a slice of its own (no
// atomics); the flush adds the four slices in a fixed order. Two buffers, as BwdAcc.
template <int NB>
struct BwdAccDet {
    float v[2][kBlock / 64][NB * kGrad];
};

// Backward reduction on the matrix cores: each wavefront's dL/dpower values of 8 Gaussians for its
// 64 pixels (one word per (Gaussian, pixel): FP16 hi in the low half, FP16 lo x 2^12 in the high
// half), transposed through LDS into the operand of v_mfma_f32_16x16x32_f16. Rows padded to 68
// words. Row 0 doubles as the 8 x 8 table of the product's results (moments) once the operand has
// been read. The rows are zero whenever a half-group starts.
constexpr int kDgStride = 68;
struct alignas(16) BwdMM {
    uint32_t dg[kBlock / 64][8][kDgStride];
};

// Raw attributes of one list entry, fetched in the prefetch step.
struct GRaw {
    float x, y, A, B, C, o, r, g, b;
    uint32_t id;
    bool valid;
};

struct __attribute__((aligned(4))) F3 { float a, b, c; };

// a*x + b*y to full FP32 relative accuracy: the rounding error of a*x is recovered with an FMA.
__device__ inline float dot2_acc(float a, float x, float b, float y) {
    const float p = __fmul_rn(a, x);
    const float pe = fmaf(a, x, -p);
    return fmaf(b, y, p) + pe;
}
// Q = A dx^2 + 2 B dx dy + C dy^2 as dx*gx + dy*gy with g = Sigma^-1 (dx, dy) from dot2_acc.
__device__ inline float quad_acc(float A, float B, float C, float dx, float dy, float &gx, float &gy) {
    gx = dot2_acc(A, dx, B, dy);
    gy = dot2_acc(C, dy, B, dx);
    return fmaf(dx, gx, __fmul_rn(dy, gy));
}

// A list entry (Gaussian index) loaded ahead of its use. The load is unconditional (an invalid
// slot reads the list's entry `fallback`, which exists) and validity is applied only at the use,
// so that nothing waits for the load before then.
constexpr uint32_t kNoEntry = 0xffffffffu;
struct Entry {
    uint32_t raw;
    bool valid;
    __device__ uint32_t id() const { return valid ? raw : kNoEntry; }
};
__device__ inline Entry load_entry(const uint32_t *plist, int64_t pos, bool valid, int64_t fallback) {
    return Entry{plist[valid ? pos : fallback], valid};
}

// Attributes of the Gaussian `id` (from load_entry). Needs n > 0. An index >= n (kNoEntry, or an
// inconsistent list) gives an invalid entry, which stage() makes inert; its loads read Gaussian 0
// instead, so that no load is conditional: the loads of a batch stay in flight until the batch
// is staged, with no copies of their results (and no waits for them) in between.
__device__ inline GRaw fetch_attrs(uint32_t id, uint32_t n, const float2 *means, const F3 *conics,
                                   const float *opac, const F3 *colors) {
    GRaw g;
    g.valid = id < n;
    g.id = g.valid ? id : 0u;
    const float2 m = means[g.id];
    const F3 c = conics[g.id];
    const F3 col = colors[g.id];
    g.x = m.x; g.y = m.y; g.A = c.a; g.B = c.b; g.C = c.c;
    g.o = opac[g.id];
    g.r = col.a; g.g = col.b; g.b = col.c;
    return g;
}

// Where a tile's Gaussian attributes come from: the four input arrays (four scattered loads per
// list entry, each touching a cache line of its own), or the packed records of
// gsb_pack_gaussians (three 16-byte loads from one 48-byte record). Loads are unconditional in
// both, as in fetch_attrs.
template <bool kPacked> struct Attrs;
template <> struct Attrs<false> {
    const float2 *means;
    const F3 *conics;
    const float *opac;
    const F3 *colors;
    __device__ explicit Attrs(const ViewDesc &v)
        : means(reinterpret_cast<const float2 *>(v.means2d)),
          conics(reinterpret_cast<const F3 *>(v.conics)), opac(v.opacity),
          colors(reinterpret_cast<const F3 *>(v.colors)) {}
    __device__ GRaw fetch(uint32_t id, uint32_t n) const {
        return fetch_attrs(id, n, means, conics, opac, colors);
    }
};
template <> struct Attrs<true> {
    const float4 *rec;
    __device__ explicit Attrs(const ViewDesc &v) : rec(v.records) {}
    __device__ GRaw fetch(uint32_t id, uint32_t n) const {
        GRaw g;
        g.valid = id < n;
        g.id = g.valid ? id : 0u;
        const float4 *r = rec + 3 * size_t(g.id);
        const float4 a = r[0], b = r[1], c = r[2];
        g.x = a.x; g.y = a.y; g.A = a.z; g.B = a.w;
        g.C = b.x; g.o = b.y; g.r = b.z; g.g = b.w;
        g.b = c.x;
        return g;
    }
};

// Reach culling (plain form). A staged Gaussian cannot reach some quadrants of the tile:
// bit w of its mask is clear when no pixel of quadrant (w & 1, w >> 1) can have q >= kQCull, i.e.
// when the pair is skipped (alpha < 1/255) at every pixel of that quadrant. With Q the conic form
// of Eq. (power), q >= kQCull means Q(d) <= t, t = 2 (log2 o - kQCull) / log2 e, and the ellipse
// Q(d) <= t lies within |dx| <= sqrt(t Sxx), |dy| <= sqrt(t Syy) of the centre, with
// Sxx = C / det, Syy = A / det the covariance's diagonal (det = AC - B^2). The test is made
// conservative for the q the kernels compute: t is enlarged by a bound on its rounding error
// (taken as 2^-14 of the magnitudes of the terms it is formed from, far above the FP32 error of
// the per-pixel form), det is formed with the rounding error of B^2 recovered, and the
// half-widths get a relative and an absolute slack. A non-definite or non-finite conic (or a
// negative t) reaches every quadrant. (xh, yh) is the centre relative to the tile centre.
// A wavefront then skips, without evaluating q, the Gaussians that cannot reach its quadrant.
// Only the plain form uses it: there q costs a dozen instructions per pixel, while the GEMM form
// gets the q of a whole group from one product and skips a Gaussian with one compare.
__device__ inline uint32_t reach_mask(const GRaw &g, float lo2o, float xh, float yh) {
    const float gxh = fmaf(g.A, xh, g.B * yh), gyh = fmaf(g.C, yh, g.B * xh);
    const float Qh = fmaf(xh, gxh, yh * gyh);
    const float mag = kLog2e * (28.125f * (fabsf(g.A) + fabsf(g.C)) + 56.25f * fabsf(g.B) +
                                7.5f * (fabsf(gxh) + fabsf(gyh)) + 0.5f * fabsf(Qh)) + fabsf(lo2o);
    const float t = (lo2o - kQCull + fmaf(mag, 0x1p-14f, 0x1p-16f)) * (2.0f / kLog2e);
    const float bb = g.B * g.B;
    const float det = fmaf(g.A, g.C, -bb) - fmaf(g.B, g.B, -bb);
    if (!(det > 0.f)) return 0xfu;
    const float rdet = 1.0f / det;
    const float hx = fmaf(sqrtf(t * g.C * rdet), 1.0f + 0x1p-10f, fmaf(fabsf(xh), 0x1p-18f, 0x1p-6f));
    const float hy = fmaf(sqrtf(t * g.A * rdet), 1.0f + 0x1p-10f, fmaf(fabsf(yh), 0x1p-18f, 0x1p-6f));
    if (!(hx < 3.0e38f && hy < 3.0e38f)) return 0xfu;   // also NaN (A or C not positive, t < 0)
    // pixel columns (rows) of the tile are 0..15 relative to its corner; the centre is at 7.5
    const float xl = xh + 7.5f, yl = yh + 7.5f;
    const bool c0 = xl - hx <= 7.f && xl + hx >= 0.f, c1 = xl - hx <= 15.f && xl + hx >= 8.f;
    const bool r0 = yl - hy <= 7.f && yl + hy >= 0.f, r1 = yl - hy <= 15.f && yl + hy >= 8.f;
    return uint32_t(c0 && r0) | uint32_t(c1 && r0) << 1 | uint32_t(c0 && r1) << 2 |
           uint32_t(c1 && r1) << 3;
}

// The reach masks of a staged batch as one 16-bit word per (quadrant, group): bit u of
// reach[buf][w][g] is set when Gaussian u of group g can reach quadrant w (wavefront w's pixels).
// Called by whole wavefronts (slot = thread).
template <int NB>
__device__ inline void stage_reach(uint32_t m4, int buf, int slot,
                                   uint16_t (&reach)[2][4][NB / kGroup]) {
    const int l = slot & 63;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const unsigned long long bal = __builtin_amdgcn_ballot_w64(((m4 >> w) & 1u) != 0u);
        if (l < 4) reach[buf][w][(slot >> 6) * 4 + l] = uint16_t(bal >> (16 * l));
    }
}

// This wavefront's reach mask of group g (every Gaussian reaches every wavefront in the GEMM form).
template <Mode M, int NB>
__device__ inline uint32_t group_reach(const Stage<M, NB> &S, int buf, int w, int g) {
    if constexpr (M == Mode::Plain) return __builtin_amdgcn_readfirstlane(uint32_t(S.reach[buf][w][g]));
    else return 0xffffu;
}

// Writes one Gaussian into slot `slot` of buffer `buf`. (xc, yc) is the tile centre. `reach`:
// whether the plain form culls by reach (otherwise every Gaussian reaches every quadrant).
template <Mode M, int NB, bool Bwd>
__device__ inline void stage(const GRaw &g, int buf, int slot, float xc, float yc, Stage<M, NB> &S,
                             StageBwd<NB> *SB, bool reach) {
    // a Gaussian with o < 1/255 never reaches the skip threshold (alpha <= o); stage it inert
    const bool live = g.valid && g.o >= kTauCull;
    const float lo2o = live ? __log2f(g.o) : -INFINITY;
    if constexpr (M == Mode::Plain) {
        S.geo[buf][slot] = live ? make_float4(g.x, g.y, g.A, g.B) : make_float4(0.f, 0.f, 0.f, 0.f);
        S.geo2[buf][slot] = make_float2(live ? g.C : 0.f, lo2o);
    } else {
        float hi[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float lo[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float k0 = -INFINITY;
        if (live) {
            const float xh = g.x - xc, yh = g.y - yc;
            float v[5];
            v[0] = -0.5f * kLog2e * g.A;
            v[1] = -0.5f * kLog2e * g.C;
            v[2] = -kLog2e * g.B;
            float gxh, gyh;
            const float Qh = quad_acc(g.A, g.B, g.C, xh, yh, gxh, gyh);
            v[3] = -kLog2e * gxh;
            v[4] = -kLog2e * gyh;
            k0 = fmaf(Qh, -0.5f * kLog2e, lo2o);
#pragma unroll
            for (int k = 0; k < 5; ++k) hi[k] = v[k];
            const typename Op<M>::vec vh = Op<M>::cvt(hi);
#pragma unroll
            for (int k = 0; k < 5; ++k) lo[k] = (v[k] - Op<M>::back(vh, k)) * kLoScale;
        }
        S.ahi[buf][slot] = Op<M>::cvt(hi);
        S.alo[buf][slot] = Op<M>::cvt(lo);
        S.kc[buf][slot] = k0;
    }
    S.attr[buf][slot] = make_float4(lo2o, g.r, g.g, g.b);
    if constexpr (M == Mode::Plain)
        stage_reach<NB>(!reach ? 0xfu : live ? reach_mask(g, lo2o, g.x - xc, g.y - yc) : 0u, buf,
                        slot, S.reach);
    if constexpr (Bwd) {
        SB->bwd[buf][slot] = make_float2(g.x, g.y);
    }
}

// ------------------------------------------------------------------------------- per-lane setup
struct Lane {
    int t, w, l;
    int col, row;            // pixel within tile
    float px, py;            // pixel coordinates
    bool inside;
    // MFMA A-operand read: which staged Gaussian of a group this lane supplies, if any
    bool a_valid;
    int a_g;
};

__device__ inline Lane lane_setup(int64_t tile, int gx, int W, int H) {
    Lane L;
    L.t = threadIdx.x; L.w = L.t >> 6; L.l = L.t & 63;
    // wave w owns the 8x8 quadrant (w & 1, w >> 1) of the tile: compact footprints touch fewer
    // waves than with 4-row strips, so fewer (Gaussian, wave) pairs have work
    L.col = 8 * (L.w & 1) + (L.l & 7);
    L.row = 8 * (L.w >> 1) + (L.l >> 3);
    const int x0 = int(tile % gx) * kTile, y0 = int(tile / gx) * kTile;
    L.px = float(x0 + L.col); L.py = float(y0 + L.row);
    L.inside = (x0 + L.col < W) && (y0 + L.row < H);
    const int i = L.l & 31, h = L.l >> 5;
    L.a_valid = (h == ((i >> 2) & 1));
    L.a_g = 4 * (i >> 3) + (i & 3);
    return L;
}

template <Mode M>
__device__ inline void pixel_basis(const Lane &L, typename Op<M>::vec &bhi, typename Op<M>::vec &blo) {
    if constexpr (M != Mode::Plain) {
        const float xb = 7.5f - float(L.col), yb = 7.5f - float(L.row);
        float v[8] = {xb * xb, yb * yb, xb * yb, xb, yb, 0.f, 0.f, 0.f};
        bhi = Op<M>::cvt(v);
        float s[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] = v[k] * kLoScaleInv;
        blo = Op<M>::cvt(s);
    }
}

// q for 16 consecutive staged Gaussians (group g of buffer buf): one value per register.
// kOnePtr: address the A operands through one per-lane pointer (below); otherwise through a
// select per operand, which holds fewer registers (the forward's 64 keep it at 8 wavefronts per
// SIMD, the one-pointer form's 70 would not).
template <Mode M, int NB, bool kOnePtr>
__device__ inline f16x group_q_mfma(const Stage<M, NB> &S, int buf, int g, const Lane &L,
                                    const typename Op<M>::vec &bhi,
                                    const typename Op<M>::vec &blo) {
    f16x acc;
    const float4 *kc4 = reinterpret_cast<const float4 *>(&S.kc[buf][g * kGroup]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float4 k = kc4[j];
        acc[4 * j + 0] = k.x; acc[4 * j + 1] = k.y; acc[4 * j + 2] = k.z; acc[4 * j + 3] = k.w;
    }
    typedef typename Op<M>::vec vec;
    vec ah, al;
    if constexpr (kOnePtr) {
        // One address per lane: a lane off the diagonal reads zero_hi and zero_lo whatever buf
        // and g are (its steps are 0), and every lane's lo operand lies at one fixed offset from
        // its hi operand, so the lo read takes no address arithmetic of its own (the selects
        // depend on the lane only and leave the loops): one vector instruction per group instead
        // of five.
        const vec *base = L.a_valid ? &S.ahi[0][L.a_g] : &S.zero_hi;
        const int bstep = L.a_valid ? NB : 0, gstep = L.a_valid ? kGroup : 0;
        const vec *ph = base + buf * bstep + g * gstep;
        typedef Stage<M, NB> St;
        constexpr size_t kLoOff = offsetof(St, alo) - offsetof(St, ahi);
        static_assert(offsetof(St, zero_lo) - offsetof(St, zero_hi) == kLoOff,
                      "zero_lo must mirror zero_hi");
        ah = *ph;
        al = *reinterpret_cast<const vec *>(reinterpret_cast<const char *>(ph) + kLoOff);
    } else {
        ah = *(L.a_valid ? &S.ahi[buf][g * kGroup + L.a_g] : &S.zero_hi);
        al = *(L.a_valid ? &S.alo[buf][g * kGroup + L.a_g] : &S.zero_hi);
    }
    acc = Op<M>::mfma(ah, bhi, acc);
    acc = Op<M>::mfma(al, blo, acc);
    return acc;
}

// q of one staged Gaussian for this lane's pixel, per pixel in FP32 (Eq. (power)).
template <int NB>
__device__ inline float plain_q(const Stage<Mode::Plain, NB> &S, int buf, int idx, const Lane &L) {
    const float4 geo = S.geo[buf][idx];
    const float2 g2 = S.geo2[buf][idx];
    const float dx = geo.x - L.px, dy = geo.y - L.py;
    float gx, gy;
    return fmaf(quad_acc(geo.z, geo.w, g2.x, dx, dy, gx, gy), -0.5f * kLog2e, g2.y);
}

// ------------------------------------------------------------------------------- forward
struct FwdState {
    float T, r, g, b, thr;   // thr = kQCull while live, +inf once done
    int last;
};

// One front-to-back step (Alg. 1 / Alg. 2 inner loop) for this lane's pixel: a skipped pair or a
// finished pixel leaves the state unchanged. The kernel is bound by vector-instruction issue, so
// the lanes that blend update their state under the execution mask rather than through a select
// per value. (The end of a pixel stays a select: as a scalar branch on a ballot it costs more
// than it saves, since the branch waits for the compare.)
__device__ inline void composite(float q, float lo2o, float cr, float cg, float cb, int pos,
                                 FwdState &st) {
    const bool hit = q >= st.thr;
    const float a = __builtin_amdgcn_exp2f(fminf(fminf(q, lo2o), kQAlphaMax));   // <= 0.99
    const float Tn = fmaf(-a, st.T, st.T);   // T (1 - alpha), rounded once
    const bool stop = Tn < kTStop;
    if (hit && !stop) {
        const float wgt = a * st.T;
        st.r = fmaf(wgt, cr, st.r);
        st.g = fmaf(wgt, cg, st.g);
        st.b = fmaf(wgt, cb, st.b);
        st.T = Tn;
        st.last = pos + 1;
    }
    st.thr = (hit && stop) ? INFINITY : st.thr;
}

// Composites the 16 Gaussians of one group; q(u) gives Gaussian u's exponent for this lane. A
// Gaussian that some lane takes has its (log2 o, r, g, b) read at one LDS address by every lane.
// A Gaussian whose bit in `reach` (this wavefront's reach mask of the group) is clear is skipped
// without evaluating q: no lane would take it.
template <typename QFn>
__device__ inline void composite_group(const float4 *attr, int base, uint32_t reach, FwdState &st,
                                       QFn q_of) {
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
        if (((reach >> u) & 1u) == 0u) continue;
        const float q = q_of(u);
        if (__builtin_amdgcn_ballot_w64(q >= st.thr) == 0ull) continue;   // no lane takes it
        // one address for every lane (an LDS broadcast), read whole: left to itself the compiler
        // moves the colour reads into the blending lanes' branch, as separate loads
        f4x a = *reinterpret_cast<const f4x *>(&attr[u]);
        asm volatile("" : "+v"(a));
        composite(q, a.x, a.y, a.z, a.w, base + u, st);
    }
}

// Forward of one tile of one view (all 256 threads of the block take part; block-uniform control
// flow around every barrier).
template <Mode M, int NB, bool kPacked = false>
__device__ inline void fwd_tile(const ViewDesc &v, int64_t tile, Stage<M, NB> &S) {
    static_assert(NB % kGroup == 0 && NB <= kBlock, "batch must be whole groups, <= block");
    constexpr int kGroups = NB / kGroup;
    const uint32_t *plist = v.point_list;
    const uint32_t n = uint32_t(v.n);
    const Attrs<kPacked> src(v);
    const Lane L = lane_setup(tile, v.gx, v.W, v.H);
    const float xc = float(int(tile % v.gx) * kTile) + 7.5f, yc = float(int(tile / v.gx) * kTile) + 7.5f;
    typename Op<M>::vec bhi, blo;
    pixel_basis<M>(L, bhi, blo);
    if (L.t == 0) {
        float z[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if constexpr (M != Mode::Plain) S.zero_hi = S.zero_lo = Op<M>::cvt(z);
    }
    const uint2 rg = reinterpret_cast<const uint2 *>(v.ranges)[tile];
    // without Gaussians every list entry would be invalid: the tile shows the background
    const int64_t start = rg.x, len = n == 0 ? 0 : int64_t(rg.y) - int64_t(rg.x);
    const int nb = int((len + NB - 1) / NB);

    // list entries are loaded two batches ahead and attributes one batch ahead, so that neither
    // load waits on the other within an iteration
    const auto entry = [&](int bb) {          // batch bb's entry for this thread (bb < nb + 2)
        const int64_t o = int64_t(bb) * NB + L.t;
        return load_entry(plist, start + o, L.t < NB && o < len, start);
    };
    FwdState st{1.f, 0.f, 0.f, 0.f, L.inside ? kQCull : INFINITY, 0};
    GRaw nxt{};
    Entry ent{kNoEntry, false};
    if (nb > 0) {                               // (len > 0, so entry `start` exists)
        nxt = src.fetch(entry(0).id(), n);
        ent = entry(1);
    }
    for (int b = 0; b < nb; ++b) {
        const int buf = b & 1;
        if (L.t < NB) stage<M, NB, false>(nxt, buf, L.t, xc, yc, S, nullptr, v.reach != 0);
        // Barrier. Each wavefront also posts whether it still has a live pixel, and the whole
        // block leaves once none has (one barrier; the flags are double-buffered with the batch,
        // so that batch b + 2's post cannot overtake a wavefront still reading batch b's).
        const bool wave_live = __ballot(st.thr != INFINITY) != 0;   // (the whole wavefront's)
        if (L.l == 0) S.live[buf][L.w] = wave_live ? 1u : 0u;
        __syncthreads();
        {
            const uint4 f = *reinterpret_cast<const uint4 *>(S.live[buf]);
            if (__builtin_amdgcn_readfirstlane(f.x | f.y | f.z | f.w) == 0u) break;
        }
        // unconditional: past the last batch these read entry `start` and Gaussian 0, unused
        nxt = src.fetch(ent.id(), n);
        ent = entry(b + 2);
        const int base = b * NB;
        const int ng = int((len - base + kGroup - 1) / kGroup) < kGroups
                           ? int((len - base + kGroup - 1) / kGroup) : kGroups;
        for (int g = 0; g < ng; ++g) {
            if (__ballot(st.thr != INFINITY) == 0) break;
            const uint32_t reach = group_reach<M, NB>(S, buf, L.w, g);
            if (reach == 0u) continue;                 // no Gaussian of the group reaches this wave
            const float4 *attr = &S.attr[buf][g * kGroup];
            if constexpr (M == Mode::Plain) {
                composite_group(attr, base + g * kGroup, reach, st,
                                [&](int u) { return plain_q(S, buf, g * kGroup + u, L); });
            } else {
                const f16x q = group_q_mfma<M, NB, false>(S, buf, g, L, bhi, blo);
                composite_group(attr, base + g * kGroup, reach, st, [&](int u) { return q[u]; });
            }
        }
    }
    if (L.inside) {
        const int64_t p = int64_t(L.py) * v.W + int64_t(L.px);
        const int64_t HW = int64_t(v.H) * v.W;
        v.image[p] = st.r + st.T * v.bg[0];
        v.image[HW + p] = st.g + st.T * v.bg[1];
        v.image[2 * HW + p] = st.b + st.T * v.bg[2];
        v.final_T[p] = st.T;
        v.last_contrib[p] = st.last;
    }
}

// ------------------------------------------------------------------------------- backward
// u + (v moved within its 16-lane row by the DPP control Ctrl). Every control used here reads
// inside the row, so bound_ctrl (out-of-row reads give 0) never applies; it spares an `old`
// operand.
template <int Ctrl>
__device__ inline float dpp_add2(float u, float v) {
    const int y = __builtin_amdgcn_update_dpp(0, __float_as_int(v), Ctrl, 0xf, 0xf, true);
    return u + __int_as_float(y);
}
constexpr int kDppRowRor8 = 0x128, kDppRowHalfMirror = 0x141;
constexpr int kDppQuadRev = 0x1b, kDppQuadSwap = 0xb1;       // quad_perm [3,2,1,0], [1,0,3,2]

// Sum of 9 values over the whole wavefront, transposed so that the 9 totals land in distinct
// lanes (two values share each swap-and-add, so the wavefront is halved per value pair, not per
// value):
//   permlane32_swap + add on the pairs (s0,s1) (s2,s3) (s4,s5) (s6,s7): lanes 0-31 hold the
//       first value's 32 partial sums, lanes 32-63 the second's; s8, which has no partner, adds
//       lane l ^ 32 through ds_bpermute;
//   permlane16_swap + add on the register pairs: rows (16 lanes) of a hold (s0, s2, s1, s3),
//       rows of b hold (s4, s6, s5, s7); s8 adds lane l ^ 16 through ds_swizzle, so every row of
//       c holds s8;
//   a and b share one register from here: lanes 0-7 of a row take a's row values, lanes 8-15
//       b's, each summed with the lane 8 away (row_ror 8); then half_mirror, and two quad
//       permutations finish each 8-lane half; c takes the same four steps alone.
// Result: lanes 16r .. 16r+7 of ab hold s[{0,2,1,3}[r]], lanes 16r+8 .. 16r+15 hold
// s[4 + {0,2,1,3}[r]]; lanes 0-7 of c hold s8. Every lane must be active.
__device__ inline float swap_add32(float &x, float y) {   // returns [x.lo + x.hi | y.lo + y.hi]
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ inline float swap_add16(float x, float y) {    // rows: [x0+x1, y0+y1, x2+x3, y2+y3]
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ inline void wave_sum9(const float (&s)[kGrad], int lane, float &ab, float &c) {
    float x0 = s[0], x2 = s[2], x4 = s[4], x6 = s[6];
    const float p01 = swap_add32(x0, s[1]), p23 = swap_add32(x2, s[3]);
    const float p45 = swap_add32(x4, s[5]), p67 = swap_add32(x6, s[7]);
    // the ninth value alone: lane l adds lane l ^ 32 (ds_bpermute), then lane l ^ 16 (ds_swizzle,
    // xor mask 16 within each 32-lane half); both go through the LDS crossbar, not the VALU
    const float p88 = s[8] + __int_as_float(__builtin_amdgcn_ds_bpermute((lane ^ 32) << 2,
                                                                        __float_as_int(s[8])));
    const float a = swap_add16(p01, p23);
    const float b = swap_add16(p45, p67);
    c = p88 + __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(p88), 0x401f));
    const bool lo = (lane & 8) == 0;
    ab = dpp_add2<kDppRowRor8>(lo ? a : b, lo ? b : a);
    c = dpp_add2<kDppRowRor8>(c, c);
    ab = dpp_add2<kDppRowHalfMirror>(ab, ab); c = dpp_add2<kDppRowHalfMirror>(c, c);
    ab = dpp_add2<kDppQuadRev>(ab, ab);       c = dpp_add2<kDppQuadRev>(c, c);
    ab = dpp_add2<kDppQuadSwap>(ab, ab);      c = dpp_add2<kDppQuadSwap>(c, c);
    // keep the last add here, where it is one DPP add, not moved into the callers' leader branch
    // (where it would need a separate move)
    asm volatile("" : "+v"(ab), "+v"(c));
}

// The word of a Gaussian's nine sums that a leader lane (l % 8 == 0) adds after wave_sum9:
// lane 16r holds s[{0,2,1,3}[r]], lane 16r + 8 holds s[4 + {0,2,1,3}[r]] (lane 0 also s8).
__device__ inline int sum_word(int l) {
    const int r = l >> 4;
    return 2 * (r & 1) + (r >> 1) + (l & 8 ? 4 : 0);
}

struct BwdState {
    float T;        // transmittance in front of the pairs not yet visited
    // the colour behind them per unit of that transmittance: (T_final (bg . g) + sum over the
    // visited pairs of alpha T (c . g)) / T. With it dL/dalpha of the next pair (in front) is
    // T_in (c . g - beta), T_in the transmittance in front of that pair, and beta moves to
    // beta (1 - alpha) + alpha (c . g): no division by (1 - alpha) beyond the one T needs.
    float beta;
    float gr, gg, gb;
    int last;
};

// Reverse step for one (Gaussian, pixel) pair. Nothing but a compare and a scalar branch is
// spent when no lane of the wave has a live pair. Otherwise every lane evaluates the step, with no
// branch but a rare one for the clamps (a dead lane takes alpha = 0: its terms vanish and its
// state is unchanged exactly, since 1 / (1 - 0) = 1),
// the pair's 9 gradient terms are summed over the wavefront, and the totals are added into the
// Gaussian's LDS accumulator (`acc` points at the word this lane adds when it leads, see
// sum_word), which the block flushes to global memory once per batch. Raw
// sums: S_xx, S_xy, S_yy, S_x, S_y (times dL/dpower), the sum of dL/dpower without the clamp test
// (o dL/do: the final pass divides it by o, once per Gaussian instead of once per pair), and the
// three colour gradients.
// kRanged = false: the caller has checked that the whole group lies before every lane's last
// contributor, so the skip test alone decides (one compare, whose mask is the ballot).
// kDet: `acc` points into the wavefront's own slice of the batch's sums, which this Gaussian's
// totals are stored into (no other wavefront writes there), so no atomic.
template <bool kRanged, bool kDet = false>
__device__ inline void reverse_pair(float q, bool in_range, const float4 *ga, const float2 *gb,
                                    int u, const Lane &L, BwdState &st, float *acc) {
    bool alive;
    unsigned long long live;
    if constexpr (kRanged) {
        // one ballot per compare (each is just that compare's lane mask), combined and tested in
        // scalar registers: a ballot of the combined condition is copied through a vector
        // register, two more vector instructions for every Gaussian of a ranged group. The empty
        // asm statements keep the compiler from merging the two ballots back into one, and the
        // lane's own condition is read back from the combined mask (with the compares reused,
        // each mask is copied beside its ballot: two scalar moves per visit).
        unsigned long long m_range = __builtin_amdgcn_ballot_w64(in_range);
        unsigned long long m_cull = __builtin_amdgcn_ballot_w64(q >= kQCull);
        asm volatile("" : "+s"(m_range));
        asm volatile("" : "+s"(m_cull));
        live = m_range & m_cull;
        alive = __builtin_amdgcn_inverse_ballot_w64(live);
    } else {
        alive = q >= kQCull;
        live = __builtin_amdgcn_ballot_w64(alive);
    }
    if (live == 0ull) return;
    const float4 attr = ga[u];   // one address for every lane: LDS broadcasts
    const float2 bw = gb[u];
    // a dead lane has q < log2(1/255) or is past its last contributor: it blended nothing here
    const float a = alive ? __builtin_amdgcn_exp2f(fminf(fminf(q, attr.x), kQAlphaMax)) : 0.f;
    const float r = __builtin_amdgcn_rcpf(1.0f - a);  // exactly 1 for a dead lane
    const float Tb = st.T * r;                           // T in front of this Gaussian
    const float wc = a * Tb;                             // the pair's weight alpha T
    // c . g - beta as one fma chain from -beta: dL/dalpha = Tb (c . g - beta)
    const float gmb = fmaf(st.gb, attr.w, fmaf(st.gg, attr.z, fmaf(st.gr, attr.y, -st.beta)));
    st.beta = fmaf(a, gmb, st.beta);
    st.T = Tb;
    const float da = wc * gmb;                           // dL/dpower = alpha dL/dalpha
    const float dx = bw.x - L.px, dy = bw.y - L.py;
    const float tx = da * dx, ty = da * dy;
    float s[kGrad] = {tx * dx, tx * dy, ty * dy, tx, ty, da,   // dL/do = alpha/o dL/dalpha
                      wc * st.gr, wc * st.gg, wc * st.gb};
    // The clamps are rare, so one scalar test stands for them and the terms of the live lanes they
    // touch are zeroed in place: with the 0.99 clamp active dL/dpower is 0, and no gradient
    // reaches the geometry through a clamped (positive) power. (One ballot per compare, kept
    // apart by the empty asm statements, as above.)
    // (The 0.99 clamp is active where min(q, log2 o) >= kQAlphaMaxLo, so only where q is too.)
    unsigned long long m_a = __builtin_amdgcn_ballot_w64(q >= kQAlphaMaxLo);
    unsigned long long m_q = __builtin_amdgcn_ballot_w64(q > attr.x);
    asm volatile("" : "+s"(m_a));
    asm volatile("" : "+s"(m_q));
    if (((m_a | m_q) & live) != 0ull) {
        // (min(q, log2 o) >= kQAlphaMaxLo, as two compares: the step above keeps its three-way min)
        // The lane predicates are read back from the two masks: recomparing q would make the
        // compiler keep each compare's result beside its ballot, a scalar copy per live pair.
        const bool clamp_a = __builtin_amdgcn_inverse_ballot_w64(m_a);
        const bool clamp_q = __builtin_amdgcn_inverse_ballot_w64(m_q);
        const bool keep_a = !(clamp_a && attr.x >= kQAlphaMaxLo);
        const bool keep_g = keep_a && !clamp_q;
#pragma unroll
        for (int k = 0; k < 5; ++k) s[k] = keep_g ? s[k] : 0.f;
        s[5] = keep_a ? s[5] : 0.f;
    }
    float rab, rc;
    wave_sum9(s, L.l, rab, rc);
    if constexpr (kDet) {
        if ((L.l & 7) == 0) {
            // acc is this lane's word of the Gaussian's sums (see sum_word); lane 0's is word 0
            *acc = rab;
            if (L.l == 0) acc[8] = rc;
        }
    } else {
        // one LDS atomic for all nine sums: lane 1 adds s8 (its acc points at word 8)
        const float val = L.l == 1 ? rc : rab;
        if ((L.l & 7) == 0 || L.l == 1) atomicAdd(acc, val);
    }
}

// Sum of 4 values over the wavefront (wave_sum9's first stages on two value pairs): lanes 16r ..
// 16r + 15 of the result hold s[{0,2,1,3}[r]]. Every lane must be active.
__device__ inline float wave_sum4(const float (&s)[4]) {
    float x0 = s[0], x2 = s[2];
    const float p01 = swap_add32(x0, s[1]), p23 = swap_add32(x2, s[3]);
    float a = swap_add16(p01, p23);
    a = dpp_add2<kDppRowRor8>(a, a);
    a = dpp_add2<kDppRowHalfMirror>(a, a);
    a = dpp_add2<kDppQuadRev>(a, a);
    a = dpp_add2<kDppQuadSwap>(a, a);
    return a;
}

// Reverse step of reverse_pair for the matrix-core reduction: the same state update, but of the
// pair's gradient terms only the four plain sums (dL/do and the colours) are reduced on the vector
// ALUs here; dL/dpower (with no gradient through a clamped power) goes into the wavefront's
// transposition row `dgrow`, from which the five geometric sums are formed as a product with the
// pixel basis (mm_reduce). Returns whether any lane of the wavefront had a live pair.
template <bool kRanged>
__device__ inline bool reverse_pair_mm(float q, bool in_range, const float4 *ga, const float2 *gb,
                                       int u, const Lane &L, BwdState &st, float *acc,
                                       uint32_t *dgrow) {
    bool alive;
    unsigned long long live;
    if constexpr (kRanged) {
        unsigned long long m_range = __builtin_amdgcn_ballot_w64(in_range);
        unsigned long long m_cull = __builtin_amdgcn_ballot_w64(q >= kQCull);
        asm volatile("" : "+s"(m_range));
        asm volatile("" : "+s"(m_cull));
        live = m_range & m_cull;
        alive = __builtin_amdgcn_inverse_ballot_w64(live);
    } else {
        alive = q >= kQCull;
        live = __builtin_amdgcn_ballot_w64(alive);
    }
    if (live == 0ull) return false;
    const float4 attr = ga[u];
    const float2 bw = gb[u];
    const float araw = __builtin_amdgcn_exp2f(fminf(q, attr.x));
    const float a = alive ? fminf(araw, kAlphaMax) : 0.f;
    const float r = __builtin_amdgcn_rcpf(1.0f - a);
    const float Tb = st.T * r;
    const float wc = a * Tb;
    const float gmb = fmaf(st.gb, attr.w, fmaf(st.gg, attr.z, fmaf(st.gr, attr.y, -st.beta)));
    st.beta = fmaf(a, gmb, st.beta);
    st.T = Tb;
    const float da = araw < kAlphaMax ? wc * gmb : 0.f;
    const float dg = q > attr.x ? 0.f : da;
    // dg = hi + lo 2^-12 with FP16 hi and lo (truncations; the residual dg - hi is exact in FP32)
    const auto hp = __builtin_amdgcn_cvt_pkrtz(dg, 0.f);
    const float lo = (dg - float(hp[0])) * kLoScale;
    const auto pk = __builtin_amdgcn_cvt_pkrtz(dg, lo);
    dgrow[L.l] = __builtin_bit_cast(uint32_t, pk);
    const float s[4] = {da, wc * st.gr, wc * st.gg, wc * st.gb};
    const float tot = wave_sum4(s);
    if ((L.l & 15) == 0)
        atomicAdd(acc + 5 + ((L.l >> 4) == 1 ? 2 : (L.l >> 4) == 2 ? 1 : (L.l >> 4)), tot);
    return true;
}

// The pixel basis of the matrix-core reduction as the B operand of v_mfma_f32_16x16x32_f16, for
// the two 32-pixel halves c of the wavefront's quadrant: lane l supplies basis function l % 16
// (1, xb, yb, xb^2, xb yb, yb^2, then zeros) at the 8 pixels 32c + 8(l / 16) + j, j = 0..7, which
// lie in one row of the quadrant. xb = x_c - px and yb = y_c - py are quarter-integers of at most
// 7.5 in magnitude, so every value is exact in FP16.
__device__ inline void mm_basis(const Lane &L, h8 (&B)[2]) {
    const int n = L.l & 15;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const float yb = 7.5f - float(8 * (L.w >> 1) + 4 * c + (L.l >> 4));
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float xb = 7.5f - float(8 * (L.w & 1) + j);
            v[j] = n == 0 ? 1.f : n == 1 ? xb : n == 2 ? yb : n == 3 ? xb * xb
                 : n == 4 ? xb * yb : n == 5 ? yb * yb : 0.f;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) B[c][j] = _Float16(v[j]);
    }
}

// The five geometric sums of the 8 Gaussians of one half-group (staged slots base .. base + 7)
// from the wavefront's transposition rows: two v_mfma_f32_16x16x32_f16 give, per Gaussian, the
// moments sum_p dg [1, xb, yb, xb^2, xb yb, yb^2] over the 64 pixels (rows 0-7 from the hi terms,
// rows 8-15 from the lo terms, combined in FP32); with dx = xh + xb (xh = x - x_c) the sums
// of dg [dx^2, dx dy, dy^2, dx, dy] follow per Gaussian, and are added into the batch's
// accumulator. `hmask` has bit i set when Gaussian base + i had a live pair in this wavefront;
// the rows are left zero.
__device__ inline void mm_reduce(uint32_t (*rows)[kDgStride], const h8 (&B)[2], unsigned hmask,
                                 const float2 *gb, float xc, float yc, float *acc, const Lane &L) {
    __builtin_amdgcn_wave_barrier();
    const int row = L.l & 15, q = L.l >> 4;
    // hi rows take the low halves of the packed words, lo rows the high halves
    const uint32_t sel = row < 8 ? 0x05040100u : 0x07060302u;
    f4x d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const uint4 *src = reinterpret_cast<const uint4 *>(&rows[row & 7][32 * c + 8 * q]);
        const uint4 w0 = src[0], w1 = src[1];
        uint32_t av[4];
        av[0] = __builtin_amdgcn_perm(w0.y, w0.x, sel);
        av[1] = __builtin_amdgcn_perm(w0.w, w0.z, sel);
        av[2] = __builtin_amdgcn_perm(w1.y, w1.x, sel);
        av[3] = __builtin_amdgcn_perm(w1.w, w1.z, sel);
        h8 A;
        __builtin_memcpy(&A, av, sizeof(A));
        d = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, B[c], d, 0, 0, 0);
    }
    // lane l < 32 holds rows 4q + v (hi) of column l % 16; lane l + 32 the lo rows of the same
    // Gaussians: moment = hi + 2^-12 lo
    float m[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(d[v]), __float_as_uint(d[v]),
                                                        false, false);
        m[v] = fmaf(__uint_as_float(r[1]), kLoScaleInv, __uint_as_float(r[0]));
    }
    // moments table mom[g][n] in row 0 (the operand reads above have completed: the MFMA used them)
    float *mom = reinterpret_cast<float *>(rows[0]);
    if (L.l < 32 && row < 6) {
#pragma unroll
        for (int v = 0; v < 4; ++v) mom[(4 * q + v) * 8 + row] = m[v];
    }
    __builtin_amdgcn_wave_barrier();
    // lane g * 5 + k forms sum k of Gaussian g
    if (L.l < 40) {
        const int g = L.l / 5, k = L.l - 5 * g;
        if ((hmask >> g) & 1u) {
            const float4 m0 = *reinterpret_cast<const float4 *>(mom + 8 * g);
            const float2 m1 = *reinterpret_cast<const float2 *>(mom + 8 * g + 4);
            const float S1 = m0.x, Sx = m0.y, Sy = m0.z, Sxx = m0.w, Sxy = m1.x, Syy = m1.y;
            const float2 bw = gb[g];
            const float xh = bw.x - xc, yh = bw.y - yc;
            const float sx = fmaf(xh, S1, Sx), sy = fmaf(yh, S1, Sy);
            float val;
            if (k == 0) val = fmaf(xh, sx, fmaf(xh, Sx, Sxx));            // sum dg dx^2
            else if (k == 1) val = fmaf(xh, sy, fmaf(yh, Sx, Sxy));       // sum dg dx dy
            else if (k == 2) val = fmaf(yh, sy, fmaf(yh, Sy, Syy));       // sum dg dy^2
            else if (k == 3) val = sx;
            else val = sy;
            atomicAdd(acc + g * kGrad + k, val);
        }
    }
    __builtin_amdgcn_wave_barrier();
    // leave the rows zero for the next half-group
    uint4 *z = reinterpret_cast<uint4 *>(&rows[L.l >> 3][(L.l & 7) * 8]);
    z[0] = make_uint4(0u, 0u, 0u, 0u);
    z[1] = make_uint4(0u, 0u, 0u, 0u);
}

// Backward of one tile of one view.
// kMM: the five geometric sums are formed on the matrix cores (mm_reduce) instead of being
// reduced on the vector ALUs with the other four; `mm` is then the block's transposition tiles.
// kDet: the batch sums go to the wavefronts' own slices (`det`) instead of `acc_`, and the flush
// writes each list position's nine sums to v.det_partial in place of the global atomics (every
// position of the tile's list is written, those past the last contributor with zeros).
template <Mode M, int NB, bool kMM, bool kPacked = false, bool kDet = false>
__device__ inline void bwd_tile(const ViewDesc &v, int64_t tile, Stage<M, NB> &S, StageBwd<NB> &SB,
                                BwdAcc<NB> *acc_, int &s_maxlast, BwdMM *mm,
                                BwdAccDet<NB> *det = nullptr) {
    static_assert(NB % kGroup == 0 && NB <= kBlock, "batch must be whole groups, <= block");
    static_assert(!(kMM && kDet), "the deterministic backward reduces on the vector ALUs");
    constexpr int kGroups = NB / kGroup;
    const uint32_t *plist = v.point_list;
    const uint32_t n = uint32_t(v.n);
    const Attrs<kPacked> src(v);
    const Lane L = lane_setup(tile, v.gx, v.W, v.H);
    const int word = sum_word(L.l);   // the sum this lane adds when it leads a reduction
    const float xc = float(int(tile % v.gx) * kTile) + 7.5f, yc = float(int(tile / v.gx) * kTile) + 7.5f;
    typename Op<M>::vec bhi, blo;
    pixel_basis<M>(L, bhi, blo);
    if (L.t == 0) {
        float z[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if constexpr (M != Mode::Plain) S.zero_hi = S.zero_lo = Op<M>::cvt(z);
        s_maxlast = 0;
    }
    h8 mmB[2];
    uint32_t (*rows)[kDgStride] = nullptr;
    if constexpr (kMM) {
        mm_basis(L, mmB);
        rows = mm->dg[L.w];
        uint4 *z = reinterpret_cast<uint4 *>(&rows[L.l >> 3][(L.l & 7) * 8]);
        z[0] = make_uint4(0u, 0u, 0u, 0u);
        z[1] = make_uint4(0u, 0u, 0u, 0u);
    }
    if (n == 0) return;            // no Gaussian, no gradient (uniform: every thread returns)
    BwdState st{1.f, 0.f, 0.f, 0.f, 0.f, 0};
    if (L.inside) {
        const int64_t p = int64_t(L.py) * v.W + int64_t(L.px);
        const int64_t HW = int64_t(v.H) * v.W;
        st.T = v.final_T[p];
        st.last = v.last_contrib[p];
        st.gr = v.dL_dimage[p]; st.gg = v.dL_dimage[HW + p]; st.gb = v.dL_dimage[2 * HW + p];
        st.beta = v.bg[0] * st.gr + v.bg[1] * st.gg + v.bg[2] * st.gb;   // (T_final (bg . g)) / T_final
    }
    __syncthreads();
    if (st.last > 0) atomicMax(&s_maxlast, st.last);
    __syncthreads();
    const uint2 rg = reinterpret_cast<const uint2 *>(v.ranges)[tile];
    const int64_t start = rg.x;
    // positions [0, max last) are the only ones that matter (never more than the list holds)
    // (the same value in every lane: made wavefront-uniform, so that the batch and group loops
    // and their index arithmetic run on the scalar unit)
    const int maxlast = __builtin_amdgcn_readfirstlane(s_maxlast);
    const int64_t len = maxlast < int64_t(rg.y) - int64_t(rg.x) ? maxlast
                                                                : int64_t(rg.y) - int64_t(rg.x);
    const int nb = int((len + NB - 1) / NB);
    if constexpr (kDet) {
        // list positions [len, end) are never visited: their sums are zero (positions at or
        // past det_pairs, which an inconsistent range could name, are never written)
        const int64_t end = int64_t(rg.y) < v.det_pairs ? int64_t(rg.y) : v.det_pairs;
        const int64_t tail = (end - start - len) * kDetStride;
        float *dst = v.det_partial + (start + len) * kDetStride;
        for (int64_t j = L.t; j < tail; j += kBlock) dst[j] = 0.f;
    }
    if (nb == 0) return;

    // Memory operations of a batch are issued before its compute: the attribute loads of the next
    // batch, the list entries of the one after, and the global atomics that flush the previous
    // batch's sums (from the other accumulator buffer). Every wait at the top of an iteration is
    // then for operations issued a whole compute phase earlier; with the flush after the compute,
    // the next wait (the memory counter also counts atomics) would expose their latency.
    const auto entry = [&](int bb) {          // batch bb's entry for this thread (bb may be < 0)
        const int64_t o = int64_t(bb) * NB + L.t;
        return load_entry(plist, start + o, bb >= 0 && L.t < NB && o < len, start);
    };
    // Wavefront w flushes slots [w NB/4, (w + 1) NB/4). It lists the slots that
    // received a nonzero sum, in slot order, and then spreads their nine sums over its lanes,
    // item j the sum j % 9 of listed slot j / 9, so that consecutive lanes add consecutive words
    // of one Gaussian (a wavefront's atomic instruction reaches about 30 cache lines instead of
    // 64) and no lane is spent on the slots without a sum (over half of a 3-sigma list's). Each
    // item is zeroed by the lane that reads it (an unlisted slot's sums are all +-0 already),
    // ready for batch bb - 2, which reuses the buffers after the next barrier.
    // Deterministic form: word k < 9 of slot i's row is the four wavefronts' sum k added in
    // wavefront order (and zeroed in the slices), words 9..15 are zero; the row is stored at list
    // position start + bb NB + i (consecutive threads, consecutive words).
    const auto flush_det = [&](int bb) {
        const int64_t base = int64_t(bb) * NB;
        float *dst = v.det_partial + (start + base) * kDetStride;
        int64_t last = len - base < NB ? len - base : NB;          // slots of this batch
        if (start + base + last > v.det_pairs) last = v.det_pairs - start - base;
        const int64_t items = last * kDetStride;
        for (int j = L.t; j < NB * kDetStride; j += kBlock) {
            const int i = j / kDetStride, k = j % kDetStride;
            float sum = 0.f;
            if (k < kGrad) {
#pragma unroll
                for (int w = 0; w < kBlock / 64; ++w) {
                    float *p = det->v[bb & 1][w] + i * kGrad + k;
                    sum += *p;
                    *p = 0.f;
                }
            }
            if (j < items) dst[j] = sum;
        }
    };
    const auto flush = [&](int bb) {     // batch bb's sums, accumulator buffer bb & 1
        if constexpr (kDet) {
            flush_det(bb);
            return;
        }
        BwdAcc<NB> &s_acc = *acc_;
        constexpr int kPer = NB / (kBlock / 64);   // slots per wavefront, at most 64
        float *acc = s_acc.v[bb & 1];
        const uint32_t *ids = SB.ids[bb % 3];
        uint16_t *list = s_acc.list[L.w];
        const int s0 = L.w * kPer;
        // a slot is listed if any of its nine sums is nonzero (NaN included); one whose sums
        // are all +-0 adds nothing to the gradients, whether or not a pair reached it
        bool touched = false;
        if (L.l < kPer) {
            const float *p = acc + (s0 + L.l) * kGrad;
            uint32_t bits = 0u;
#pragma unroll
            for (int k = 0; k < kGrad; ++k) bits |= __float_as_uint(p[k]) & 0x7fffffffu;
            touched = bits != 0u;
        }
        const unsigned long long m = __ballot(touched);
        if (touched) list[__popcll(m & ((1ull << L.l) - 1ull))] = uint16_t(s0 + L.l);
        __builtin_amdgcn_wave_barrier();   // the list is written and read by this wavefront only
        const int items = kGrad * __popcll(m);
#pragma unroll 1
        for (int j = L.l; j < items; j += 64) {
            const int i = j / kGrad, k = j - kGrad * i;
            const int slot = list[i];
            float *p = acc + slot * kGrad + k;
            const float val = *p;
            *p = 0.f;
            if (val != 0.f) {
                const int64_t id = ids[slot];
                float *dst = k < 3 ? v.dL_dconics + 3 * id + k
                           : k < 5 ? v.dL_dmeans2d + 2 * id + (k - 3)
                           : k == 5 ? v.dL_dopacity + id
                                    : v.dL_dcolors + 3 * id + (k - 6);
                unsafeAtomicAdd(dst, val);
            }
        }
    };
    GRaw nxt = src.fetch(entry(nb - 1).id(), n);
    Entry ent = entry(nb - 2);
    // both accumulator buffers and their flags start at zero
    if constexpr (kDet) {
        for (int e = L.t; e < NB * kGrad; e += kBlock) {
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) {
                det->v[0][w][e] = 0.f;
                det->v[1][w][e] = 0.f;
            }
        }
    } else {
        for (int e = L.t; e < NB * kGrad; e += kBlock) {
            acc_->v[0][e] = 0.f;
            acc_->v[1][e] = 0.f;
        }
    }
    for (int b = nb - 1; b >= 0; --b) {
        const int buf = b & 1;
        if (L.t < NB) {
            stage<M, NB, true>(nxt, buf, L.t, xc, yc, S, &SB, v.reach != 0);
            SB.ids[b % 3][L.t] = nxt.id;
        }
        __syncthreads();
        // unconditional: before the first batch these read entry `start` and Gaussian 0, unused
        nxt = src.fetch(ent.id(), n);
        ent = entry(b - 2);
        if (b + 1 < nb) flush(b + 1);
        const int base = b * NB;
        const int ng = int((len - base + kGroup - 1) / kGroup) < kGroups
                           ? int((len - base + kGroup - 1) / kGroup) : kGroups;
        for (int g = ng - 1; g >= 0; --g) {
            // nothing to do for this wave unless one of its pixels blended past the group start
            // and a Gaussian of the group can reach it (see reach_mask)
            if (__ballot(st.last > base + g * kGroup) == 0) continue;
            const uint32_t reach = group_reach<M, NB>(S, buf, L.w, g);
            if (reach == 0u) continue;
            // the group's first slot, held in a vector register: each Gaussian's LDS addresses are
            // then immediate offsets from it (from a scalar base the compiler copies the base
            // into a vector register again for every Gaussian)
            int slot0 = g * kGroup;
            asm volatile("" : "+v"(slot0));
            const float4 *ga = &S.attr[buf][slot0];   // the group's staged values
            const float2 *gb = &SB.bwd[buf][slot0];
            // the group's sums, Gaussian 0 (deterministic: this wavefront's slice)
            float *accw = kDet ? det->v[buf][L.w] + g * kGroup * kGrad
                               : acc_->slot(buf, g * kGroup);
            // this lane's word (VALU reduction; with atomics lane 1 adds word 8)
            float *acc = accw + (kMM ? 0 : !kDet && L.l == 1 ? 8 : word);
            const int rel = st.last - (base + g * kGroup);   // positions < last are in range
            // the whole group is in range for every lane (the common case once past the lanes'
            // last contributors; never for a partial tile, whose outside lanes have last = 0)
            const bool whole = __builtin_amdgcn_ballot_w64(rel < kGroup) == 0ull;
            f16x qm;
            if constexpr (M != Mode::Plain) qm = group_q_mfma<M, NB, true>(S, buf, g, L, bhi, blo);
            const auto q_of = [&](int u) {
                if constexpr (M == Mode::Plain) return plain_q(S, buf, slot0 + u, L);
                else return qm[u];
            };
            if constexpr (kMM) {
                // two half-groups of 8: Gaussians 15..8, then 7..0, each followed by its product
#pragma unroll
                for (int h = 1; h >= 0; --h) {
                    unsigned hmask = 0u;
                    if (whole) {
#pragma unroll
                        for (int i = 7; i >= 0; --i) {
                            const int u = 8 * h + i;
                            if (((reach >> u) & 1u) == 0u) continue;
                            if (reverse_pair_mm<false>(q_of(u), true, ga, gb, u, L, st,
                                                       acc + u * kGrad, rows[i]))
                                hmask |= 1u << i;
                        }
                    } else {
#pragma unroll
                        for (int i = 7; i >= 0; --i) {
                            const int u = 8 * h + i;
                            if (((reach >> u) & 1u) == 0u) continue;
                            if (reverse_pair_mm<true>(q_of(u), u < rel, ga, gb, u, L, st,
                                                      acc + u * kGrad, rows[i]))
                                hmask |= 1u << i;
                        }
                    }
                    if (hmask != 0u)
                        mm_reduce(rows, mmB, hmask, gb + 8 * h, xc, yc, accw + 8 * h * kGrad, L);
                }
            } else if (whole) {
#pragma unroll
                for (int u = kGroup - 1; u >= 0; --u) {
                    if (((reach >> u) & 1u) == 0u) continue;
                    reverse_pair<false, kDet>(q_of(u), true, ga, gb, u, L, st, acc + u * kGrad);
                }
            } else {
#pragma unroll
                for (int u = kGroup - 1; u >= 0; --u) {
                    if (((reach >> u) & 1u) == 0u) continue;
                    reverse_pair<true, kDet>(q_of(u), u < rel, ga, gb, u, L, st, acc + u * kGrad);
                }
            }
        }
        // Buffers: the next iteration stages into the other stage buffer. The accumulator buffer
        // of batch b + 1 and its flags, flushed above, were zeroed by the flush itself, item by
        // item; the barrier orders that before batch b - 1 adds into them.
    }
    __syncthreads();
    flush(0);
}

// ------------------------------------------------------------------------------- kernels
// Wavefronts per SIMD that a kernel's launch bound asks for: its register target, but never more
// than the blocks that fit in a compute unit's 160 KB of LDS (a 256-thread block puts one
// wavefront on each SIMD), so the compiler is not held to an occupancy the LDS rules out.
constexpr size_t kLdsPerCu = 160 * 1024;
constexpr int fit_waves(int target, size_t lds) {
    return int(kLdsPerCu / lds) < target ? int(kLdsPerCu / lds) : target;
}
// LDS of one block: the staged batches (and, backward, the gradient accumulators), plus the few
// scalars the kernels share
template <Mode M, int NB> constexpr size_t lds_fwd() { return sizeof(Stage<M, NB>) + 64; }
template <Mode M, int NB, bool kMM> constexpr size_t lds_bwd() {
    return sizeof(Stage<M, NB>) + sizeof(StageBwd<NB>) + sizeof(BwdAcc<NB>) +
           (kMM ? sizeof(BwdMM) : 0) + 64;
}
// The transposition tiles exist only in the matrix-core reduction's kernels.
struct NoMM {};
template <bool kMM> using MMTiles = typename std::conditional<kMM, BwdMM, NoMM>::type;
template <bool kMM> __device__ inline BwdMM *mm_ptr(MMTiles<kMM> &t) {
    if constexpr (kMM) return &t;
    else return nullptr;
}
// Register targets of the one-tile-per-block backward kernels; the matrix-core reduction keeps
// the product's operands and results live across each half-group and needs more registers
// (fewer targets spill). (6 wavefronts per SIMD for the GEMM forms fit in LDS, 26.9 KB per block,
// but at 80 registers a few values spill and the backward is about 1% slower than at 5.)
template <Mode M, bool kMM> constexpr int waves_bwd_tile() {
    return kMM ? (M == Mode::Plain ? 5 : 4) : (M == Mode::Plain ? 7 : 5);
}
// Single view: block b renders tile xcd_tile(b).
template <Mode M, int NB>
__global__ __launch_bounds__(kBlock, fit_waves(M == Mode::Plain ? 8 : 7, lds_fwd<M, NB>()))
void k_blend_fwd(ViewDesc v) {
    __shared__ Stage<M, NB> S;
    const int64_t tile = xcd_tile(blockIdx.x, v.n_tiles, v.gx);
    if (tile >= v.n_tiles) return;
    fwd_tile<M, NB>(v, tile, S);
}

template <Mode M, int NB, bool kMM>
__global__ __launch_bounds__(kBlock, fit_waves(waves_bwd_tile<M, kMM>(), lds_bwd<M, NB, kMM>()))
void k_blend_bwd(ViewDesc v) {
    __shared__ Stage<M, NB> S;
    __shared__ StageBwd<NB> SB;
    __shared__ BwdAcc<NB> s_acc;   // per-Gaussian gradient sums of the current batch
    __shared__ MMTiles<kMM> s_mm;
    __shared__ int s_maxlast;
    const int64_t tile = xcd_tile(blockIdx.x, v.n_tiles, v.gx);
    if (tile >= v.n_tiles) return;
    bwd_tile<M, NB, kMM>(v, tile, S, SB, &s_acc, s_maxlast, mm_ptr<kMM>(s_mm));
}

// Single view, packed records (gsb_pack_gaussians): the default launch shape (LDS batches of 128,
// vector-ALU reduction), attributes from one 48-byte record per list entry.
template <Mode M>
__global__ __launch_bounds__(kBlock, fit_waves(M == Mode::Plain ? 8 : 7, lds_fwd<M, 128>()))
void k_blend_fwd_rec(ViewDesc v) {
    __shared__ Stage<M, 128> S;
    const int64_t tile = xcd_tile(blockIdx.x, v.n_tiles, v.gx);
    if (tile >= v.n_tiles) return;
    fwd_tile<M, 128, true>(v, tile, S);
}

template <Mode M>
__global__ __launch_bounds__(kBlock, fit_waves(waves_bwd_tile<M, false>(), lds_bwd<M, 128, false>()))
void k_blend_bwd_rec(ViewDesc v) {
    __shared__ Stage<M, 128> S;
    __shared__ StageBwd<128> SB;
    __shared__ BwdAcc<128> s_acc;
    __shared__ int s_maxlast;
    const int64_t tile = xcd_tile(blockIdx.x, v.n_tiles, v.gx);
    if (tile >= v.n_tiles) return;
    bwd_tile<M, 128, false, true>(v, tile, S, SB, &s_acc, s_maxlast, nullptr);
}

// Deterministic backward, one tile per block: LDS batches of 64 (the four wavefront slices of the
// batch sums take four times the LDS of the shared accumulator), records as attributes.
constexpr int kDetBatch = 64;
template <Mode M> constexpr size_t lds_bwd_det() {
    return sizeof(Stage<M, kDetBatch>) + sizeof(StageBwd<kDetBatch>) +
           sizeof(BwdAccDet<kDetBatch>) + 64;
}
template <Mode M>
__global__ __launch_bounds__(kBlock, fit_waves(waves_bwd_tile<M, false>(), lds_bwd_det<M>()))
void k_blend_bwd_det(ViewDesc v) {
    __shared__ Stage<M, kDetBatch> S;
    __shared__ StageBwd<kDetBatch> SB;
    __shared__ BwdAccDet<kDetBatch> s_det;
    __shared__ int s_maxlast;
    const int64_t tile = xcd_tile(blockIdx.x, v.n_tiles, v.gx);
    if (tile >= v.n_tiles) return;
    bwd_tile<M, kDetBatch, false, true, true>(v, tile, S, SB, nullptr, s_maxlast, nullptr, &s_det);
}

// Grouping of the list positions by Gaussian: keys = the list's Gaussian indices, values = the
// positions; the count for the sort and empty per-Gaussian ranges.
__global__ __launch_bounds__(256) void k_det_init(const uint32_t *plist, int64_t pairs,
                                                  uint32_t *keys, uint32_t *vals,
                                                  unsigned long long *count, uint32_t *seg,
                                                  int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < pairs) {
        // an index outside [0, n) (inconsistent input) is grouped with the last Gaussian: the
        // backward stages such an entry inert, so its sums are zero
        const uint32_t g = plist[i];
        keys[i] = g < uint64_t(n) ? g : uint32_t(n - 1);
        vals[i] = uint32_t(i);
    }
    if (i < 2 * n) seg[i] = 0u;
    if (i == 0) *count = (unsigned long long)pairs;
}

// Per Gaussian g: the nine sums of its list positions in a fixed order, then turned into the
// gradients as k_bwd_finish does. One wavefront per Gaussian (kGatherPer Gaussians in turn): lane
// l adds the rows of the Gaussian's positions l, l + 64, ... of its run (in list order, the order
// the stable sort left them in), and the 64 lane sums are combined by wave_sum9's fixed reduction
// tree. A thread per Gaussian would leave most lanes of a wavefront idle behind its largest
// footprint (list runs are heavy-tailed: a few Gaussians cover hundreds of tiles).
constexpr int kGatherPer = 4;
__global__ __launch_bounds__(256) void k_det_gather(const float4 *rec, const float *partial,
                                                    const uint32_t *pos, const uint32_t *seg,
                                                    int64_t n, float *dmeans, float *dconics,
                                                    float *dopac, float *dcolors) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    for (int r = 0; r < kGatherPer; ++r) {
        const int64_t g = wave * kGatherPer + r;
        if (g >= n) return;                       // the same in every lane
        const uint32_t a = seg[2 * g], b = seg[2 * g + 1];
        float sum[kGrad];
#pragma unroll
        for (int k = 0; k < kGrad; ++k) sum[k] = 0.f;
        for (uint32_t j = a + uint32_t(lane); j < b; j += 64) {
            const float *p = partial + int64_t(pos[j]) * kDetStride;
            const float4 p0 = *reinterpret_cast<const float4 *>(p);
            const float4 p1 = *reinterpret_cast<const float4 *>(p + 4);
            sum[0] += p0.x; sum[1] += p0.y; sum[2] += p0.z; sum[3] += p0.w;
            sum[4] += p1.x; sum[5] += p1.y; sum[6] += p1.z; sum[7] += p1.w;
            sum[8] += p[8];
        }
        float ab, c;
        wave_sum9(sum, lane, ab, c);
        // lane 16r holds sum {0,2,1,3}[r], lane 16r + 8 sum 4 + {0,2,1,3}[r]; lane 0 of c sum 8
        const auto at = [](float x, int l) {
            return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
        };
        float t[kGrad];
        t[0] = at(ab, 0);  t[2] = at(ab, 16); t[1] = at(ab, 32); t[3] = at(ab, 48);
        t[4] = at(ab, 8);  t[6] = at(ab, 24); t[5] = at(ab, 40); t[7] = at(ab, 56);
        t[8] = at(c, 0);
        if (lane == 0) {
            const float4 r0 = rec[3 * g], r1 = rec[3 * g + 1];
            const float A = r0.z, B = r0.w, C = r1.x;
            dconics[3 * g] = -0.5f * t[0];
            dconics[3 * g + 1] = -t[1];
            dconics[3 * g + 2] = -0.5f * t[2];
            dmeans[2 * g] = -(A * t[3] + B * t[4]);
            dmeans[2 * g + 1] = -(B * t[3] + C * t[4]);
            dopac[g] = opacity_grad(t[5], r1.y);
            dcolors[3 * g] = t[6];
            dcolors[3 * g + 1] = t[7];
            dcolors[3 * g + 2] = t[8];
        }
    }
}

// One record per Gaussian: (x, y, A, B), (C, o, r, g), (b, 0, 0, 0). A block assembles its 256
// records in LDS and writes them out as consecutive 16-byte words, so that every store
// instruction covers one contiguous kilobyte (thread t writing its own record's three words at a
// 48-byte stride wrote 18% more bytes than the records hold).
__global__ __launch_bounds__(256) void k_pack(const float2 *means, const F3 *conics,
                                              const float *opac, const F3 *colors, int64_t n,
                                              float4 *rec) {
    __shared__ float4 s_rec[3 * 256];
    const int t = threadIdx.x;
    const int64_t i0 = int64_t(blockIdx.x) * 256;
    const int64_t i = i0 + t;
    if (i < n) {
        const float2 m = means[i];
        const F3 c = conics[i], col = colors[i];
        s_rec[3 * t] = make_float4(m.x, m.y, c.a, c.b);
        s_rec[3 * t + 1] = make_float4(c.c, opac[i], col.a, col.b);
        s_rec[3 * t + 2] = make_float4(col.c, 0.f, 0.f, 0.f);
    }
    __syncthreads();
    const int words = 3 * int(n - i0 < 256 ? n - i0 : 256);   // the block has at least one record
    for (int k = t; k < words; k += 256) rec[3 * i0 + k] = s_rec[k];
}

// Many views, one persistent launch. The (view, tile) items are split into 8 queues, one per XCD:
// queue x holds the ranks [n_tiles * x / 8, n_tiles * (x + 1) / 8) of every view (tiles in the
// strip order of strip_tile), views in plan
// order (heaviest per-tile cost first). A block serves the queue of its own XCD (block b runs on
// XCD b % 8) so that neighbouring tiles share that XCD's L2, and moves on to the next queue when
// its own is empty, so every block exits once all queues are drained.
// prefix[x * (n_views + 1) + k] = items of queue x that belong to views before k.
struct Queues {
    const ViewDesc *views;
    const int64_t *prefix;
    unsigned int *counters;    // 8 per direction
    int n_views;
};

__device__ inline int64_t band_lo(int64_t n_tiles, int x) { return n_tiles * x / kXcds; }

__device__ inline int64_t uniform_i64(int64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(x)));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(x) >> 32));
    return int64_t((uint64_t(hi) << 32) | lo);
}

// Next item for the calling block (thread 0 only): returns false when every queue is drained.
__device__ inline bool next_item(const Queues &Q, int &q, int &tried, int &view, int64_t &tile) {
    while (tried < kXcds) {
        const int64_t *pre = Q.prefix + int64_t(q) * (Q.n_views + 1);
        const int64_t total = pre[Q.n_views];
        const int64_t i = total > 0 ? int64_t(atomicAdd(&Q.counters[q], 1u)) : total;
        if (i < total) {
            int lo = 0, hi = Q.n_views - 1;       // last k with pre[k] <= i
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (pre[mid] <= i) lo = mid; else hi = mid - 1;
            }
            view = lo;
            const ViewDesc &vw = Q.views[lo];
            tile = strip_tile(band_lo(vw.n_tiles, q) + (i - pre[lo]), vw.n_tiles, vw.gx);
            return true;
        }
        q = (q + 1) % kXcds;
        ++tried;
    }
    return false;
}

// Register budgets for the persistent kernels (waves per SIMD): left alone the compiler spreads
// their registers over the loop and gives up a wave or more against the single-view kernels;
// these are the highest targets reached without spilling.
template <Mode M> constexpr int waves_fwd() { return M == Mode::Plain ? 7 : 4; }
template <Mode M> constexpr int waves_bwd() { return M == Mode::Plain ? 5 : 4; }

template <Mode M, int NB>
__global__ __launch_bounds__(kBlock, fit_waves(waves_fwd<M>(), lds_fwd<M, NB>()))
void k_blend_fwd_batched(Queues Q) {
    __shared__ Stage<M, NB> S;
    __shared__ int s_view;
    __shared__ int64_t s_tile;
    int q = int(blockIdx.x % kXcds), tried = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            int view = -1;
            int64_t tile = 0;
            if (!next_item(Q, q, tried, view, tile)) view = -1;
            s_view = view;
            s_tile = tile;
        }
        __syncthreads();
        // the item is block-uniform: move it to scalar registers so the view descriptor is read
        // with scalar loads and its pointers stay in SGPRs
        const int view = __builtin_amdgcn_readfirstlane(s_view);
        const int64_t tile = uniform_i64(s_tile);
        __syncthreads();
        if (view < 0) break;
        const ViewDesc vd = Q.views[view];
        fwd_tile<M, NB>(vd, tile, S);
        __syncthreads();
    }
}

template <Mode M, int NB, bool kMM>
__global__ __launch_bounds__(kBlock, fit_waves(kMM ? 3 : waves_bwd<M>(), lds_bwd<M, NB, kMM>()))
void k_blend_bwd_batched(Queues Q) {
    __shared__ Stage<M, NB> S;
    __shared__ StageBwd<NB> SB;
    __shared__ BwdAcc<NB> s_acc;
    __shared__ MMTiles<kMM> s_mm;
    __shared__ int s_maxlast;
    __shared__ int s_view;
    __shared__ int64_t s_tile;
    int q = int(blockIdx.x % kXcds), tried = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            int view = -1;
            int64_t tile = 0;
            if (!next_item(Q, q, tried, view, tile)) view = -1;
            s_view = view;
            s_tile = tile;
        }
        __syncthreads();
        const int view = __builtin_amdgcn_readfirstlane(s_view);
        const int64_t tile = uniform_i64(s_tile);
        __syncthreads();
        if (view < 0) break;
        const ViewDesc vd = Q.views[view];
        bwd_tile<M, NB, kMM>(vd, tile, S, SB, &s_acc, s_maxlast, mm_ptr<kMM>(s_mm));
        __syncthreads();
    }
}

// The same items in one non-persistent launch: block b takes item b / 8 of queue b % 8 (the
// dispatcher places block b on XCD b % 8 and hands out blocks in index order, so each XCD still
// walks its own bands heaviest view first). No loop state: registers as in the single-view
// kernels.
__device__ inline bool grid_item(const Queues &Q, int64_t b, int &view, int64_t &tile) {
    const int x = int(b % kXcds);
    const int64_t i = b / kXcds;
    const int64_t *pre = Q.prefix + int64_t(x) * (Q.n_views + 1);
    if (i >= pre[Q.n_views]) return false;
    int lo = 0, hi = Q.n_views - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= i) lo = mid; else hi = mid - 1;
    }
    view = lo;
    const ViewDesc &vw = Q.views[lo];
    tile = strip_tile(band_lo(vw.n_tiles, x) + (i - pre[lo]), vw.n_tiles, vw.gx);
    return true;
}

template <Mode M, int NB>
__global__ __launch_bounds__(kBlock, fit_waves(M == Mode::Plain ? 8 : 7, lds_fwd<M, NB>()))
void k_blend_fwd_grid(Queues Q) {
    __shared__ Stage<M, NB> S;
    int view;
    int64_t tile;
    if (!grid_item(Q, blockIdx.x, view, tile)) return;
    const ViewDesc vd = Q.views[view];
    fwd_tile<M, NB>(vd, tile, S);
}

template <Mode M, int NB, bool kMM>
__global__ __launch_bounds__(kBlock, fit_waves(waves_bwd_tile<M, kMM>(), lds_bwd<M, NB, kMM>()))
void k_blend_bwd_grid(Queues Q) {
    __shared__ Stage<M, NB> S;
    __shared__ StageBwd<NB> SB;
    __shared__ BwdAcc<NB> s_acc;
    __shared__ MMTiles<kMM> s_mm;
    __shared__ int s_maxlast;
    int view;
    int64_t tile;
    if (!grid_item(Q, blockIdx.x, view, tile)) return;
    const ViewDesc vd = Q.views[view];
    bwd_tile<M, NB, kMM>(vd, tile, S, SB, &s_acc, s_maxlast, mm_ptr<kMM>(s_mm));
}

// Raw sums -> gradients of the stored scalars: d/dA = -S_xx/2, d/dB = -S_xy, d/dC = -S_yy/2,
// d/dx = -(A S_x + B S_y), d/dy = -(B S_x + C S_y) (power = -A dx^2/2 - B dx dy - C dy^2/2).
// blockIdx.y selects the view.
__global__ __launch_bounds__(256) void k_bwd_finish(const ViewDesc *views, ViewDesc single) {
    const ViewDesc &v = views ? views[blockIdx.y] : single;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= v.n) return;
    F3 c;
    float o;
    if (v.records) {                 // (x, y, A, B), (C, o, ...): conic and opacity from the record
        const float4 r0 = v.records[3 * i], r1 = v.records[3 * i + 1];
        c = F3{r0.z, r0.w, r1.x};
        o = r1.y;
    } else {
        c = reinterpret_cast<const F3 *>(v.conics)[i];
        o = v.opacity[i];
    }
    v.dL_dopacity[i] = opacity_grad(v.dL_dopacity[i], o);
    F3 *dc = reinterpret_cast<F3 *>(v.dL_dconics);
    float2 *dm = reinterpret_cast<float2 *>(v.dL_dmeans2d);
    const F3 s = dc[i];
    const float2 m = dm[i];
    dc[i] = F3{-0.5f * s.a, -s.b, -0.5f * s.c};
    dm[i] = make_float2(-(c.a * m.x + c.b * m.y), -(c.b * m.x + c.c * m.y));
}

// Zero every gradient output (graph-capturable: a kernel, not a memset). blockIdx.y = view.
__global__ __launch_bounds__(256) void k_zero_grads(const ViewDesc *views, ViewDesc single) {
    const ViewDesc &v = views ? views[blockIdx.y] : single;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= v.n) return;
    v.dL_dmeans2d[2 * i] = 0.f; v.dL_dmeans2d[2 * i + 1] = 0.f;
    v.dL_dconics[3 * i] = 0.f; v.dL_dconics[3 * i + 1] = 0.f; v.dL_dconics[3 * i + 2] = 0.f;
    v.dL_dopacity[i] = 0.f;
    v.dL_dcolors[3 * i] = 0.f; v.dL_dcolors[3 * i + 1] = 0.f; v.dL_dcolors[3 * i + 2] = 0.f;
}

__global__ void k_reset_counters(unsigned int *c, int m) {
    if (int(threadIdx.x) < m) c[threadIdx.x] = 0u;
}

// ------------------------------------------------------------------------------- dispatch
bool valid_batch(int nb) { return nb == 64 || nb == 128 || nb == 256; }

template <Mode M>
void launch_fwd_single(const ViewDesc &v, int nb, hipStream_t s) {
    const dim3 grid(unsigned(xcd_grid(v.n_tiles)));
    if (nb == 64) k_blend_fwd<M, 64><<<grid, kBlock, 0, s>>>(v);
    else if (nb == 128) k_blend_fwd<M, 128><<<grid, kBlock, 0, s>>>(v);
    else k_blend_fwd<M, 256><<<grid, kBlock, 0, s>>>(v);
}

template <Mode M, bool kMM>
void launch_bwd_single(const ViewDesc &v, int nb, hipStream_t s) {
    const dim3 grid(unsigned(xcd_grid(v.n_tiles)));
    if (nb == 64) k_blend_bwd<M, 64, kMM><<<grid, kBlock, 0, s>>>(v);
    else if (nb == 128) k_blend_bwd<M, 128, kMM><<<grid, kBlock, 0, s>>>(v);
    else k_blend_bwd<M, 256, kMM><<<grid, kBlock, 0, s>>>(v);
}
template <Mode M>
void launch_bwd_single(const ViewDesc &v, int nb, bool mm, hipStream_t s) {
    if (mm) launch_bwd_single<M, true>(v, nb, s);
    else launch_bwd_single<M, false>(v, nb, s);
}

template <Mode M>
const void *fwd_batched_fn(int nb) {
    if (nb == 64) return reinterpret_cast<const void *>(&k_blend_fwd_batched<M, 64>);
    if (nb == 128) return reinterpret_cast<const void *>(&k_blend_fwd_batched<M, 128>);
    return reinterpret_cast<const void *>(&k_blend_fwd_batched<M, 256>);
}
template <Mode M, bool kMM>
const void *bwd_batched_fn(int nb) {
    if (nb == 64) return reinterpret_cast<const void *>(&k_blend_bwd_batched<M, 64, kMM>);
    if (nb == 128) return reinterpret_cast<const void *>(&k_blend_bwd_batched<M, 128, kMM>);
    return reinterpret_cast<const void *>(&k_blend_bwd_batched<M, 256, kMM>);
}
template <Mode M>
const void *bwd_batched_fn(int nb, bool mm) {
    return mm ? bwd_batched_fn<M, true>(nb) : bwd_batched_fn<M, false>(nb);
}
const void *batched_fn(gsb_precision prec, bool fwd, int nb, bool mm) {
    switch (prec) {
        case GSB_FP32_PLAIN: return fwd ? fwd_batched_fn<Mode::Plain>(nb) : bwd_batched_fn<Mode::Plain>(nb, mm);
        case GSB_FP16_GEMM: return fwd ? fwd_batched_fn<Mode::F16>(nb) : bwd_batched_fn<Mode::F16>(nb, mm);
        default: return fwd ? fwd_batched_fn<Mode::BF16>(nb) : bwd_batched_fn<Mode::BF16>(nb, mm);
    }
}

}  // namespace

ViewDesc make_view(int32_t W, int32_t H, const uint32_t *ranges, const uint32_t *point_list,
                   const float *means2d, const float *conics, const float *opacity,
                   const float *colors, int64_t n, const float bg[3]) {
    ViewDesc v{};
    v.W = W; v.H = H; v.gx = int32_t(grid_x(W));
    v.n_tiles = grid_x(W) * grid_y(H);
    v.ranges = ranges; v.point_list = point_list; v.n = n;
    v.means2d = means2d; v.conics = conics; v.opacity = opacity; v.colors = colors;
    v.bg[0] = bg[0]; v.bg[1] = bg[1]; v.bg[2] = bg[2];
    return v;
}

gsb_status blend_forward(const ViewDesc &v, gsb_precision prec, int nb, hipStream_t s) {
    if (!valid_batch(nb)) return fail(GSB_ERR_INVALID, "batch %d not in {64, 128, 256}", nb);
    switch (prec) {
        case GSB_FP32_PLAIN: launch_fwd_single<Mode::Plain>(v, nb, s); break;
        case GSB_FP16_GEMM: launch_fwd_single<Mode::F16>(v, nb, s); break;
        case GSB_BF16_GEMM: launch_fwd_single<Mode::BF16>(v, nb, s); break;
        default: return fail(GSB_ERR_INVALID, "unknown precision %d", int(prec));
    }
    return check_launch("blend_forward");
}

gsb_status blend_backward(const ViewDesc &v, gsb_precision prec, int nb, bool mm, hipStream_t s) {
    if (!valid_batch(nb)) return fail(GSB_ERR_INVALID, "batch %d not in {64, 128, 256}", nb);
    if (prec != GSB_FP32_PLAIN && prec != GSB_FP16_GEMM && prec != GSB_BF16_GEMM)
        return fail(GSB_ERR_INVALID, "unknown precision %d", int(prec));
    const unsigned gz = unsigned((v.n + 255) / 256);
    if (v.n > 0) k_zero_grads<<<dim3(gz, 1), 256, 0, s>>>(nullptr, v);
    switch (prec) {
        case GSB_FP32_PLAIN: launch_bwd_single<Mode::Plain>(v, nb, mm, s); break;
        case GSB_FP16_GEMM: launch_bwd_single<Mode::F16>(v, nb, mm, s); break;
        default: launch_bwd_single<Mode::BF16>(v, nb, mm, s); break;
    }
    if (v.n > 0) k_bwd_finish<<<dim3(gz, 1), 256, 0, s>>>(nullptr, v);
    return check_launch("blend_backward");
}

gsb_status pack_gaussians(const float *means2d, const float *conics, const float *opacity,
                          const float *colors, int64_t n, float *records, hipStream_t s) {
    if (n > 0)
        k_pack<<<dim3(unsigned((n + 255) / 256)), 256, 0, s>>>(
            reinterpret_cast<const float2 *>(means2d), reinterpret_cast<const F3 *>(conics),
            opacity, reinterpret_cast<const F3 *>(colors), n, reinterpret_cast<float4 *>(records));
    return check_launch("pack_gaussians");
}

gsb_status blend_forward_packed(const ViewDesc &v, gsb_precision prec, hipStream_t s) {
    const dim3 grid(unsigned(xcd_grid(v.n_tiles)));
    switch (prec) {
        case GSB_FP32_PLAIN: k_blend_fwd_rec<Mode::Plain><<<grid, kBlock, 0, s>>>(v); break;
        case GSB_FP16_GEMM: k_blend_fwd_rec<Mode::F16><<<grid, kBlock, 0, s>>>(v); break;
        case GSB_BF16_GEMM: k_blend_fwd_rec<Mode::BF16><<<grid, kBlock, 0, s>>>(v); break;
        default: return fail(GSB_ERR_INVALID, "unknown precision %d", int(prec));
    }
    return check_launch("blend_forward_packed");
}

gsb_status blend_backward_packed(const ViewDesc &v, gsb_precision prec, hipStream_t s) {
    if (prec != GSB_FP32_PLAIN && prec != GSB_FP16_GEMM && prec != GSB_BF16_GEMM)
        return fail(GSB_ERR_INVALID, "unknown precision %d", int(prec));
    const unsigned gz = unsigned((v.n + 255) / 256);
    const dim3 grid(unsigned(xcd_grid(v.n_tiles)));
    if (v.n > 0) k_zero_grads<<<dim3(gz, 1), 256, 0, s>>>(nullptr, v);
    switch (prec) {
        case GSB_FP32_PLAIN: k_blend_bwd_rec<Mode::Plain><<<grid, kBlock, 0, s>>>(v); break;
        case GSB_FP16_GEMM: k_blend_bwd_rec<Mode::F16><<<grid, kBlock, 0, s>>>(v); break;
        default: k_blend_bwd_rec<Mode::BF16><<<grid, kBlock, 0, s>>>(v); break;
    }
    if (v.n > 0) k_bwd_finish<<<dim3(gz, 1), 256, 0, s>>>(nullptr, v);
    return check_launch("blend_backward_packed");
}

// Deterministic-backward workspace: per list position its nine sums, the (Gaussian, position)
// pairs in two buffers each for the sort, the sort's scratch, the pair count and the per-Gaussian
// ranges of the sorted positions.
namespace {
struct DetLayout {
    size_t partial, ka, kb, va, vb, count, seg, scratch, end;
};
size_t al256(size_t b) { return (b + 255) & ~size_t(255); }
DetLayout det_layout(int64_t n, int64_t pairs) {
    const size_t P = size_t(pairs > 0 ? pairs : 1), N = size_t(n > 0 ? n : 1);
    DetLayout L;
    size_t o = 0;
    L.partial = o; o += al256(sizeof(float) * kDetStride * P);
    L.ka = o;      o += al256(sizeof(uint32_t) * P);
    L.kb = o;      o += al256(sizeof(uint32_t) * P);
    L.va = o;      o += al256(sizeof(uint32_t) * P);
    L.vb = o;      o += al256(sizeof(uint32_t) * P);
    L.count = o;   o += al256(sizeof(unsigned long long));
    L.seg = o;     o += al256(sizeof(uint32_t) * 2 * N);
    L.scratch = o; o += al256(pair_sort_scratch_bytes(pairs));
    L.end = o;
    return L;
}
int bits_for(int64_t n) {
    int b = 1;
    while (b < 32 && (int64_t(1) << b) < n) ++b;
    return b;
}
}  // namespace

size_t backward_det_workspace_bytes(int64_t n, int64_t pairs) { return det_layout(n, pairs).end; }

gsb_status blend_backward_det(const ViewDesc &v0, gsb_precision prec, int64_t pairs, void *ws,
                              hipStream_t s) {
    const DetLayout D = det_layout(v0.n, pairs);
    char *w = static_cast<char *>(ws);
    ViewDesc v = v0;
    v.det_partial = reinterpret_cast<float *>(w + D.partial);
    v.det_pairs = pairs;
    uint32_t *ka = reinterpret_cast<uint32_t *>(w + D.ka), *kb = reinterpret_cast<uint32_t *>(w + D.kb);
    uint32_t *va = reinterpret_cast<uint32_t *>(w + D.va), *vb = reinterpret_cast<uint32_t *>(w + D.vb);
    auto *count = reinterpret_cast<unsigned long long *>(w + D.count);
    uint32_t *seg = reinterpret_cast<uint32_t *>(w + D.seg);
    const int64_t m = std::max(pairs, 2 * v.n);
    if (m > 0)
        k_det_init<<<dim3(unsigned((m + 255) / 256)), 256, 0, s>>>(v.point_list, pairs, ka, va,
                                                                    count, seg, v.n);
    const dim3 grid(unsigned(xcd_grid(v.n_tiles)));
    switch (prec) {
        case GSB_FP32_PLAIN: k_blend_bwd_det<Mode::Plain><<<grid, kBlock, 0, s>>>(v); break;
        case GSB_FP16_GEMM: k_blend_bwd_det<Mode::F16><<<grid, kBlock, 0, s>>>(v); break;
        case GSB_BF16_GEMM: k_blend_bwd_det<Mode::BF16><<<grid, kBlock, 0, s>>>(v); break;
        default: return fail(GSB_ERR_INVALID, "unknown precision %d", int(prec));
    }
    if (pairs > 0 && v.n > 0) {
        const int passes = pair_sort(ka, kb, va, vb, count, pairs, bits_for(v.n), w + D.scratch, s);
        const uint32_t *skeys = passes % 2 ? kb : ka;
        const uint32_t *spos = passes % 2 ? vb : va;
        key_ranges(skeys, count, pairs, seg, s);
        if (v.n > 0)
            k_det_gather<<<dim3(unsigned((v.n + 4 * kGatherPer - 1) / (4 * kGatherPer))), 256, 0, s>>>(
                v.records, v.det_partial, spos, seg, v.n, v.dL_dmeans2d, v.dL_dconics,
                v.dL_dopacity, v.dL_dcolors);
    } else if (v.n > 0) {
        k_zero_grads<<<dim3(unsigned((v.n + 255) / 256), 1), 256, 0, s>>>(nullptr, v);
    }
    return check_launch("blend_backward_deterministic");
}

// ------------------------------------------------------------------------------- plans
struct Plan {
    int device = 0;
    int n_views = 0;
    gsb_precision prec = GSB_FP16_GEMM;
    Tuning tune{};
    int64_t max_n = 0;
    ViewDesc *d_views = nullptr;    // device copy, plan order
    int64_t *d_prefix = nullptr;    // [8][n_views + 1]
    unsigned int *d_counters = nullptr;   // [16]: forward queues, backward queues
    int grid_fwd = 0, grid_bwd = 0;   // persistent grids
    int64_t grid_items = 0;            // one-shot grid: 8 x the longest queue
};

gsb_status plan_create(const ViewDesc *views, int n_views, gsb_precision prec, const Tuning &t,
                       Plan **out) {
    if (!valid_batch(t.batch_fwd) || !valid_batch(t.batch_bwd))
        return fail(GSB_ERR_INVALID, "batch sizes must be 64, 128 or 256");
    if (t.launch != kLaunchPersistent && t.launch != kLaunchGrid)
        return fail(GSB_ERR_INVALID, "launch mode %d unknown", t.launch);
    Plan *p = new Plan();
    p->n_views = n_views;
    p->prec = prec;
    p->tune = t;
    hipError_t e = hipGetDevice(&p->device);
    // heaviest-first: Gaussians per tile is proportional to the mean tile list length
    std::vector<int> order(n_views);
    for (int i = 0; i < n_views; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return double(views[a].n) / double(views[a].n_tiles) > double(views[b].n) / double(views[b].n_tiles);
    });
    std::vector<ViewDesc> ordered(n_views);
    for (int i = 0; i < n_views; ++i) {
        ordered[i] = views[order[i]];
        p->max_n = std::max(p->max_n, ordered[i].n);
    }
    std::vector<int64_t> prefix(size_t(kXcds) * (n_views + 1), 0);
    for (int x = 0; x < kXcds; ++x) {
        int64_t run = 0;
        for (int k = 0; k < n_views; ++k) {
            prefix[size_t(x) * (n_views + 1) + k] = run;
            const int64_t T = ordered[k].n_tiles;
            run += T * (x + 1) / kXcds - T * x / kXcds;
        }
        prefix[size_t(x) * (n_views + 1) + n_views] = run;
        p->grid_items = std::max(p->grid_items, run * kXcds);
    }
    if (e == hipSuccess) e = hipMalloc(&p->d_views, sizeof(ViewDesc) * size_t(n_views));
    if (e == hipSuccess) e = hipMalloc(&p->d_prefix, sizeof(int64_t) * prefix.size());
    if (e == hipSuccess) e = hipMalloc(&p->d_counters, sizeof(unsigned int) * 2 * kXcds);
    if (e == hipSuccess) e = hipMemcpy(p->d_views, ordered.data(), sizeof(ViewDesc) * size_t(n_views), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_prefix, prefix.data(), sizeof(int64_t) * prefix.size(), hipMemcpyHostToDevice);
    int cus = 0, occ_f = 0, occ_b = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_f, batched_fn(prec, true, t.batch_fwd, false), kBlock, 0);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_b, batched_fn(prec, false, t.batch_bwd, t.bwd_mm != 0), kBlock, 0);
    if (e != hipSuccess) {
        (void)plan_destroy(p);      // the creation error is the one reported
        return fail(GSB_ERR_HIP, "plan_create: %s", hipGetErrorString(e));
    }
    const int want = t.blocks_per_cu > 0 ? t.blocks_per_cu : 1 << 30;
    p->grid_fwd = cus * std::max(1, std::min(want, occ_f));
    p->grid_bwd = cus * std::max(1, std::min(want, occ_b));
    // a multiple of 8 keeps every XCD's queue served by the same number of blocks
    p->grid_fwd = (p->grid_fwd + kXcds - 1) / kXcds * kXcds;
    p->grid_bwd = (p->grid_bwd + kXcds - 1) / kXcds * kXcds;
    *out = p;
    return GSB_OK;
}

hipError_t plan_destroy(Plan *p) {
    if (!p) return hipSuccess;
    // every buffer is freed; the first failure is the one reported
    hipError_t e = hipSuccess;
    for (void *d : {static_cast<void *>(p->d_views), static_cast<void *>(p->d_prefix),
                    static_cast<void *>(p->d_counters)}) {
        if (!d) continue;
        const hipError_t f = hipFree(d);
        if (e == hipSuccess) e = f;
    }
    delete p;
    return e;
}

template <Mode M>
void launch_fwd_batched(const Queues &Q, int nb, const Plan &p, hipStream_t s) {
    if (p.tune.launch == kLaunchGrid) {
        const dim3 g(unsigned(p.grid_items));
        if (nb == 64) k_blend_fwd_grid<M, 64><<<g, kBlock, 0, s>>>(Q);
        else if (nb == 128) k_blend_fwd_grid<M, 128><<<g, kBlock, 0, s>>>(Q);
        else k_blend_fwd_grid<M, 256><<<g, kBlock, 0, s>>>(Q);
        return;
    }
    const int grid = p.grid_fwd;
    if (nb == 64) k_blend_fwd_batched<M, 64><<<grid, kBlock, 0, s>>>(Q);
    else if (nb == 128) k_blend_fwd_batched<M, 128><<<grid, kBlock, 0, s>>>(Q);
    else k_blend_fwd_batched<M, 256><<<grid, kBlock, 0, s>>>(Q);
}
template <Mode M, bool kMM>
void launch_bwd_batched(const Queues &Q, int nb, const Plan &p, hipStream_t s) {
    if (p.tune.launch == kLaunchGrid) {
        const dim3 g(unsigned(p.grid_items));
        if (nb == 64) k_blend_bwd_grid<M, 64, kMM><<<g, kBlock, 0, s>>>(Q);
        else if (nb == 128) k_blend_bwd_grid<M, 128, kMM><<<g, kBlock, 0, s>>>(Q);
        else k_blend_bwd_grid<M, 256, kMM><<<g, kBlock, 0, s>>>(Q);
        return;
    }
    const int grid = p.grid_bwd;
    if (nb == 64) k_blend_bwd_batched<M, 64, kMM><<<grid, kBlock, 0, s>>>(Q);
    else if (nb == 128) k_blend_bwd_batched<M, 128, kMM><<<grid, kBlock, 0, s>>>(Q);
    else k_blend_bwd_batched<M, 256, kMM><<<grid, kBlock, 0, s>>>(Q);
}
template <Mode M>
void launch_bwd_batched(const Queues &Q, int nb, const Plan &p, hipStream_t s) {
    if (p.tune.bwd_mm) launch_bwd_batched<M, true>(Q, nb, p, s);
    else launch_bwd_batched<M, false>(Q, nb, p, s);
}

gsb_status plan_forward(Plan *p, hipStream_t s) {
    if (p->n_views == 0) return GSB_OK;
    Queues Q{p->d_views, p->d_prefix, p->d_counters, p->n_views};
    if (p->tune.launch == kLaunchPersistent) k_reset_counters<<<1, 64, 0, s>>>(p->d_counters, kXcds);
    switch (p->prec) {
        case GSB_FP32_PLAIN: launch_fwd_batched<Mode::Plain>(Q, p->tune.batch_fwd, *p, s); break;
        case GSB_FP16_GEMM: launch_fwd_batched<Mode::F16>(Q, p->tune.batch_fwd, *p, s); break;
        default: launch_fwd_batched<Mode::BF16>(Q, p->tune.batch_fwd, *p, s); break;
    }
    return check_launch("blend_batched_forward");
}

gsb_status plan_backward(Plan *p, hipStream_t s) {
    if (p->n_views == 0) return GSB_OK;
    Queues Q{p->d_views, p->d_prefix, p->d_counters + kXcds, p->n_views};
    const dim3 gz(unsigned((p->max_n + 255) / 256 > 0 ? (p->max_n + 255) / 256 : 1), unsigned(p->n_views));
    k_zero_grads<<<gz, 256, 0, s>>>(p->d_views, ViewDesc{});
    if (p->tune.launch == kLaunchPersistent)
        k_reset_counters<<<1, 64, 0, s>>>(p->d_counters + kXcds, kXcds);
    switch (p->prec) {
        case GSB_FP32_PLAIN: launch_bwd_batched<Mode::Plain>(Q, p->tune.batch_bwd, *p, s); break;
        case GSB_FP16_GEMM: launch_bwd_batched<Mode::F16>(Q, p->tune.batch_bwd, *p, s); break;
        default: launch_bwd_batched<Mode::BF16>(Q, p->tune.batch_bwd, *p, s); break;
    }
    k_bwd_finish<<<gz, 256, 0, s>>>(p->d_views, ViewDesc{});
    return check_launch("blend_batched_backward");
}

}  // namespace gsb
