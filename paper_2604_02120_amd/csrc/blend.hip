// Tile blending of depth-sorted projected 2D Gaussians on gfx950: forward (Eq. (volume-render)
// with the per-pixel loop of Alg. 1) and backward, with the Gaussian exponent evaluated either
//   PLAIN : per pixel on the vector ALUs in FP32 from Eq. (power), or
//   F16 / BF16 : as the product M_power = M_g . M_p of Eq. (power rewritten) / Eq. (matrix
//          multiplication) on the matrix cores (MFMA), FP16 or BF16 operands, FP32 accumulation.
//
// Launch shape: one 256-thread block (4 wavefronts) per 16x16 tile, one pixel per lane; wave w
// owns tile rows 4w..4w+3. The tile's sorted list is walked in batches of 256 Gaussians: every
// thread stages one Gaussian into LDS (double-buffered; the next batch's global loads are issued
// before the current batch is composited), then each wave composites the batch for its pixels.
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

#include "gsb_internal.h"

namespace gsb {
namespace {

enum class Mode { Plain, F16, BF16 };

constexpr int kGroup = 16;                  // Gaussians per MFMA group
// Gaussians staged per batch (at most one per thread): forward and backward defaults.
constexpr int kBatchFwd = 256;
constexpr int kBatchBwd = 128;
constexpr float kLog2e = 0x1.715476p+0f;    // log2(e) rounded to FP32
constexpr float kQCull = -0x1.ffa37cp+2f;   // log2(fp32(1/255)) rounded to FP32
constexpr float kTauCull = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTStop = 1e-4f;
constexpr float kLoScale = 4096.0f;         // 2^12
constexpr float kLoScaleInv = 1.0f / 4096.0f;
constexpr float kF16Max = 65504.0f;

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
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
    vec alo[2][NB];            // v_g lo terms * 2^12
    float kc[2][NB];           // accumulator init: constant term + log2 o (-inf = inert)
    float4 attr[2][NB];        // (log2 o, r, g, b)
    vec zero;
};
template <int NB>
struct Stage<Mode::Plain, NB> {  // plain form
    float4 geo[2][NB];         // (x, y, A, B)
    float2 geo2[2][NB];        // (C, log2 o)
    float4 attr[2][NB];        // (log2 o, r, g, b)
};

template <int NB>
struct StageBwd {
    float4 bwd[2][NB];         // (x, y, 1/o, index bits)
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

// An index >= n (an inconsistent list) is treated as an empty slot rather than dereferenced.
__device__ inline GRaw fetch(const uint32_t *plist, int64_t pos, bool valid, uint32_t n,
                             const float2 *means, const F3 *conics, const float *opac,
                             const F3 *colors) {
    GRaw g;
    g.id = valid ? plist[pos] : 0u;
    valid = valid && g.id < n;
    g.valid = valid;
    if (valid) {
        const float2 m = means[g.id];
        const F3 c = conics[g.id];
        const F3 col = colors[g.id];
        g.x = m.x; g.y = m.y; g.A = c.a; g.B = c.b; g.C = c.c;
        g.o = opac[g.id];
        g.r = col.a; g.g = col.b; g.b = col.c;
    } else {
        g.id = 0; g.x = g.y = g.A = g.B = g.C = g.o = g.r = g.g = g.b = 0.f;
    }
    return g;
}

// Writes one Gaussian into slot `slot` of buffer `buf`. (xc, yc) is the tile centre.
template <Mode M, int NB, bool Bwd>
__device__ inline void stage(const GRaw &g, int buf, int slot, float xc, float yc, Stage<M, NB> &S,
                             StageBwd<NB> *SB) {
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
    if constexpr (Bwd) {
        SB->bwd[buf][slot] = make_float4(g.x, g.y, live ? 1.0f / g.o : 0.f, __uint_as_float(g.id));
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
    L.col = L.l & 15; L.row = 4 * L.w + (L.l >> 4);
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
template <Mode M, int NB>
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
    const typename Op<M>::vec *ph = L.a_valid ? &S.ahi[buf][g * kGroup + L.a_g] : &S.zero;
    const typename Op<M>::vec *pl = L.a_valid ? &S.alo[buf][g * kGroup + L.a_g] : &S.zero;
    const typename Op<M>::vec ah = *ph, al = *pl;
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

__device__ inline void composite(float q, const float4 *attr, int idx, int pos, FwdState &st) {
    if (q >= st.thr) {
        const float4 at = attr[idx];
        const float a = fminf(__builtin_amdgcn_exp2f(fminf(q, at.x)), kAlphaMax);
        const float Tn = st.T * (1.0f - a);
        if (Tn < kTStop) {
            st.thr = INFINITY;
        } else {
            const float wgt = a * st.T;
            st.r += wgt * at.y; st.g += wgt * at.z; st.b += wgt * at.w;
            st.T = Tn;
            st.last = pos + 1;
        }
    }
}

template <Mode M, int NB>
__global__ __launch_bounds__(kBlock) void k_blend_fwd(
    int W, int H, int gx, int64_t n_tiles, const uint2 *ranges, const uint32_t *plist,
    uint32_t n, const float2 *means, const F3 *conics, const float *opac, const F3 *colors, float bg0,
    float bg1, float bg2, float *image, float *final_T, int32_t *last_contrib) {
    static_assert(NB % kGroup == 0 && NB <= kBlock, "batch must be whole groups, <= block");
    constexpr int kGroups = NB / kGroup;
    __shared__ Stage<M, NB> S;
    const int64_t tile = xcd_tile(blockIdx.x, n_tiles);
    if (tile >= n_tiles) return;
    const Lane L = lane_setup(tile, gx, W, H);
    const float xc = float(int(tile % gx) * kTile) + 7.5f, yc = float(int(tile / gx) * kTile) + 7.5f;
    typename Op<M>::vec bhi, blo;
    pixel_basis<M>(L, bhi, blo);
    if (L.t == 0) {
        float z[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if constexpr (M != Mode::Plain) S.zero = Op<M>::cvt(z);
    }
    const uint2 rg = ranges[tile];
    const int64_t start = rg.x, len = int64_t(rg.y) - int64_t(rg.x);
    const int nb = int((len + NB - 1) / NB);

    FwdState st{1.f, 0.f, 0.f, 0.f, L.inside ? kQCull : INFINITY, 0};
    GRaw nxt = fetch(plist, start + L.t, L.t < NB && L.t < len, n, means, conics, opac, colors);
    for (int b = 0; b < nb; ++b) {
        const int buf = b & 1;
        if (L.t < NB) stage<M, NB, false>(nxt, buf, L.t, xc, yc, S, nullptr);
        // barrier; also counts the pixels still live (the whole block leaves once none is)
        if (__syncthreads_count(st.thr != INFINITY) == 0) break;
        if (b + 1 < nb) {
            const int64_t o = int64_t(b + 1) * NB + L.t;
            nxt = fetch(plist, start + o, L.t < NB && o < len, n, means, conics, opac, colors);
        }
        const int base = b * NB;
        const int ng = int((len - base + kGroup - 1) / kGroup) < kGroups
                           ? int((len - base + kGroup - 1) / kGroup) : kGroups;
        for (int g = 0; g < ng; ++g) {
            if (__ballot(st.thr != INFINITY) == 0) break;
            if constexpr (M == Mode::Plain) {
#pragma unroll
                for (int v = 0; v < kGroup; ++v) {
                    const int idx = g * kGroup + v;
                    composite(plain_q(S, buf, idx, L), S.attr[buf], idx, base + idx, st);
                }
            } else {
                const f16x q = group_q_mfma<M, NB>(S, buf, g, L, bhi, blo);
#pragma unroll
                for (int v = 0; v < kGroup; ++v)
                    composite(q[v], S.attr[buf], g * kGroup + v, base + g * kGroup + v, st);
            }
        }
    }
    if (L.inside) {
        const int64_t p = int64_t(L.py) * W + int64_t(L.px);
        const int64_t HW = int64_t(H) * W;
        image[p] = st.r + st.T * bg0;
        image[HW + p] = st.g + st.T * bg1;
        image[2 * HW + p] = st.b + st.T * bg2;
        final_T[p] = st.T;
        last_contrib[p] = st.last;
    }
}

// ------------------------------------------------------------------------------- backward
// Sum over each row of 16 lanes with DPP row shifts; lane 15 of every row (lanes 15, 31, 47, 63)
// ends up holding its row's total. Call with every lane active.
template <int Ctrl>
__device__ inline float dpp_add(float x) {
    const int y = __builtin_amdgcn_update_dpp(0, __float_as_int(x), Ctrl, 0xf, 0xf, false);
    return x + __int_as_float(y);
}
__device__ inline float row_sum16(float x) {
    x = dpp_add<0x111>(x);  // row_shr:1
    x = dpp_add<0x112>(x);  // row_shr:2
    x = dpp_add<0x114>(x);  // row_shr:4
    x = dpp_add<0x118>(x);  // row_shr:8
    return x;
}

constexpr int kGrad = 9;   // per-Gaussian sums kept per batch

struct BwdState {
    float T, Tfin, behind, gr, gg, gb, bgg;
    int last;
};

// Reverse step for one (Gaussian, pixel) pair. Nothing but a compare and a scalar branch is
// spent when no lane of the wave has a live pair. Otherwise the pair's 9 gradient terms are summed
// over each row of 16 lanes and the row totals are added into the Gaussian's LDS accumulator
// (`acc`), which the block flushes to global memory once per batch. Raw sums: S_xx, S_xy, S_yy,
// S_x, S_y (times dL/dpower), dL/do, and the three colour gradients.
__device__ inline void reverse_pair(float q, bool in_range, const float4 *attr_p,
                                    const float4 *bw_p, const Lane &L, BwdState &st, float *acc) {
    const bool alive = in_range && (q >= kQCull);
    const unsigned long long live = __builtin_amdgcn_ballot_w64(alive);
    if (live == 0ull) return;
    float s[kGrad] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (alive) {
        const float4 attr = *attr_p;
        const float araw = __builtin_amdgcn_exp2f(fminf(q, attr.x));
        const float a = fminf(araw, kAlphaMax);
        const float r = __builtin_amdgcn_rcpf(1.0f - a);
        const float Tb = st.T * r;                       // T in front of this Gaussian
        const float gc = st.gr * attr.y + st.gg * attr.z + st.gb * attr.w;
        const float dLda = Tb * gc - (st.behind + st.Tfin * st.bgg) * r;
        const float wc = a * Tb;
        st.behind = fmaf(wc, gc, st.behind);
        st.T = Tb;
        s[6] = wc * st.gr; s[7] = wc * st.gg; s[8] = wc * st.gb;
        const bool clamp_a = araw >= kAlphaMax;
        const bool clamp_p = q > attr.x;   // power > 0
        if (!clamp_a) {
            const float4 bw = *bw_p;
            s[5] = a * bw.z * dLda;        // d alpha / d o = alpha / o
            if (!clamp_p) {
                const float dP = a * dLda;  // d alpha / d power = alpha
                const float dx = bw.x - L.px, dy = bw.y - L.py;
                const float tx = dP * dx, ty = dP * dy;
                s[0] = tx * dx; s[1] = tx * dy; s[2] = ty * dy;
                s[3] = tx; s[4] = ty;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kGrad; ++k) s[k] = row_sum16(s[k]);
    const bool row_live = ((live >> (L.l & 48)) & 0xffffull) != 0ull;
    if ((L.l & 15) == 15 && row_live) {
#pragma unroll
        for (int k = 0; k < kGrad; ++k) atomicAdd(&acc[k], s[k]);
    }
}

template <Mode M, int NB>
__global__ __launch_bounds__(kBlock) void k_blend_bwd(
    int W, int H, int gx, int64_t n_tiles, const uint2 *ranges, const uint32_t *plist,
    uint32_t n, const float2 *means, const F3 *conics, const float *opac, const F3 *colors, float bg0,
    float bg1, float bg2, const float *final_T, const int32_t *last_contrib,
    const float *dL_dimage, float *dmeans, float *dconics, float *dopac, float *dcolors) {
    static_assert(NB % kGroup == 0 && NB <= kBlock, "batch must be whole groups, <= block");
    constexpr int kGroups = NB / kGroup;
    __shared__ Stage<M, NB> S;
    __shared__ StageBwd<NB> SB;
    __shared__ float s_acc[NB][kGrad];   // per-Gaussian gradient sums of the current batch
    __shared__ int s_maxlast;
    const int64_t tile = xcd_tile(blockIdx.x, n_tiles);
    if (tile >= n_tiles) return;
    const Lane L = lane_setup(tile, gx, W, H);
    const float xc = float(int(tile % gx) * kTile) + 7.5f, yc = float(int(tile / gx) * kTile) + 7.5f;
    typename Op<M>::vec bhi, blo;
    pixel_basis<M>(L, bhi, blo);
    if (L.t == 0) {
        float z[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if constexpr (M != Mode::Plain) S.zero = Op<M>::cvt(z);
        s_maxlast = 0;
    }
    BwdState st{1.f, 1.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0};
    if (L.inside) {
        const int64_t p = int64_t(L.py) * W + int64_t(L.px);
        const int64_t HW = int64_t(H) * W;
        st.T = st.Tfin = final_T[p];
        st.last = last_contrib[p];
        st.gr = dL_dimage[p]; st.gg = dL_dimage[HW + p]; st.gb = dL_dimage[2 * HW + p];
        st.bgg = bg0 * st.gr + bg1 * st.gg + bg2 * st.gb;
    }
    __syncthreads();
    if (st.last > 0) atomicMax(&s_maxlast, st.last);
    __syncthreads();
    const uint2 rg = ranges[tile];
    const int64_t start = rg.x;
    // positions [0, max last) are the only ones that matter (never more than the list holds)
    const int64_t len = s_maxlast < int64_t(rg.y) - int64_t(rg.x) ? s_maxlast
                                                                   : int64_t(rg.y) - int64_t(rg.x);
    const int nb = int((len + NB - 1) / NB);
    if (nb == 0) return;

    GRaw nxt;
    {
        const int64_t o = int64_t(nb - 1) * NB + L.t;
        nxt = fetch(plist, start + o, L.t < NB && o < len, n, means, conics, opac, colors);
    }
    for (int b = nb - 1; b >= 0; --b) {
        const int buf = b & 1;
        if (L.t < NB) {
            stage<M, NB, true>(nxt, buf, L.t, xc, yc, S, &SB);
#pragma unroll
            for (int k = 0; k < kGrad; ++k) s_acc[L.t][k] = 0.f;
        }
        __syncthreads();
        if (b > 0) {
            const int64_t o = int64_t(b - 1) * NB + L.t;
            nxt = fetch(plist, start + o, L.t < NB && o < len, n, means, conics, opac, colors);
        }
        const int base = b * NB;
        const int ng = int((len - base + kGroup - 1) / kGroup) < kGroups
                           ? int((len - base + kGroup - 1) / kGroup) : kGroups;
        for (int g = ng - 1; g >= 0; --g) {
            // nothing to do for this wave unless one of its pixels blended past the group start
            if (__ballot(st.last > base + g * kGroup) == 0) continue;
            if constexpr (M == Mode::Plain) {
                const float4 *attr = &S.attr[buf][g * kGroup];
                const float4 *bw = &SB.bwd[buf][g * kGroup];
                float *acc = &s_acc[g * kGroup][0];
                const int rel = st.last - (base + g * kGroup);   // positions < last are in range
#pragma unroll
                for (int v = kGroup - 1; v >= 0; --v) {
                    const float q = plain_q(S, buf, g * kGroup + v, L);
                    reverse_pair(q, v < rel, attr + v, bw + v, L, st, acc + v * kGrad);
                }
            } else {
                const f16x q = group_q_mfma<M, NB>(S, buf, g, L, bhi, blo);
                const float4 *attr = &S.attr[buf][g * kGroup];
                const float4 *bw = &SB.bwd[buf][g * kGroup];
                float *acc = &s_acc[g * kGroup][0];
                const int rel = st.last - (base + g * kGroup);
#pragma unroll
                for (int v = kGroup - 1; v >= 0; --v)
                    reverse_pair(q[v], v < rel, attr + v, bw + v, L, st, acc + v * kGrad);
            }
        }
        // flush: thread t owns staged Gaussian t's sums (a Gaussian with no live pair in this
        // tile has all-zero sums and costs no atomics)
        __syncthreads();
        if (L.t >= NB) continue;
        float a9[kGrad];
        bool any = false;
#pragma unroll
        for (int k = 0; k < kGrad; ++k) {
            a9[k] = s_acc[L.t][k];
            any |= a9[k] != 0.f;
        }
        if (any) {
            const uint32_t id = __float_as_uint(SB.bwd[buf][L.t].w);
            unsafeAtomicAdd(&dconics[3 * id + 0], a9[0]);
            unsafeAtomicAdd(&dconics[3 * id + 1], a9[1]);
            unsafeAtomicAdd(&dconics[3 * id + 2], a9[2]);
            unsafeAtomicAdd(&dmeans[2 * id + 0], a9[3]);
            unsafeAtomicAdd(&dmeans[2 * id + 1], a9[4]);
            unsafeAtomicAdd(&dopac[id], a9[5]);
            unsafeAtomicAdd(&dcolors[3 * id + 0], a9[6]);
            unsafeAtomicAdd(&dcolors[3 * id + 1], a9[7]);
            unsafeAtomicAdd(&dcolors[3 * id + 2], a9[8]);
        }
        // the next iteration stages into the other buffer and re-zeroes slot t (program order
        // after this read); the buffer read here is rewritten two iterations later
    }
}

// Raw sums -> gradients of the stored scalars: d/dA = -S_xx/2, d/dB = -S_xy, d/dC = -S_yy/2,
// d/dx = -(A S_x + B S_y), d/dy = -(B S_x + C S_y) (power = -A dx^2/2 - B dx dy - C dy^2/2).
__global__ __launch_bounds__(256) void k_bwd_finish(int64_t n, const F3 *conics, float2 *dmeans,
                                                    F3 *dconics) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const F3 c = conics[i];
    const F3 s = dconics[i];
    const float2 m = dmeans[i];
    dconics[i] = F3{-0.5f * s.a, -s.b, -0.5f * s.c};
    dmeans[i] = make_float2(-(c.a * m.x + c.b * m.y), -(c.b * m.x + c.c * m.y));
}

__global__ __launch_bounds__(256) void k_zero_f32(float *p, int64_t m) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < m) p[i] = 0.f;
}

template <Mode M, int NB = kBatchFwd>
void launch_fwd(const BlendArgs &a, float *image, float *final_T, int32_t *last, hipStream_t s) {
    const int gx = int(grid_x(a.W));
    const int64_t n_tiles = int64_t(gx) * grid_y(a.H);
    k_blend_fwd<M, NB><<<dim3(unsigned(xcd_grid(n_tiles))), kBlock, 0, s>>>(
        a.W, a.H, gx, n_tiles, reinterpret_cast<const uint2 *>(a.ranges), a.point_list, uint32_t(a.n),
        reinterpret_cast<const float2 *>(a.means2d), reinterpret_cast<const F3 *>(a.conics),
        a.opacity, reinterpret_cast<const F3 *>(a.colors), a.bg[0], a.bg[1], a.bg[2], image,
        final_T, last);
}

template <Mode M, int NB = kBatchBwd>
void launch_bwd(const BlendArgs &a, const float *final_T, const int32_t *last, const float *dimg,
                float *dm, float *dc, float *dop, float *dcol, hipStream_t s) {
    const int gx = int(grid_x(a.W));
    const int64_t n_tiles = int64_t(gx) * grid_y(a.H);
    k_blend_bwd<M, NB><<<dim3(unsigned(xcd_grid(n_tiles))), kBlock, 0, s>>>(
        a.W, a.H, gx, n_tiles, reinterpret_cast<const uint2 *>(a.ranges), a.point_list, uint32_t(a.n),
        reinterpret_cast<const float2 *>(a.means2d), reinterpret_cast<const F3 *>(a.conics),
        a.opacity, reinterpret_cast<const F3 *>(a.colors), a.bg[0], a.bg[1], a.bg[2], final_T,
        last, dimg, dm, dc, dop, dcol);
}

}  // namespace

gsb_status blend_forward(const BlendArgs &a, gsb_precision prec, float *image, float *final_T,
                         int32_t *last, hipStream_t s) {
    switch (prec) {
        case GSB_FP32_PLAIN: launch_fwd<Mode::Plain>(a, image, final_T, last, s); break;
        case GSB_FP16_GEMM: launch_fwd<Mode::F16>(a, image, final_T, last, s); break;
        case GSB_BF16_GEMM: launch_fwd<Mode::BF16>(a, image, final_T, last, s); break;
        default: return fail(GSB_ERR_INVALID, "unknown precision %d", int(prec));
    }
    return check_launch("blend_forward");
}

gsb_status blend_backward(const BlendArgs &a, gsb_precision prec, const float *final_T,
                          const int32_t *last, const float *dimg, float *dm, float *dc,
                          float *dop, float *dcol, hipStream_t s) {
    if (prec != GSB_FP32_PLAIN && prec != GSB_FP16_GEMM && prec != GSB_BF16_GEMM)
        return fail(GSB_ERR_INVALID, "unknown precision %d", int(prec));
    if (a.n > 0) {
        const unsigned zb2 = unsigned((2 * a.n + 255) / 256), zb3 = unsigned((3 * a.n + 255) / 256);
        k_zero_f32<<<zb2, 256, 0, s>>>(dm, 2 * a.n);
        k_zero_f32<<<zb3, 256, 0, s>>>(dc, 3 * a.n);
        k_zero_f32<<<unsigned((a.n + 255) / 256), 256, 0, s>>>(dop, a.n);
        k_zero_f32<<<zb3, 256, 0, s>>>(dcol, 3 * a.n);
    }
    switch (prec) {
        case GSB_FP32_PLAIN: launch_bwd<Mode::Plain>(a, final_T, last, dimg, dm, dc, dop, dcol, s); break;
        case GSB_FP16_GEMM: launch_bwd<Mode::F16>(a, final_T, last, dimg, dm, dc, dop, dcol, s); break;
        default: launch_bwd<Mode::BF16>(a, final_T, last, dimg, dm, dc, dop, dcol, s); break;
    }
    if (a.n > 0)
        k_bwd_finish<<<unsigned((a.n + 255) / 256), 256, 0, s>>>(
            a.n, reinterpret_cast<const F3 *>(a.conics), reinterpret_cast<float2 *>(dm),
            reinterpret_cast<F3 *>(dc));
    return check_launch("blend_backward");
}

}  // namespace gsb
