// Tile binning on the GPU: duplication with tile|depth keys (paper §2.1(b)), depth sort (§2.1(c))
// and per-tile [start, end) ranges of the sorted list (the per-tile index lists that Alg. 1 and
// Alg. 2 consume).
//
// The result is the list of (tile, Gaussian) pairs ordered by (tile, depth, Gaussian index). It is
// produced without ever sorting 64-bit tile|depth keys:
//   1. the Gaussians themselves are sorted by depth (stable LSD radix sort of N 32-bit keys, so
//      equal depths keep increasing index): this fixes every Gaussian's rank in (depth, index);
//   2. pairs are emitted in rank order, each with its tile id as key (16-bit when the grid has at
//      most 65536 tiles, else 32-bit);
//   3. a stable LSD radix sort of the pairs on the tile id alone (ceil(log2 tiles / 8) passes, 2
//      up to 65536 tiles) then leaves each tile's pairs in rank order, i.e. (depth, index) order.
// Against sorting (tile << 32 | depth) pairs directly this moves ~40 instead of ~200 bytes per
// pair. Everything is integer work and bit-exact: the covered-tile rectangle is evaluated in
// integer arithmetic (floor((x - r)/16) == (floor(x) - r) >> 4 for integer r).
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>
#include <utility>

#include "gsb_internal.h"

namespace gsb {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;                           // per thread
constexpr int kScanTile = kScanThreads * kScanItems;     // 4096 elements per block
constexpr int kScanTopThreads = 1024;
constexpr int kScanTopItems = 4;
constexpr int kScanMaxBlocks = kScanTopThreads * kScanTopItems;   // single-block top level
constexpr int64_t kScanMaxLen = int64_t(kScanTile) * kScanMaxBlocks;  // 16.7M elements
constexpr int kScanSmallBlocks = 1;   // arrays of at most one block: the one-block scan (one launch)

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;                           // keys per thread
constexpr int kSortTile = kSortThreads * kSortItems;     // 4096 keys per block
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

constexpr int kBigRect = 32;   // mode 0: rectangles with more tiles are emitted by the whole wavefront

// The tile sort's keys are tile ids: 16-bit when the grid has at most 65536 tiles (a 4096 x 4096
// image), which cuts the bytes of the pair emission, the sort passes and the range pass, and
// 32-bit otherwise. The pair order is the same either way.
constexpr int64_t kMaxTiles16 = int64_t(1) << 16;

// Four consecutive keys [idx, idx + 4) with one vector load (idx a multiple of 4; key buffers are
// 256-byte aligned and padded, so a load that straddles the count stays inside the buffer).
__device__ inline uint4 load4(const uint32_t *k, int64_t idx) {
    return *reinterpret_cast<const uint4 *>(k + idx);
}
__device__ inline uint4 load4(const uint16_t *k, int64_t idx) {
    const uint2 v = *reinterpret_cast<const uint2 *>(k + idx);
    return make_uint4(v.x & 0xffffu, v.x >> 16, v.y & 0xffffu, v.y >> 16);
}


struct BinHeader {
    unsigned long long total;     // pairs counted by bin_count
    unsigned long long pairs;     // min(total, capacity), set by bin_fill
    unsigned long long gaussians; // n, for the depth sort
    uint32_t pad[10];
};

// State of one radix sort: the global digit counts of every pass (from the histogram kernel) and
// the ticket counter from which each pass's blocks draw their tile of keys.
constexpr int kMaxPasses = 4;
struct SortState {
    uint32_t hist[kMaxPasses][kRadix];
    uint32_t ticket[kMaxPasses];
    uint32_t pad[64 - kMaxPasses];
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct Layout {
    // bin_count's part (depends on n only)
    size_t hdr, counts, masks, recs, partials;
    // bin_fill's part
    size_t sorts, dkey_a, dkey_b, dval_a, dval_b, offs, rects, tkey_a, tkey_b, vals_tmp, sortbuf, end;
};

int64_t sort_blocks(int64_t m) { return (m + kSortTile - 1) / kSortTile; }

Layout layout(int64_t n, int64_t cap) {
    Layout L;
    const size_t nn = size_t(n > 0 ? n : 1), cc = size_t(cap > 0 ? cap : 1);
    size_t o = 0;
    L.hdr = o;       o += align256(sizeof(BinHeader));
    L.counts = o;    o += align256(sizeof(unsigned long long) * nn);
    L.masks = o;     o += align256(sizeof(unsigned long long) * nn);
    L.recs = o;      o += align256(sizeof(uint4) * nn);
    L.partials = o;  o += align256(sizeof(unsigned long long) * kScanMaxBlocks);
    L.sorts = o;     o += align256(sizeof(SortState));
    L.dkey_a = o;    o += align256(sizeof(uint32_t) * nn);
    L.dkey_b = o;    o += align256(sizeof(uint32_t) * nn);
    L.dval_a = o;    o += align256(sizeof(uint32_t) * nn);
    L.dval_b = o;    o += align256(sizeof(uint32_t) * nn);
    L.offs = o;      o += align256(sizeof(unsigned long long) * nn);
    L.rects = o;     o += align256(sizeof(unsigned long long) * nn);
    L.tkey_a = o;    o += align256(sizeof(uint32_t) * cc);
    L.tkey_b = o;    o += align256(sizeof(uint32_t) * cc);
    L.vals_tmp = o;  o += align256(sizeof(uint32_t) * cc);
    // depth sort: look-back words of every pass, [pass][block][digit]; tile sort, afterwards:
    // the per-block digit histograms of one pass, [digit][block]
    const int64_t lb_d = int64_t(kMaxPasses) * sort_blocks(n > 0 ? n : 1);
    const int64_t lb_t = sort_blocks(cap > 0 ? cap : 1);
    L.sortbuf = o;   o += align256(sizeof(uint32_t) * kRadix * size_t(lb_d > lb_t ? lb_d : lb_t));
    L.end = o;
    return L;
}

template <typename T>
T *at(void *ws, size_t off) { return reinterpret_cast<T *>(static_cast<char *>(ws) + off); }

// ------------------------------------------------------------------------------- block scan
// Exclusive scan of one value per thread across the block; `total` receives the block sum.
// `s_wave` holds one slot per wavefront.
template <typename T>
__device__ T block_exclusive_scan(T v, T *s_wave, T &total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[w] = x;
    __syncthreads();
    T pre = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        T s = s_wave[i];
        pre += (i < w) ? s : T(0);
        tot += s;
    }
    __syncthreads();
    total = tot;
    return pre + x - v;
}

// ------------------------------------------------------------------------------- device scan
// Exclusive prefix sum, in place. Short arrays: one block walks the array in chunks with a running
// carry. Long arrays: per-block sums, then a per-block scan whose blocks add up the sums before
// them. The total goes to *total_a / *total_b if given (a total-only call scans the per-block
// sums in one block instead).
template <typename T>
__global__ __launch_bounds__(kScanTopThreads) void k_scan_small(T *data, int64_t m,
                                                                unsigned long long *total_a,
                                                                long long *total_b) {
    constexpr int kItems = 16;
    __shared__ T s_wave[kScanTopThreads / 64];
    T carry = 0;
    for (int64_t base = 0; base < m; base += int64_t(kScanTopThreads) * kItems) {
        const int64_t b = base + int64_t(threadIdx.x) * kItems;
        T v[kItems], sum = 0;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            v[k] = (b + k < m) ? data[b + k] : T(0);
            sum += v[k];
        }
        T tot;
        T run = block_exclusive_scan<T>(sum, s_wave, tot) + carry;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (b + k < m) data[b + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        if (total_a) *total_a = (unsigned long long)carry;
        if (total_b) *total_b = (long long)carry;
    }
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const T *in, int64_t m, T *partial) {
    __shared__ T s_wave[kScanThreads / 64];
    const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
    T sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < m) sum += in[base + k];
    T tot;
    block_exclusive_scan<T>(sum, s_wave, tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

template <typename T>
__global__ __launch_bounds__(kScanTopThreads) void k_scan_top(T *partial, int64_t nb,
                                                               unsigned long long *total_a,
                                                               long long *total_b) {
    __shared__ T s_wave[kScanTopThreads / 64];
    const int64_t base = int64_t(threadIdx.x) * kScanTopItems;
    T v[kScanTopItems], sum = 0;
#pragma unroll
    for (int k = 0; k < kScanTopItems; ++k) {
        v[k] = (base + k < nb) ? partial[base + k] : T(0);
        sum += v[k];
    }
    T tot;
    T run = block_exclusive_scan<T>(sum, s_wave, tot);
#pragma unroll
    for (int k = 0; k < kScanTopItems; ++k) {
        if (base + k < nb) partial[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) {
        if (total_a) *total_a = (unsigned long long)tot;
        if (total_b) *total_b = (long long)tot;
    }
}

// The down pass with the block offsets formed in place: block b sums the per-block totals
// partial[0, b) itself (a few hundred values at most, read from L2) instead of a separate
// single-block scan of them, which saves a launch; the last block writes the total.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_down_fused(T *data, int64_t m,
                                                                   const T *partial, int64_t nb,
                                                                   unsigned long long *total_a,
                                                                   long long *total_b) {
    __shared__ T s_wave[kScanThreads / 64];
    const int64_t blk = blockIdx.x;
    T mine = 0;
    for (int64_t i = threadIdx.x; i < blk; i += kScanThreads) mine += partial[i];
    T offset;
    block_exclusive_scan<T>(mine, s_wave, offset);       // offset = sum of partial[0, blk)
    const int64_t base = blk * kScanTile + int64_t(threadIdx.x) * kScanItems;
    T v[kScanItems], sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < m) ? data[base + k] : T(0);
        sum += v[k];
    }
    T tot;
    T run = block_exclusive_scan<T>(sum, s_wave, tot) + offset;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < m) data[base + k] = run;
        run += v[k];
    }
    if (blk == nb - 1 && threadIdx.x == 0) {
        if (total_a) *total_a = (unsigned long long)(offset + tot);
        if (total_b) *total_b = (long long)(offset + tot);
    }
}

// scan (down = true) or total only (down = false)
template <typename T>
void launch_scan(T *data, int64_t m, T *partial, unsigned long long *total_a, long long *total_b,
                 hipStream_t s, bool down = true) {
    const int64_t nb = (m + kScanTile - 1) / kScanTile;
    if (down && nb <= kScanSmallBlocks) {
        k_scan_small<T><<<1, kScanTopThreads, 0, s>>>(data, m, total_a, total_b);
        return;
    }
    if (nb > 0) k_scan_reduce<T><<<dim3(unsigned(nb)), kScanThreads, 0, s>>>(data, m, partial);
    if (down)
        k_scan_down_fused<T><<<dim3(unsigned(nb)), kScanThreads, 0, s>>>(data, m, partial, nb,
                                                                          total_a, total_b);
    else
        k_scan_top<T><<<1, kScanTopThreads, 0, s>>>(partial, nb, total_a, total_b);
}

// ------------------------------------------------------------------------------- mode 1
// Binning mode 1 keeps a pair (tile, Gaussian) of the 3-sigma rectangle only when the Gaussian can
// reach alpha >= 1/255 on a pixel of the tile inside the image (opacity-aware extent, a tighter
// binning; images and final T are unchanged because every dropped pair would be skipped):
//   o >= fp32(1/255), and min over the tile's pixel rectangle of Q = d^T Sigma^-1 d <= theta,
//   theta = 2 (e * ln2_up + (m - 1)) + 0.1 with 255 o = m 2^e, m in [1, 2)
// (an upper bound of 2 ln(255 o) without a logarithm, plus a margin far above any exponent error
// of the blend). The minimum of Q over the rectangle of d = (x - px, y - py) is 0 if the rectangle
// contains 0, else it lies on an edge: a 1D quadratic minimised inside the edge or at an end.
// Division-free double-precision tests in a fixed order with contraction off: the decision is
// reproducible bit for bit by any implementation taking the same steps.
constexpr double kLn2Up = 0x1.62e42fefa39fp-1;   // the double just above ln 2
constexpr double kCullMargin = 0.1;

__device__ inline double vis_theta(double o) {
#pragma clang fp contract(off)
    const double z = 255.0 * o;                   // exact: o is an fp32 value
    const unsigned long long bits = (unsigned long long)__double_as_longlong(z);
    const long long e = (long long)((bits >> 52) & 0x7ffull) - 1023;
    const double m = __longlong_as_double(
        (long long)((bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull));
    const double t1 = double(e) * kLn2Up;
    const double t2 = m - 1.0;
    return 2.0 * (t1 + t2) + kCullMargin;
}

// one edge: u fixed at a, v in [c, d]; Q = P a^2 + 2 B a v + R v^2
__device__ inline bool vis_edge(double P, double R, double B, double det, double theta, double a,
                                double c, double d) {
#pragma clang fp contract(off)
    const double ba = B * a;
    const double nba = -ba;
    if (c * R <= nba && nba <= d * R) {           // interior minimum a^2 det / R
        const double lhs = (a * a) * det;
        const double rhs = theta * R;
        return lhs <= rhs;
    }
    const double pa2 = P * (a * a);
    const double qc = (pa2 + (2.0 * ba) * c) + R * (c * c);
    const double qd = (pa2 + (2.0 * ba) * d) + R * (d * d);
    return qc <= theta || qd <= theta;
}

struct GaussVis {
    double x, y, A, B, C, det, theta;
    // Shortcuts that settle most tiles with the same answer as the tests below: with d the point
    // of the tile's rectangle nearest the mean, lmin |d|^2 <= min Q <= Q(d) <= lmax |d|^2 (lmin,
    // lmax the eigenvalues of Sigma^-1). Beyond margins far above the tests' rounding:
    //   |d|^2 > far  => invisible,   |d|^2 < near => visible.
    double far2, near2;
    bool live;                                    // o >= fp32(1/255)
};

__device__ inline GaussVis vis_setup(float2 m, const float *conic, float o) {
#pragma clang fp contract(off)
    GaussVis g;
    g.x = m.x; g.y = m.y;
    g.A = conic[0]; g.B = conic[1]; g.C = conic[2];
    g.live = o >= 1.0f / 255.0f;
    g.det = g.A * g.C - g.B * g.B;
    g.theta = vis_theta(double(o));
    g.far2 = INFINITY;                            // no shortcut unless positive definite
    g.near2 = -1.0;
    if (g.A > 0.0 && g.det > 0.0) {
        const double h = 0.5 * (g.A + g.C), r = sqrt(0.25 * (g.A - g.C) * (g.A - g.C) + g.B * g.B);
        const double lmax = (h + r) * (1.0 + 1e-9);
        const double lmin = (g.det / (h + r)) * (1.0 - 1e-9);
        g.far2 = (g.theta + 1e-6 * (1.0 + g.theta)) / lmin;
        g.near2 = (g.theta - 1e-6 * (1.0 + g.theta)) / lmax;
    }
    return g;
}

__device__ inline bool tile_visible(const GaussVis &g, int32_t tx, int32_t ty, int32_t W,
                                    int32_t H) {
#pragma clang fp contract(off)
    if (!g.live) return false;
    const int32_t px1 = tx * kTile + kTile - 1 < W - 1 ? tx * kTile + kTile - 1 : W - 1;
    const int32_t py1 = ty * kTile + kTile - 1 < H - 1 ? ty * kTile + kTile - 1 : H - 1;
    const double dxl = g.x - double(px1), dxh = g.x - double(tx * kTile);
    const double dyl = g.y - double(py1), dyh = g.y - double(ty * kTile);
    if (dxl <= 0.0 && 0.0 <= dxh && dyl <= 0.0 && 0.0 <= dyh) return true;
    const double cx = dxl > 0.0 ? dxl : (dxh < 0.0 ? dxh : 0.0);
    const double cy = dyl > 0.0 ? dyl : (dyh < 0.0 ? dyh : 0.0);
    const double d2 = cx * cx + cy * cy;
    if (d2 > g.far2) return false;
    if (d2 < g.near2) return true;
    // only the edges facing the mean can hold the minimum (at most one in x, one in y)
    if (dxl > 0.0 && vis_edge(g.A, g.C, g.B, g.det, g.theta, dxl, dyl, dyh)) return true;
    if (dxh < 0.0 && vis_edge(g.A, g.C, g.B, g.det, g.theta, dxh, dyl, dyh)) return true;
    if (dyl > 0.0 && vis_edge(g.C, g.A, g.B, g.det, g.theta, dyl, dxl, dxh)) return true;
    if (dyh < 0.0 && vis_edge(g.C, g.A, g.B, g.det, g.theta, dyh, dxl, dxh)) return true;
    return false;
}

// The candidate tiles of mode 1: the 3-sigma rectangle cut to the tiles that the bounding box of
// {Q <= theta} (half-widths sqrt(theta C / det), sqrt(theta A / det), plus one pixel) can reach.
// Every tile cut away has Q > theta on all its pixels by a wide margin, so the tests above would
// reject it: the cut changes which tiles are tested, never a decision. Empty when o < 1/255.
__device__ inline Rect cand_rect(const GaussVis &g, const Rect &R) {
    if (!g.live) return Rect{0, 0, 0, 0};
    if (!(g.A > 0.0 && g.C > 0.0 && g.det > 0.0)) return R;
    const double hx = fmin(sqrt(g.theta * g.C / g.det) + 1.0, 1e8);
    const double hy = fmin(sqrt(g.theta * g.A / g.det) + 1.0, 1e8);
    Rect C = R;
    const int64_t bx0 = int64_t(floor((g.x - hx - 15.0) / 16.0)), bx1 = int64_t(floor((g.x + hx) / 16.0)) + 1;
    const int64_t by0 = int64_t(floor((g.y - hy - 15.0) / 16.0)), by1 = int64_t(floor((g.y + hy) / 16.0)) + 1;
    if (bx0 > C.tx0) C.tx0 = int32_t(bx0 < C.tx1 ? bx0 : C.tx1);
    if (bx1 < C.tx1) C.tx1 = int32_t(bx1 > C.tx0 ? bx1 : C.tx0);
    if (by0 > C.ty0) C.ty0 = int32_t(by0 < C.ty1 ? by0 : C.ty1);
    if (by1 < C.ty1) C.ty1 = int32_t(by1 > C.ty0 ? by1 : C.ty0);
    return C;
}

// visible-tile masks: a Gaussian with at most this many candidates keeps its answer as one bit per
// candidate (row-major), so that emission needs no second test
constexpr uint32_t kMaskBits = 64;

// ------------------------------------------------------------------------------- balanced pairs
// The candidate tiles of a wavefront's 64 rectangles are enumerated in chunks of 64, one candidate
// per lane, whatever the rectangles' sizes: a candidate's rectangle (its owner lane) is found by a
// binary search over the wavefront's exclusive prefix of areas, and the tile from the index within
// that rectangle (row-major). Owners' visibility parameters sit in LDS.
struct WaveCands {
    uint32_t excl;     // this lane's exclusive prefix of areas
    uint32_t total;    // the wavefront's number of candidates
};

__device__ inline WaveCands wave_cands(uint32_t area) {
    const int lane = threadIdx.x & 63;
    uint32_t x = area;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return WaveCands{x - area, uint32_t(__shfl(x, 63, 64))};
}

// the lane owning candidate k: the last lane whose exclusive prefix is <= k
__device__ inline int cand_owner(uint32_t excl, uint32_t k) {
    int o = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1)
        if (uint32_t(__shfl(int(excl), o + step, 64)) <= k) o += step;
    return o;
}

// a / b and a % b for a < 2^25, 0 < b < 2^13: a float quotient (error < 8) corrected exactly
__device__ inline void divmod_small(uint32_t a, uint32_t b, uint32_t &q, uint32_t &r) {
    uint32_t qq = uint32_t(float(a) * __builtin_amdgcn_rcpf(float(b)));
    int32_t rr = int32_t(a) - int32_t(qq * b);
    while (rr < 0) { --qq; rr += int32_t(b); }
    while (rr >= int32_t(b)) { ++qq; rr -= int32_t(b); }
    q = qq;
    r = uint32_t(rr);
}

// lanes [s, e) of a 64-bit lane mask (0 <= s <= e <= 64)
__device__ inline unsigned long long lane_range(int s, int e) {
    const unsigned long long hi = e >= 64 ? ~0ull : ((1ull << e) - 1ull);
    const unsigned long long lo = s >= 64 ? ~0ull : ((1ull << s) - 1ull);
    return hi & ~lo;
}

// candidates of owner lane l that fall in the chunk [cb, cb + 64)
__device__ inline unsigned long long owner_run(uint32_t excl, uint32_t area, uint32_t cb) {
    const int64_t s0 = int64_t(excl) - int64_t(cb), e0 = s0 + int64_t(area);
    const int s = int(s0 < 0 ? 0 : (s0 > 64 ? 64 : s0)), e = int(e0 < 0 ? 0 : (e0 > 64 ? 64 : e0));
    return lane_range(s, e);
}

// Pair counts per Gaussian. Mode 0: the rectangle's area. Mode 1: its visible candidates, with
// the candidates of each wavefront balanced over its lanes; a Gaussian with at most kMaskBits
// candidates also records which ones are visible (masks).
// A Gaussian's pair count and emission rectangle in one 16-byte record, stored by Gaussian index:
// the depth sort's last pass gathers both with one load and lays them out in rank order, so that
// the pair emission reads them in order instead of gathering means and radii by rank. Tile
// coordinates are at most 4096 and fit 16 bits.
__device__ inline uint4 count_rect(unsigned long long cnt, const Rect &R) {
    return make_uint4(uint32_t(cnt), uint32_t(cnt >> 32), uint32_t(R.tx0) | (uint32_t(R.tx1) << 16),
                      uint32_t(R.ty0) | (uint32_t(R.ty1) << 16));
}
__device__ inline Rect unpack_rect(unsigned long long p) {
    const uint32_t x = uint32_t(p), y = uint32_t(p >> 32);
    return Rect{int32_t(x & 0xffffu), int32_t(x >> 16), int32_t(y & 0xffffu), int32_t(y >> 16)};
}

__global__ __launch_bounds__(256) void k_bin_count(const float2 *means, const int32_t *radii,
                                                   const float *conics, const float *opac,
                                                   int32_t mode, int64_t n, int32_t gx,
                                                   int32_t gy, int32_t W, int32_t H,
                                                   unsigned long long *counts,
                                                   unsigned long long *masks, uint4 *recs) {
    __shared__ GaussVis s_vis[256];
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (mode == 0) {
        if (i >= n) return;
        const float2 m = means[i];
        const Rect R = tile_rect(m.x, m.y, radii[i], gx, gy);
        const unsigned long long cnt =
            (unsigned long long)(R.tx1 - R.tx0) * (unsigned long long)(R.ty1 - R.ty0);
        counts[i] = cnt;
        recs[i] = count_rect(cnt, R);
        return;
    }
    if (int64_t(blockIdx.x) * blockDim.x >= n) return;   // block-uniform
    const bool valid = i < n;
    Rect CR{0, 0, 0, 0};
    GaussVis g{};
    if (valid) {
        const float2 m = means[i];
        g = vis_setup(m, conics + 3 * i, opac[i]);
        CR = cand_rect(g, tile_rect(m.x, m.y, radii[i], gx, gy));
    }
    s_vis[threadIdx.x] = g;   // read only by this wavefront's lanes
    __builtin_amdgcn_wave_barrier();
    const int w = CR.tx1 - CR.tx0;
    const uint32_t area = uint32_t(w * (CR.ty1 - CR.ty0));
    const WaveCands wc = wave_cands(area);
    const int lane = threadIdx.x & 63, wbase = threadIdx.x & ~63;
    unsigned long long cnt = 0, mask = 0;
    for (uint32_t cb = 0; cb < wc.total; cb += 64) {
        const uint32_t k = cb + lane;
        const bool act = k < wc.total;
        const int o = cand_owner(wc.excl, act ? k : wc.total - 1);
        const uint32_t jl = (act ? k : 0u) - uint32_t(__shfl(int(wc.excl), o, 64));
        const int ow = __shfl(w, o, 64), otx0 = __shfl(CR.tx0, o, 64), oty0 = __shfl(CR.ty0, o, 64);
        uint32_t qy = 0, rx = 0;
        if (act) divmod_small(jl, uint32_t(ow), qy, rx);
        bool v = false;
        if (act) v = tile_visible(s_vis[wbase + o], otx0 + int(rx), oty0 + int(qy), W, H);
        // as an owner: my candidates in this chunk are lanes [rs, re)
        const unsigned long long mine = __ballot(v) & owner_run(wc.excl, area, cb);
        cnt += __popcll(mine);
        if (area <= kMaskBits && mine) {
            const int64_t rs = int64_t(wc.excl) - int64_t(cb);
            const int s0 = rs > 0 ? int(rs) : 0;
            const int j0 = rs > 0 ? 0 : int(-rs);      // my first candidate index in this chunk
            mask |= (mine >> s0) << j0;
        }
    }
    if (valid) {
        counts[i] = cnt;
        masks[i] = mask;
        recs[i] = count_rect(cnt, CR);
    }
}

// Depth keys: the float's bits, made order-preserving for any sign (a no-op flip of the sign bit
// for the positive depths of the contract).
__device__ inline uint32_t depth_key(float d) {
    const uint32_t b = __float_as_uint(d);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Emits the pairs of the Gaussian of rank j at offs[j]: tile id as key, Gaussian index as value.
// The block's 256 consecutive ranks own one contiguous output segment; when it fits in LDS the
// pairs are assembled there and written out in order (coalesced), otherwise straight to memory.
// A lane emits its own rectangle when it is small; larger ones are emitted by the whole wavefront
// together, one after the other.
// Pairs staged per block: 4096, or 6144 where a block's 256 ranks are expected to emit more than
// 7/8 of 4096 (the host estimates it from the capacity per Gaussian). Blocks whose segment does
// not fit write straight to memory, uncoalesced: at 4K 82% of the blocks overflow 4096 (binning
// 1.211 -> 1.151 ms with 6144), while at 1080p the larger stage only costs occupancy.
constexpr int kFillStage = 4096, kFillStageLarge = 6144;

template <typename K, int kStage> struct PairSink {
    K *keys;                         // global
    uint32_t *vals;
    K *skey;                         // LDS segment, or null
    uint32_t *sval;
    unsigned long long seg0, cap;    // first output index of the block, capacity
    __device__ inline void put(unsigned long long o, uint32_t key, uint32_t val) const {
        if (skey) {
            if (o - seg0 >= (unsigned long long)kStage) return;   // never for consistent counts
            skey[o - seg0] = K(key);
            sval[o - seg0] = val;
        } else if (o < cap) {
            keys[o] = K(key);
            vals[o] = val;
        }
    }
};

template <typename K, int kStage>
__global__ __launch_bounds__(256) void k_bin_fill(const float2 *means, const float *conics,
                                                  const float *opac,
                                                  int32_t mode, int32_t W, int32_t H,
                                                  const uint32_t *sorted_idx, int64_t n,
                                                  int32_t gx, int32_t gy,
                                                  const unsigned long long *offs,
                                                  const unsigned long long *counts,
                                                  const unsigned long long *masks,
                                                  const unsigned long long *rank_rects,
                                                  BinHeader *hdr, int64_t cap, K *keys,
                                                  uint32_t *vals, int32_t *status) {
    __shared__ K s_key[kStage];
    __shared__ uint32_t s_val[kStage];
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j == 0) {
        const unsigned long long total = hdr->total;
        hdr->pairs = total < (unsigned long long)cap ? total : (unsigned long long)cap;
        if (total > (unsigned long long)cap) *status = GSB_ERR_CAPACITY;
    }
    const int64_t j0 = int64_t(blockIdx.x) * blockDim.x;
    if (j0 >= n) return;   // block-uniform (only the single block of an empty launch)
    const bool valid = j < n;
    const uint32_t i = valid ? sorted_idx[j] : 0u;
    // the rectangle to emit from (laid out in rank order by the depth sort): mode 0 the 3-sigma
    // one, mode 1 the candidates (cand_rect)
    Rect R{0, 0, 0, 0};
    GaussVis g{};
    unsigned long long base = 0, vmask = 0;
    if (valid) {
        R = unpack_rect(rank_rects[j]);
        base = offs[j];
        if (mode != 0) {
            g = vis_setup(means[i], conics + 3 * int64_t(i), opac[i]);
            vmask = masks[i];
        }
    }
    // the block's segment: [first rank's offset, last rank's offset + its count)
    const int64_t jl = (j0 + int64_t(blockDim.x) < n ? j0 + int64_t(blockDim.x) : n) - 1;
    const unsigned long long seg0 = offs[j0];
    const unsigned long long seg1 = offs[jl] + counts[sorted_idx[jl]];
    const unsigned long long ucap = (unsigned long long)cap;
    const bool staged = (seg1 - seg0) <= (unsigned long long)kStage && seg1 <= ucap;
    const PairSink<K, kStage> sink{keys, vals, staged ? s_key : nullptr, staged ? s_val : nullptr,
                                   seg0, ucap};

    const int w = R.tx1 - R.tx0;
    const int area = w * (R.ty1 - R.ty0);
    // small rectangles: the lane emits its own (mode 1: the recorded visible candidates); large
    // ones: the whole wavefront together, one after the other (mode 1: testing each candidate)
    const bool big = mode == 0 ? area > kBigRect : area > int(kMaskBits);
    if (!big) {
        unsigned long long o = base;
        if (mode == 0) {
            for (int32_t ty = R.ty0; ty < R.ty1; ++ty)
                for (int32_t tx = R.tx0; tx < R.tx1; ++tx, ++o)
                    sink.put(o, uint32_t(int64_t(ty) * gx + tx), i);
        } else {
            // row by row: bits [r w, r w + w) of the mask are row r of the candidates
            const unsigned long long rowm = w >= 64 ? ~0ull : ((1ull << w) - 1ull);
            for (int32_t ty = R.ty0, sh = 0; ty < R.ty1; ++ty, sh += w) {
                for (unsigned long long mk = (vmask >> sh) & rowm; mk; mk &= mk - 1, ++o) {
                    const int bx = __ffsll((long long)mk) - 1;
                    sink.put(o, uint32_t(int64_t(ty) * gx + (R.tx0 + bx)), i);
                }
            }
        }
    }
    unsigned long long todo = __ballot(big);
    const int lane = threadIdx.x & 63;
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
    while (todo) {
        const int src = __ffsll((long long)todo) - 1;
        todo &= todo - 1;
        const int stx0 = __builtin_amdgcn_readlane(R.tx0, src);
        const int sty0 = __builtin_amdgcn_readlane(R.ty0, src);
        const int sw = __builtin_amdgcn_readlane(w, src);
        const int sarea = __builtin_amdgcn_readlane(area, src);
        const uint32_t si = __builtin_amdgcn_readlane(i, src);
        const unsigned long long sbase =
            ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane(uint32_t(base >> 32), src) << 32) |
            (uint32_t)__builtin_amdgcn_readlane(uint32_t(base), src);
        if (mode == 0) {
            for (int k = lane; k < sarea; k += 64) {
                const int ty = sty0 + k / sw, tx = stx0 + k % sw;
                sink.put(sbase + k, uint32_t(int64_t(ty) * gx + tx), si);
            }
        } else {
            GaussVis sg;
            sg.x = __shfl(g.x, src); sg.y = __shfl(g.y, src);
            sg.A = __shfl(g.A, src); sg.B = __shfl(g.B, src); sg.C = __shfl(g.C, src);
            sg.det = __shfl(g.det, src); sg.theta = __shfl(g.theta, src);
            sg.far2 = __shfl(g.far2, src); sg.near2 = __shfl(g.near2, src);
            sg.live = true;
            unsigned long long o = sbase;       // visible candidates in row-major order
            for (int k0 = 0; k0 < sarea; k0 += 64) {
                const int k = k0 + lane;
                const int ty = sty0 + k / sw, tx = stx0 + k % sw;
                const bool v = k < sarea && tile_visible(sg, tx, ty, W, H);
                const unsigned long long vb = __ballot(v);
                if (v) sink.put(o + __popcll(vb & lt_mask), uint32_t(int64_t(ty) * gx + tx), si);
                o += __popcll(vb);
            }
        }
    }
    if (staged) {   // block-uniform
        __syncthreads();
        const int len = int(seg1 - seg0);
        for (int k = threadIdx.x; k < len; k += blockDim.x) {
            keys[seg0 + k] = s_key[k];
            vals[seg0 + k] = s_val[k];
        }
    }
}

// ------------------------------------------------------------------------------- radix sort
// Stable LSD radix sort of (key, u32 value) on 8-bit digits. The depth sort (u32 keys) takes one
// kernel per pass plus one histogram kernel per sort (a "onesweep" organisation with decoupled
// look-back):
//   * k_sort_hist reads the keys once and accumulates the global digit counts of every pass (at
//     most 256 blocks, so few blocks add into each global count); it also clears the look-back
//     words of every pass.
//   * k_radix_pass<chained>, one launch per pass: each block draws the index of its tile of 4096 keys from
//     a ticket counter (so a block only ever waits on tiles whose blocks are already running),
//     ranks its keys stably in LDS, publishes its per-digit counts, and walks back over the
//     preceding tiles' published words (16 per step) until it meets an inclusive prefix. A digit's global
//     start is the exclusive scan of the pass's digit counts plus that prefix. Keys are then
//     written out in digit order (contiguous runs, so the global writes coalesce).
// The tile sort (u16 or u32 keys, see sort_tiles) runs each pass as a per-block histogram, its
// scan and k_radix_pass<unchained>, which reads its digit offsets instead of looking back.
// A look-back word is flag << 30 | value: flag 1 = the tile's own count, 2 = inclusive prefix.
// Every wait is bounded; an expired wait reports GSB_ERR_INTERNAL in the status word instead of
// hanging. The element count is read from device memory (*count).
constexpr uint32_t kFlagAgg = 1u << 30, kFlagInc = 2u << 30, kValMask = (1u << 30) - 1u;
constexpr uint32_t kSpinLimit = 1u << 22;
constexpr int kLookback = 16;           // preceding tiles read per look-back step
constexpr int kHistBlocks = 256;        // histogram kernel: at most this many blocks

__global__ void k_zero_u32(uint32_t *p, int64_t m) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < m) p[i] = 0u;
}

// kDepth: the keys are made here from the depths (and written with the identity values);
// otherwise they are read from keys_io.
template <bool kDepth>
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const float *depths, uint32_t *keys_io,
                                                            uint32_t *vals_out,
                                                            const unsigned long long *count,
                                                            int passes, SortState *st,
                                                            uint32_t *lookback, int64_t nblk) {
    __shared__ uint32_t s_h[kMaxPasses][kRadix];
    const int t = threadIdx.x;
    for (int p = 0; p < passes; ++p) s_h[p][t] = 0u;
    // this block's tiles: blockIdx.x, + gridDim.x, ... (their look-back words are cleared here)
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x)
        for (int p = 0; p < passes; ++p) lookback[(int64_t(p) * nblk + b) * kRadix + t] = 0u;
    __syncthreads();
    const int64_t P = int64_t(*count);
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int64_t base = b * kSortTile;
        if (base >= P) break;
        // four consecutive entries per thread and step: the keys and identity values are stored
        // with 16-byte writes (the workspace buffers are 256-byte aligned)
#pragma unroll
        for (int k = 0; k < kSortItems / 4; ++k) {
            const int64_t idx = base + 4 * (int64_t(k) * kSortThreads + t);
            if (idx >= P) continue;
            uint32_t key[4];
            if constexpr (kDepth) {
#pragma unroll
                for (int j = 0; j < 4; ++j) key[j] = idx + j < P ? depth_key(depths[idx + j]) : 0u;
                if (idx + 4 <= P) {
                    *reinterpret_cast<uint4 *>(keys_io + idx) = make_uint4(key[0], key[1], key[2], key[3]);
                    const uint32_t i0 = uint32_t(idx);
                    *reinterpret_cast<uint4 *>(vals_out + idx) = make_uint4(i0, i0 + 1, i0 + 2, i0 + 3);
                } else {
                    for (int j = 0; idx + j < P; ++j) {
                        keys_io[idx + j] = key[j];
                        vals_out[idx + j] = uint32_t(idx + j);
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) key[j] = idx + j < P ? keys_io[idx + j] : 0u;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (idx + j >= P) break;
                for (int p = 0; p < passes; ++p)
                    atomicAdd(&s_h[p][(key[j] >> (kRadixBits * p)) & (kRadix - 1)], 1u);
            }
        }
    }
    __syncthreads();
    for (int p = 0; p < passes; ++p)
        if (s_h[p][t]) atomicAdd(&st->hist[p][t], s_h[p][t]);
}

// Per-block digit histogram of one pass, stored digit-major ([digit][block]) so that one
// exclusive scan yields every block's output offset per digit.
template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_block_hist(const K *keys,
                                                             const unsigned long long *count,
                                                             int shift, uint32_t *hist,
                                                             int64_t nblk) {
    __shared__ uint32_t s_h[kRadix];
    const int t = threadIdx.x;
    s_h[t] = 0;
    __syncthreads();
    const int64_t P = int64_t(*count);
    const int64_t base = int64_t(blockIdx.x) * kSortTile;
    // four keys per load (order does not matter to a histogram), all loads issued before any is
    // counted (from index 0 where past P: entries >= P are ignored)
    uint4 q[kSortItems / 4];
#pragma unroll
    for (int k = 0; k < kSortItems / 4; ++k) {
        const int64_t idx = base + 4 * (int64_t(k) * kSortThreads + t);
        q[k] = load4(keys, idx < P ? idx : 0);
    }
#pragma unroll
    for (int k = 0; k < kSortItems / 4; ++k) {
        const int64_t idx = base + 4 * (int64_t(k) * kSortThreads + t);
        if (idx < P) {
            const uint4 v = q[k];
            atomicAdd(&s_h[(v.x >> shift) & (kRadix - 1)], 1u);
            if (idx + 1 < P) atomicAdd(&s_h[(v.y >> shift) & (kRadix - 1)], 1u);
            if (idx + 2 < P) atomicAdd(&s_h[(v.z >> shift) & (kRadix - 1)], 1u);
            if (idx + 3 < P) atomicAdd(&s_h[(v.w >> shift) & (kRadix - 1)], 1u);
        }
    }
    __syncthreads();
    hist[int64_t(t) * nblk + blockIdx.x] = s_h[t];
}

__device__ inline void lb_publish(uint32_t *w, uint32_t v) {
    __hip_atomic_store(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t lb_read(const uint32_t *w) {
    return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// kRankCounts (last pass of the depth sort): also writes, at each Gaussian's rank, the number of
// pairs it emits and its emission rectangle (from the record recs_by_idx[value]) into
// rank_counts and rank_rects.
// kChained: the block's tile comes from `ticket` and its digit offsets from the look-back over
// `lookback` plus the pass's digit counts `ghist`; otherwise tile = blockIdx.x and the offsets are
// read from `hist_off` ([digit][block], the exclusive scan of the per-block histograms).
template <bool kChained, bool kRankCounts, typename K = uint32_t>
__global__ __launch_bounds__(kSortThreads) void k_radix_pass(
    const K *kin, const uint32_t *vin, K *kout, uint32_t *vout,
    const unsigned long long *count, int shift, const uint32_t *ghist, uint32_t *lookback,
    uint32_t *ticket, int32_t *status, const uint32_t *hist_off, int64_t nblk,
    const uint4 *recs_by_idx, unsigned long long *rank_counts, unsigned long long *rank_rects) {
    __shared__ uint32_t s_wcnt[kSortThreads / 64][kRadix];  // per-wave digit counts, then prefixes
    __shared__ uint32_t s_dstart[kRadix];                     // block-local start of each digit
    __shared__ uint32_t s_gofs[kRadix];                       // global start of each digit
    __shared__ uint32_t s_wave[kSortThreads / 64];
    __shared__ K s_key[kSortTile];
    __shared__ uint32_t s_val[kSortTile];
    __shared__ uint32_t s_tile;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (kChained && t == 0) s_tile = atomicAdd(ticket, 1u);
#pragma unroll
    for (int d = 0; d < kSortThreads / 64; ++d) s_wcnt[d][t] = 0;
    __syncthreads();
    const int64_t tile = kChained ? int64_t(s_tile) : int64_t(blockIdx.x);
    const int64_t P = int64_t(*count);
    const int64_t base = tile * kSortTile;
    if (base >= P) return;   // block-uniform; every later ticket is empty too

    // Wave w ranks keys [base + 1024 w, base + 1024 (w + 1)) in 16 steps of 64 consecutive keys,
    // so rank order within the wave is index order. All loads are issued first, from an index
    // clamped into [base, P) (validity applied afterwards), so that they are in flight together.
    uint32_t key[kSortItems], val[kSortItems], loc[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = base + int64_t(w) * (kSortItems * 64) + k * 64 + lane;
        const int64_t ci = idx < P ? idx : P - 1;   // P > base here
        key[k] = uint32_t(kin[ci]);
        val[k] = vin[ci];
    }
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = base + int64_t(w) * (kSortItems * 64) + k * 64 + lane;
        const bool valid = idx < P;
        const uint32_t d = (key[k] >> shift) & (kRadix - 1);
        // lanes holding the same digit: intersect, over the digit's bits, the lanes whose bit
        // equals this lane's (the ballot of the set bits, flipped where this lane's bit is clear),
        // on the two 32-bit halves of the mask
        const unsigned long long vmask = __builtin_amdgcn_ballot_w64(valid);
        uint32_t plo = uint32_t(vmask), phi = uint32_t(vmask >> 32);
        const uint32_t nd = ~d;
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const uint32_t flip = uint32_t(int32_t(nd << (31 - b)) >> 31);  // ones if bit b clear
            const unsigned long long vote = __builtin_amdgcn_ballot_w64(flip == 0u);
            plo &= uint32_t(vote) ^ flip;
            phi &= uint32_t(vote >> 32) ^ flip;
        }
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi(phi, __builtin_amdgcn_mbcnt_lo(plo, 0u));
        uint32_t prior = 0;
        if (valid) prior = s_wcnt[w][d];
        if (valid && rank == 0) s_wcnt[w][d] = prior + uint32_t(__popc(plo) + __popc(phi));
        loc[k] = prior + rank;
    }
    __syncthreads();
    // thread t = digit t: exclusive prefix over waves, then the tile's count of digit t
    uint32_t c[kSortThreads / 64], run = 0;
#pragma unroll
    for (int i = 0; i < kSortThreads / 64; ++i) {
        c[i] = s_wcnt[i][t];
        s_wcnt[i][t] = run;
        run += c[i];
    }
    uint32_t excl = 0;
    uint32_t *my = kChained ? lookback + tile * kRadix + t : nullptr;
    if (kChained) lb_publish(my, (tile == 0 ? kFlagInc : kFlagAgg) | run);
    if (kChained && tile > 0) {
        // walk back over the preceding tiles kLookback at a time (independent loads), summing
        // their counts up to the first inclusive prefix; a tile that has published nothing yet is
        // waited for
        int64_t j = tile - 1;
        uint32_t spins = 0;
        bool done = false;
        while (!done) {
            uint32_t wv[kLookback];
#pragma unroll
            for (int k = 0; k < kLookback; ++k)
                wv[k] = (j - k >= 0) ? lb_read(lookback + (j - k) * kRadix + t) : kFlagInc;
            int k = 0;
            for (; k < kLookback; ++k) {
                const uint32_t flag = wv[k] & ~kValMask;
                if (flag == 0u) break;              // not published yet: re-read from here
                excl += wv[k] & kValMask;
                if (flag == kFlagInc) { done = true; break; }
            }
            if (done) break;
            j -= k;
            if (k < kLookback) {
                if (++spins > kSpinLimit) {         // never expected: report instead of hanging
                    *status = GSB_ERR_INTERNAL;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        lb_publish(my, kFlagInc | (excl + run));
    }
    uint32_t tot;
    if constexpr (kChained) {
        const uint32_t dglob = block_exclusive_scan<uint32_t>(ghist[t], s_wave, tot);
        s_gofs[t] = dglob + excl;
    } else {
        s_gofs[t] = hist_off[int64_t(t) * nblk + tile];
    }
    s_dstart[t] = block_exclusive_scan<uint32_t>(run, s_wave, tot);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = base + int64_t(w) * (kSortItems * 64) + k * 64 + lane;
        if (idx < P) {
            const uint32_t d = (key[k] >> shift) & (kRadix - 1);
            const uint32_t r = s_dstart[d] + s_wcnt[w][d] + loc[k];
            s_key[r] = K(key[k]);
            s_val[r] = val[k];
        }
    }
    __syncthreads();
    const int64_t nvalid = (P - base) < kSortTile ? (P - base) : kSortTile;
    for (int64_t j = t; j < nvalid; j += kSortThreads) {
        const K k = s_key[j];
        const uint32_t d = (uint32_t(k) >> shift) & (kRadix - 1);
        const int64_t pos = int64_t(s_gofs[d]) + (j - int64_t(s_dstart[d]));
        kout[pos] = k;
        vout[pos] = s_val[j];
        if constexpr (kRankCounts) {
            const uint4 r = recs_by_idx[s_val[j]];
            rank_counts[pos] = (static_cast<unsigned long long>(r.y) << 32) | r.x;
            rank_rects[pos] = (static_cast<unsigned long long>(r.w) << 32) | r.z;
        }
    }
}

// Depth sort of the n Gaussians (count on the device): keys made from `depths`, values the
// indices, 4 chained passes; the last one also writes each Gaussian's pair count at its rank
// (rank_counts). The sorted indices end in va (4 passes, an even number).
void sort_depth(const float *depths, uint32_t *ka, uint32_t *kb, uint32_t *va, uint32_t *vb,
                const unsigned long long *count, int64_t n, SortState *st, uint32_t *lookback,
                int32_t *status, const uint4 *recs_by_idx, unsigned long long *rank_counts,
                unsigned long long *rank_rects, hipStream_t s) {
    constexpr int passes = 32 / kRadixBits;
    const int64_t nblk = sort_blocks(n);
    if (nblk == 0) return;
    const int64_t hb = nblk < kHistBlocks ? nblk : kHistBlocks;
    k_sort_hist<true><<<dim3(unsigned(hb)), kSortThreads, 0, s>>>(depths, ka, va, count, passes,
                                                                  st, lookback, nblk);
    uint32_t *kin = ka, *kout = kb, *vin = va, *vout = vb;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * kRadixBits;
        uint32_t *lb = lookback + int64_t(p) * nblk * kRadix;
        if (p == passes - 1)
            k_radix_pass<true, true><<<dim3(unsigned(nblk)), kSortThreads, 0, s>>>(
                kin, vin, kout, vout, count, shift, st->hist[p], lb, &st->ticket[p], status,
                nullptr, nblk, recs_by_idx, rank_counts, rank_rects);
        else
            k_radix_pass<true, false><<<dim3(unsigned(nblk)), kSortThreads, 0, s>>>(
                kin, vin, kout, vout, count, shift, st->hist[p], lb, &st->ticket[p], status,
                nullptr, nblk, nullptr, nullptr, nullptr);
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
}

// Tile sort of up to cap pairs (count on the device) on key bits [0, bits): per pass a per-block
// histogram, its exclusive scan and the scatter. (With thousands of tiles of keys the chained
// passes wait on long look-back chains; the three-step pass does not.) The data ends in (ka, va)
// after an even number of passes, in (kb, vb) after an odd one; returns the number of passes.
template <typename K>
int sort_tiles(K *ka, K *kb, uint32_t *va, uint32_t *vb, const unsigned long long *count,
               int64_t cap, int bits, uint32_t *hist, uint32_t *partial, int32_t *status,
               hipStream_t s) {
    const int64_t nblk = sort_blocks(cap);
    const int passes = (bits + kRadixBits - 1) / kRadixBits;
    if (nblk == 0) return passes;
    K *kin = ka, *kout = kb;
    uint32_t *vin = va, *vout = vb;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * kRadixBits;
        k_block_hist<<<dim3(unsigned(nblk)), kSortThreads, 0, s>>>(kin, count, shift, hist, nblk);
        launch_scan<uint32_t>(hist, int64_t(kRadix) * nblk, partial, nullptr, nullptr, s);
        k_radix_pass<false, false, K><<<dim3(unsigned(nblk)), kSortThreads, 0, s>>>(
            kin, vin, kout, vout, count, shift, nullptr, nullptr, nullptr, status, hist, nblk,
            nullptr, nullptr, nullptr);
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    return passes;
}

// Start of bin_fill: empty ranges, zeroed sort states, the Gaussian count for the depth sort and
// a clean status word (later kernels only ever write error codes into it).
__global__ __launch_bounds__(256) void k_bin_init(uint32_t *ranges, int64_t m, SortState *sorts,
                                                  BinHeader *hdr, int64_t n, int32_t *status) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < m) ranges[i] = 0u;
    if (blockIdx.x == 0) {
        uint32_t *w = reinterpret_cast<uint32_t *>(sorts);
        for (int k = threadIdx.x; k < int(sizeof(SortState) / 4); k += blockDim.x) w[k] = 0u;
        if (threadIdx.x == 0) {
            hdr->gaussians = (unsigned long long)n;
            *status = GSB_OK;
        }
    }
}

// Tile boundaries in the sorted tile ids: four consecutive pairs per thread (one vector load and
// the two neighbours outside it). `tiles` is 256-byte aligned.
template <typename K>
__global__ __launch_bounds__(256) void k_ranges(const K *tiles, const unsigned long long *count,
                                                uint32_t *ranges) {
    const int64_t P = int64_t(*count);
    const int64_t i0 = 4 * (int64_t(blockIdx.x) * blockDim.x + threadIdx.x);
    if (i0 >= P) return;
    uint32_t t[6];                       // tiles[i0 - 1 .. i0 + 4]; outside [0, P): no tile
    t[0] = i0 > 0 ? tiles[i0 - 1] : 0xffffffffu;
    if (i0 + 4 <= P) {
        const uint4 v = load4(tiles, i0);
        t[1] = v.x; t[2] = v.y; t[3] = v.z; t[4] = v.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) t[1 + k] = i0 + k < P ? tiles[i0 + k] : 0xffffffffu;
    }
    t[5] = i0 + 4 < P ? tiles[i0 + 4] : 0xffffffffu;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = i0 + k;
        if (i >= P) break;
        if (t[k] != t[k + 1]) ranges[2 * int64_t(t[k + 1])] = uint32_t(i);
        if (t[k + 2] != t[k + 1]) ranges[2 * int64_t(t[k + 1]) + 1] = uint32_t(i + 1);
    }
}

int ceil_log2(int64_t v) {
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

}  // namespace

size_t bin_workspace_bytes(int64_t n, int64_t pair_capacity, int64_t /*n_tiles*/) {
    // bin_count uses the leading part, which does not depend on the capacity; bin_fill all of it
    return layout(n, pair_capacity).end;
}

int64_t bin_max_gaussians() { return kScanMaxLen; }
// the tile sort scans [256][blocks] histograms with the single-top-level scan
int64_t bin_max_pairs() { return int64_t(kScanMaxLen / kRadix) * kSortTile; }

gsb_status bin_count(const float *means2d, const int32_t *radii, const float *conics,
                     const float *opacity, int32_t mode, int64_t n, int32_t W, int32_t H, void *ws,
                     int64_t *n_pairs_dev, hipStream_t s) {
    const Layout L = layout(n, 0);
    auto *hdr = at<BinHeader>(ws, L.hdr);
    auto *counts = at<unsigned long long>(ws, L.counts);
    auto *partial = at<unsigned long long>(ws, L.partials);
    const int32_t gx = int32_t(grid_x(W)), gy = int32_t(grid_y(H));
    if (n > 0)
        k_bin_count<<<dim3(unsigned((n + 255) / 256)), 256, 0, s>>>(
            reinterpret_cast<const float2 *>(means2d), radii, conics, opacity, mode, n, gx, gy, W,
            H, counts, at<unsigned long long>(ws, L.masks), at<uint4>(ws, L.recs));
    // the total only: offsets are formed in depth order by bin_fill
    launch_scan<unsigned long long>(counts, n, partial, &hdr->total,
                                    reinterpret_cast<long long *>(n_pairs_dev), s, false);
    return check_launch("bin_count");
}

gsb_status bin_fill(const float *means2d, const int32_t *radii, const float *conics,
                    const float *opacity, int32_t mode, const float *depths, int64_t n, int32_t W,
                    int32_t H, void *ws, uint32_t *point_list, int64_t cap, uint32_t *ranges,
                    int32_t *status_dev, hipStream_t s) {
    const Layout L = layout(n, cap);
    auto *hdr = at<BinHeader>(ws, L.hdr);
    auto *counts = at<unsigned long long>(ws, L.counts);
    auto *partial64 = at<unsigned long long>(ws, L.partials);
    auto *partial32 = at<uint32_t>(ws, L.partials);
    auto *sorts = at<SortState>(ws, L.sorts);
    auto *sortbuf = at<uint32_t>(ws, L.sortbuf);
    uint32_t *dka = at<uint32_t>(ws, L.dkey_a), *dkb = at<uint32_t>(ws, L.dkey_b);
    uint32_t *dva = at<uint32_t>(ws, L.dval_a), *dvb = at<uint32_t>(ws, L.dval_b);
    auto *offs = at<unsigned long long>(ws, L.offs);
    uint32_t *vtmp = at<uint32_t>(ws, L.vals_tmp);
    const int32_t gx = int32_t(grid_x(W)), gy = int32_t(grid_y(H));
    const int64_t n_tiles = int64_t(gx) * gy;
    const unsigned gn = unsigned(n > 0 ? (n + 255) / 256 : 1);

    k_bin_init<<<dim3(unsigned((2 * n_tiles + 255) / 256)), 256, 0, s>>>(ranges, 2 * n_tiles,
                                                                       sorts, hdr, n, status_dev);
    // 1. Gaussians by depth (ties by index: the sort is stable over index order); the last pass
    //    also lays out each Gaussian's pair count and emission rectangle in rank order
    sort_depth(depths, dka, dkb, dva, dvb, &hdr->gaussians, n, sorts, sortbuf, status_dev,
               at<uint4>(ws, L.recs), offs, at<unsigned long long>(ws, L.rects), s);
    const uint32_t *sorted_idx = dva;
    // 2. offsets in rank order; pairs emitted in rank order
    launch_scan<unsigned long long>(offs, n, partial64, nullptr, nullptr, s);
    const int tile_bits = ceil_log2(n_tiles) > 0 ? ceil_log2(n_tiles) : 1;
    const int tp = (tile_bits + kRadixBits - 1) / kRadixBits;
    // the last pass must land the values in point_list
    uint32_t *v_first = (tp % 2 == 0) ? point_list : vtmp;
    uint32_t *v_second = (tp % 2 == 0) ? vtmp : point_list;
    // 3. stable sort of the pairs on the tile id; 4. the tiles' ranges. The emission stages 6144
    //    pairs per block when 256 ranks are expected to emit more than 3584 (capacity per Gaussian)
    const bool large_stage = n > 0 && 256.0 * double(cap) > 3584.0 * double(n);
    const auto emit_sort_range = [&](auto *tka, auto *tkb) {
        using K = std::remove_pointer_t<decltype(tka)>;
        const auto fill = large_stage ? k_bin_fill<K, kFillStageLarge> : k_bin_fill<K, kFillStage>;
        fill<<<gn, 256, 0, s>>>(reinterpret_cast<const float2 *>(means2d), conics, opacity, mode, W,
                                H, sorted_idx, n, gx, gy, offs, counts,
                                at<unsigned long long>(ws, L.masks),
                                at<unsigned long long>(ws, L.rects), hdr, cap, tka, v_first,
                                status_dev);
        sort_tiles<K>(tka, tkb, v_first, v_second, &hdr->pairs, cap, tile_bits, sortbuf,
                      partial32, status_dev, s);
        const K *tiles_sorted = (tp % 2 == 0) ? tka : tkb;
        if (cap > 0)
            k_ranges<K><<<dim3(unsigned((cap + 1023) / 1024)), 256, 0, s>>>(tiles_sorted,
                                                                             &hdr->pairs, ranges);
    };
    if (n_tiles <= kMaxTiles16)
        emit_sort_range(at<uint16_t>(ws, L.tkey_a), at<uint16_t>(ws, L.tkey_b));
    else
        emit_sort_range(at<uint32_t>(ws, L.tkey_a), at<uint32_t>(ws, L.tkey_b));
    return check_launch("bin_fill");
}

// ------------------------------------------------------------------------------- pair sort
// The binning's stable pair sort and range extraction, for other steps that group (key, value)
// pairs by key (the deterministic backward groups list positions by Gaussian).
size_t pair_sort_scratch_bytes(int64_t cap) {
    return align256(sizeof(uint32_t) * kRadix * size_t(sort_blocks(cap > 0 ? cap : 1))) +
           align256(sizeof(unsigned long long) * kScanMaxBlocks);
}

int pair_sort(uint32_t *ka, uint32_t *kb, uint32_t *va, uint32_t *vb,
              const unsigned long long *count, int64_t cap, int bits, void *scratch,
              hipStream_t s) {
    uint32_t *hist = static_cast<uint32_t *>(scratch);
    uint32_t *partial = reinterpret_cast<uint32_t *>(
        static_cast<char *>(scratch) +
        align256(sizeof(uint32_t) * kRadix * size_t(sort_blocks(cap > 0 ? cap : 1))));
    return sort_tiles<uint32_t>(ka, kb, va, vb, count, cap, bits, hist, partial, nullptr, s);
}

void key_ranges(const uint32_t *sorted_keys, const unsigned long long *count, int64_t cap,
                uint32_t *ranges, hipStream_t s) {
    if (cap > 0)
        k_ranges<uint32_t><<<dim3(unsigned((cap + 1023) / 1024)), 256, 0, s>>>(sorted_keys, count,
                                                                                ranges);
}

// ------------------------------------------------------------------------------- no-alloc binning
// Library-held binning workspace for callers that cannot allocate device memory. One copy of the
// array lives on every GPU the library runs on, at its own address, from module load to process
// end. In host code the name `scratch` only stands in for the symbol: its device address comes
// from hipGetSymbolAddress, once per device, with that device current, and only that address is
// passed to kernels.
static __device__ __align__(256) unsigned char scratch[GSB_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices];   // device address of `scratch` per device (null = not yet)
}  // namespace

gsb_status bin_noalloc(const float *means2d, const int32_t *radii, const float *conics,
                       const float *opacity, int32_t mode, const float *depths, int64_t n,
                       int32_t W, int32_t H, uint32_t *point_list, int64_t cap, uint32_t *ranges,
                       int64_t *n_pairs_dev, int32_t *status_dev, hipStream_t s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(GSB_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kScratchDevices)
        return fail(GSB_ERR_UNSUPPORTED, "device id %d out of range", dev);
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (g_scratch_ptr[dev] == nullptr) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || p == nullptr)
                return fail(GSB_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            g_scratch_ptr[dev] = p;
        }
        ws = g_scratch_ptr[dev];
    }
    // Every word of the workspace that the binning reads is written earlier in the same call
    // (counts, scans, the sort state and look-back words are initialised by its own kernels), so
    // what a previous call left in the array needs no clearing.
    const gsb_status st = bin_count(means2d, radii, conics, opacity, mode, n, W, H, ws,
                                    n_pairs_dev, s);
    if (st != GSB_OK) return st;
    return bin_fill(means2d, radii, conics, opacity, mode, depths, n, W, H, ws, point_list, cap,
                    ranges, status_dev, s);
}

}  // namespace gsb
