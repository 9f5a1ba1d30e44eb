// Tile binning on the GPU: per-Gaussian tile count and prefix sum, duplication with
// tile|depth keys (paper §2.1(b)), stable LSD radix sort of the keys (§2.1(c)), and per-tile
// [start, end) ranges of the sorted list (the per-tile index lists consumed by Alg. 1 / Alg. 2).
//
// Everything is integer work and bit-exact: the covered-tile rectangle is evaluated in integer
// arithmetic (floor((x - r)/16) == (floor(x) - r) >> 4 for integer r), and the sort is stable over
// Gaussian-major emission order, so ties in depth keep increasing Gaussian index.
#include <hip/hip_runtime.h>

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

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;                           // keys per thread
constexpr int kSortTile = kSortThreads * kSortItems;     // 4096 keys per block
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

struct BinHeader {
    unsigned long long total;   // pairs counted by bin_count
    unsigned long long pairs;   // min(total, capacity), set by bin_fill
    uint32_t pad[12];
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct Layout {
    size_t hdr, offsets, partials, keys_a, keys_b, vals_tmp, hist, end;
};

Layout layout(int64_t n, int64_t cap) {
    Layout L;
    size_t o = 0;
    L.hdr = o;       o += align256(sizeof(BinHeader));
    L.offsets = o;   o += align256(sizeof(unsigned long long) * size_t(n > 0 ? n : 1));
    L.partials = o;  o += align256(sizeof(unsigned long long) * kScanMaxBlocks);
    // everything below depends on the pair capacity (bin_count uses only the part above)
    const int64_t nblk = (cap + kSortTile - 1) / kSortTile;
    L.keys_a = o;    o += align256(sizeof(unsigned long long) * size_t(cap));
    L.keys_b = o;    o += align256(sizeof(unsigned long long) * size_t(cap));
    L.vals_tmp = o;  o += align256(sizeof(uint32_t) * size_t(cap));
    L.hist = o;      o += align256(sizeof(uint32_t) * size_t(kRadix) * size_t(nblk > 0 ? nblk : 1));
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
// Exclusive prefix sum in three launches: per-block sums, a single-block scan of those, then a
// per-block scan with the block's offset. `in` and `out` may alias.
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

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const T *in, T *out, int64_t m,
                                                             const T *partial) {
    __shared__ T s_wave[kScanThreads / 64];
    const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
    T v[kScanItems], sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < m) ? in[base + k] : T(0);
        sum += v[k];
    }
    T tot;
    T run = block_exclusive_scan<T>(sum, s_wave, tot) + partial[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < m) out[base + k] = run;
        run += v[k];
    }
}

template <typename T>
void launch_scan(T *data, int64_t m, T *partial, unsigned long long *total_a, long long *total_b,
                 hipStream_t s) {
    const int64_t nb = (m + kScanTile - 1) / kScanTile;
    if (nb > 0) k_scan_reduce<T><<<dim3(unsigned(nb)), kScanThreads, 0, s>>>(data, m, partial);
    k_scan_top<T><<<1, kScanTopThreads, 0, s>>>(partial, nb, total_a, total_b);
    if (nb > 0) k_scan_down<T><<<dim3(unsigned(nb)), kScanThreads, 0, s>>>(data, data, m, partial);
}

// ------------------------------------------------------------------------------- tile rectangle
// Covered tiles [tx0, tx1) x [ty0, ty1) of a Gaussian at (x, y) with radius r: tx in
// [floor((x - r)/16), floor((x + r + 15)/16)) clamped to [0, gx], same for y. With x = ix + f,
// 0 <= f < 1, and r an integer, floor((x - r)/16) = floor((ix - r)/16) = (ix - r) >> 4 exactly.
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

__global__ __launch_bounds__(256) void k_bin_count(const float2 *means, const int32_t *radii,
                                                   int64_t n, int32_t gx, int32_t gy,
                                                   unsigned long long *counts) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 m = means[i];
    const Rect R = tile_rect(m.x, m.y, radii[i], gx, gy);
    counts[i] = (unsigned long long)(R.tx1 - R.tx0) * (unsigned long long)(R.ty1 - R.ty0);
}

// One thread per Gaussian writes its keys at its prefix-sum offset, row-major over its tiles.
__global__ __launch_bounds__(256) void k_bin_fill(const float2 *means, const int32_t *radii,
                                                  const float *depths, int64_t n, int32_t gx,
                                                  int32_t gy, const unsigned long long *offsets,
                                                  BinHeader *hdr, int64_t cap,
                                                  unsigned long long *keys, uint32_t *vals,
                                                  int32_t *status) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i == 0) {
        const unsigned long long total = hdr->total;
        hdr->pairs = total < (unsigned long long)cap ? total : (unsigned long long)cap;
        *status = total > (unsigned long long)cap ? GSB_ERR_CAPACITY : GSB_OK;
    }
    if (i >= n) return;
    const float2 m = means[i];
    const Rect R = tile_rect(m.x, m.y, radii[i], gx, gy);
    const unsigned long long dbits = __float_as_uint(depths[i]);
    unsigned long long o = offsets[i];
    for (int32_t ty = R.ty0; ty < R.ty1; ++ty)
        for (int32_t tx = R.tx0; tx < R.tx1; ++tx, ++o) {
            if (o >= (unsigned long long)cap) return;
            keys[o] = ((unsigned long long)(int64_t(ty) * gx + tx) << 32) | dbits;
            vals[o] = uint32_t(i);
        }
}

// ------------------------------------------------------------------------------- radix sort
// One pass of a stable LSD radix sort on an 8-bit digit, in three steps: per-block digit
// histograms (digit-major, so one exclusive scan yields every block's output offset per digit),
// the scan, and a scatter in which each block ranks its keys stably in LDS and writes them out
// in digit order (contiguous runs, so the global writes coalesce).

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const unsigned long long *keys,
                                                             const BinHeader *hdr, int shift,
                                                             uint32_t *hist, int64_t nblk) {
    __shared__ uint32_t s_h[kRadix];
    const int t = threadIdx.x;
    s_h[t] = 0;
    __syncthreads();
    const int64_t P = int64_t(hdr->pairs);
    const int64_t base = int64_t(blockIdx.x) * kSortTile;
#pragma unroll 4
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = base + int64_t(k) * kSortThreads + t;
        if (idx < P) atomicAdd(&s_h[(keys[idx] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    hist[int64_t(t) * nblk + blockIdx.x] = s_h[t];
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const unsigned long long *kin, const uint32_t *vin, unsigned long long *kout, uint32_t *vout,
    const BinHeader *hdr, int shift, const uint32_t *hist_off, int64_t nblk) {
    __shared__ uint32_t s_wcnt[kSortThreads / 64][kRadix];  // per-wave digit counts, then prefixes
    __shared__ uint32_t s_dstart[kRadix];                     // block-local start of each digit
    __shared__ uint32_t s_gofs[kRadix];                       // global start of each digit
    __shared__ uint32_t s_wave[kSortThreads / 64];
    __shared__ unsigned long long s_key[kSortTile];
    __shared__ uint32_t s_val[kSortTile];

    const int64_t P = int64_t(hdr->pairs);
    const int64_t base = int64_t(blockIdx.x) * kSortTile;
    if (base >= P) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
    for (int d = 0; d < kSortThreads / 64; ++d) s_wcnt[d][t] = 0;
    s_gofs[t] = hist_off[int64_t(t) * nblk + blockIdx.x];
    __syncthreads();

    // Wave w ranks keys [base + 1024 w, base + 1024 (w + 1)) in 16 steps of 64 consecutive keys,
    // so rank order within the wave is index order.
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
    unsigned long long key[kSortItems];
    uint32_t val[kSortItems], loc[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = base + int64_t(w) * (kSortItems * 64) + k * 64 + lane;
        const bool valid = idx < P;
        key[k] = valid ? kin[idx] : 0ull;
        val[k] = valid ? vin[idx] : 0u;
        const uint32_t d = uint32_t(key[k] >> shift) & (kRadix - 1);
        // lanes holding the same digit: intersect the ballots of every digit bit
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long vote = __ballot(bit);
            peers &= bit ? vote : ~vote;
        }
        const uint32_t rank = __popcll(peers & lt_mask);
        uint32_t prior = 0;
        if (valid) prior = s_wcnt[w][d];
        if (valid && rank == 0) s_wcnt[w][d] = prior + uint32_t(__popcll(peers));
        loc[k] = prior + rank;
    }
    __syncthreads();
    // thread t = digit t: exclusive prefix over waves, then over digits
    uint32_t c[kSortThreads / 64], run = 0;
#pragma unroll
    for (int i = 0; i < kSortThreads / 64; ++i) {
        c[i] = s_wcnt[i][t];
        s_wcnt[i][t] = run;
        run += c[i];
    }
    uint32_t tot;
    s_dstart[t] = block_exclusive_scan<uint32_t>(run, s_wave, tot);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = base + int64_t(w) * (kSortItems * 64) + k * 64 + lane;
        if (idx < P) {
            const uint32_t d = uint32_t(key[k] >> shift) & (kRadix - 1);
            const uint32_t r = s_dstart[d] + s_wcnt[w][d] + loc[k];
            s_key[r] = key[k];
            s_val[r] = val[k];
        }
    }
    __syncthreads();
    const int64_t nvalid = (P - base) < kSortTile ? (P - base) : kSortTile;
    for (int64_t j = t; j < nvalid; j += kSortThreads) {
        const unsigned long long k = s_key[j];
        const uint32_t d = uint32_t(k >> shift) & (kRadix - 1);
        const int64_t pos = int64_t(s_gofs[d]) + (j - int64_t(s_dstart[d]));
        kout[pos] = k;
        vout[pos] = s_val[j];
    }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, int64_t m, uint32_t v) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < m) p[i] = v;
}

__global__ __launch_bounds__(256) void k_ranges(const unsigned long long *keys,
                                                const BinHeader *hdr, uint32_t *ranges) {
    const int64_t P = int64_t(hdr->pairs);
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const uint32_t t = uint32_t(keys[i] >> 32);
    if (i == 0 || uint32_t(keys[i - 1] >> 32) != t) ranges[2 * int64_t(t)] = uint32_t(i);
    if (i == P - 1 || uint32_t(keys[i + 1] >> 32) != t) ranges[2 * int64_t(t) + 1] = uint32_t(i + 1);
}

int ceil_log2(int64_t v) {
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

}  // namespace

size_t bin_workspace_bytes(int64_t n, int64_t pair_capacity, int64_t /*n_tiles*/) {
    return layout(n, pair_capacity).end;
}

int64_t bin_max_gaussians() { return kScanMaxLen; }
int64_t bin_max_pairs() { return int64_t(kScanMaxLen / kRadix) * kSortTile; }

gsb_status bin_count(const float *means2d, const int32_t *radii, int64_t n, int32_t W, int32_t H,
                     void *ws, int64_t *n_pairs_dev, hipStream_t s) {
    const Layout L = layout(n, 0);
    auto *hdr = at<BinHeader>(ws, L.hdr);
    auto *offsets = at<unsigned long long>(ws, L.offsets);
    auto *partial = at<unsigned long long>(ws, L.partials);
    const int32_t gx = int32_t(grid_x(W)), gy = int32_t(grid_y(H));
    if (n > 0)
        k_bin_count<<<dim3(unsigned((n + 255) / 256)), 256, 0, s>>>(
            reinterpret_cast<const float2 *>(means2d), radii, n, gx, gy, offsets);
    launch_scan<unsigned long long>(offsets, n, partial, &hdr->total,
                                    reinterpret_cast<long long *>(n_pairs_dev), s);
    return check_launch("bin_count");
}

gsb_status bin_fill(const float *means2d, const int32_t *radii, const float *depths, int64_t n,
                    int32_t W, int32_t H, void *ws, uint32_t *point_list, int64_t cap,
                    uint32_t *ranges, int32_t *status_dev, hipStream_t s) {
    const Layout L = layout(n, cap);
    auto *hdr = at<BinHeader>(ws, L.hdr);
    auto *offsets = at<unsigned long long>(ws, L.offsets);
    auto *keys_a = at<unsigned long long>(ws, L.keys_a);
    auto *keys_b = at<unsigned long long>(ws, L.keys_b);
    auto *vals_tmp = at<uint32_t>(ws, L.vals_tmp);
    auto *hist = at<uint32_t>(ws, L.hist);
    auto *partial = at<uint32_t>(ws, L.partials);
    const int32_t gx = int32_t(grid_x(W)), gy = int32_t(grid_y(H));
    const int64_t n_tiles = int64_t(gx) * gy;
    const int key_bits = 32 + (ceil_log2(n_tiles) > 0 ? ceil_log2(n_tiles) : 1);
    const int passes = (key_bits + kRadixBits - 1) / kRadixBits;
    // the last pass must land the values in point_list
    uint32_t *v_first = (passes % 2 == 0) ? point_list : vals_tmp;
    uint32_t *v_second = (passes % 2 == 0) ? vals_tmp : point_list;

    k_fill_u32<<<dim3(unsigned((2 * n_tiles + 255) / 256)), 256, 0, s>>>(ranges, 2 * n_tiles, 0u);
    k_bin_fill<<<dim3(unsigned(n > 0 ? (n + 255) / 256 : 1)), 256, 0, s>>>(
        reinterpret_cast<const float2 *>(means2d), radii, depths, n, gx, gy, offsets, hdr, cap,
        keys_a, v_first, status_dev);
    const int64_t nblk = (cap + kSortTile - 1) / kSortTile;
    if (nblk > 0) {
        unsigned long long *kin = keys_a, *kout = keys_b;
        uint32_t *vin = v_first, *vout = v_second;
        for (int p = 0; p < passes; ++p) {
            const int shift = p * kRadixBits;
            k_radix_hist<<<dim3(unsigned(nblk)), kSortThreads, 0, s>>>(kin, hdr, shift, hist, nblk);
            launch_scan<uint32_t>(hist, int64_t(kRadix) * nblk, partial, nullptr, nullptr, s);
            k_radix_scatter<<<dim3(unsigned(nblk)), kSortThreads, 0, s>>>(kin, vin, kout, vout, hdr,
                                                                          shift, hist, nblk);
            std::swap(kin, kout);
            std::swap(vin, vout);
        }
        k_ranges<<<dim3(unsigned((cap + 255) / 256)), 256, 0, s>>>(kin, hdr, ranges);
    }
    return check_launch("bin_fill");
}

}  // namespace gsb
