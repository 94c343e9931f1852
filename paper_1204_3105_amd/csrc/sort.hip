// sort.hip -- device-wide exclusive scan and stable LSD radix sort.
//
// The radix sort orders (key, index) pairs by key, keeping equal keys in
// index order, so the sorted permutation is unique.  Each pass handles 7 to
// 10 bits: per-tile digit histograms, one exclusive scan over the
// [digit][tile] table, and a scatter in which every element's rank among
// equal digits of its tile is found with wave64 ballots (a match mask per
// lane) and per-wave counters in LDS.  Tiles are read in striped order, so
// ranks follow the original order and the pass is stable.
#include <algorithm>

#include "fmm_internal.h"

namespace fmm {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// ------------------------------------------------------------------ scan
__device__ __forceinline__ int32_t wave_incl_scan(int32_t v)
{
    int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the prefix and
// writes the block total to *total.
__device__ int32_t block_excl_scan(int32_t v, int32_t *total)
{
    __shared__ int32_t wsum[16];
    __shared__ int32_t wtot;
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int32_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t acc = 0;
        for (int k = 0; k < nw; ++k) {
            int32_t t = wsum[k];
            wsum[k] = acc;
            acc += t;
        }
        wtot = acc;
    }
    __syncthreads();
    int32_t res = inc - v + wsum[w];
    *total = wtot;
    __syncthreads();
    return res;
}

__global__ void k_scan_tile_sums(const int32_t *__restrict__ in, int64_t n, int32_t *__restrict__ sums)
{
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int32_t acc = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (i < n) acc += in[i];
    }
    int32_t tot;
    block_excl_scan(acc, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Single-block exclusive scan of the tile sums (in place); total -> *total.
__global__ void k_scan_sums(int32_t *__restrict__ sums, int64_t n, int32_t *__restrict__ total)
{
    int64_t per = (n + blockDim.x - 1) / blockDim.x;
    int64_t b = per * threadIdx.x, e = b + per < n ? b + per : n;
    int32_t acc = 0;
    for (int64_t i = b; i < e; ++i) acc += sums[i];
    int32_t tot;
    int32_t off = block_excl_scan(acc, &tot);
    for (int64_t i = b; i < e; ++i) {
        int32_t t = sums[i];
        sums[i] = off;
        off += t;
    }
    if (threadIdx.x == 0 && total) *total = tot;
}

__global__ void k_scan_apply(const int32_t *__restrict__ in, int32_t *__restrict__ out, int64_t n,
                             const int32_t *__restrict__ sums)
{
    // Blocked layout: thread t owns kScanItems consecutive elements.
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = i < n ? in[i] : 0;
        acc += v[k];
    }
    int32_t tot;
    int32_t off = block_excl_scan(acc, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = off;
        off += v[k];
    }
}

// One block of 1024 threads for short arrays (up to 32 Ki elements): the
// array is read with coalesced loads (all in flight together) into LDS,
// where thread t scans the 32 consecutive elements from 32 t after a block
// scan of the run totals; the result leaves LDS with coalesced stores.  LDS
// index i + i/32 keeps both access patterns free of bank conflicts.
constexpr int kScanSmallRun = 32;
constexpr int64_t kScanSmall = 1024 * kScanSmallRun;
__global__ __launch_bounds__(1024) void k_scan_small(const int32_t *__restrict__ in, int32_t *__restrict__ out,
                                                     int64_t n, int32_t *__restrict__ total)
{
    __shared__ int32_t sh[kScanSmall + kScanSmall / 32];
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < kScanSmallRun; ++k) {
        const int i = k * 1024 + t;
        sh[i + (i >> 5)] = i < n ? in[i] : 0;
    }
    __syncthreads();
    int32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanSmallRun; ++k) acc += sh[33 * t + k];
    int32_t tot;
    int32_t off = block_excl_scan(acc, &tot);   // synchronizes the block
#pragma unroll
    for (int k = 0; k < kScanSmallRun; ++k) {
        const int32_t v = sh[33 * t + k];
        sh[33 * t + k] = off;
        off += v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanSmallRun; ++k) {
        const int i = k * 1024 + t;
        if (i < n) out[i] = sh[i + (i >> 5)];
    }
    if (t == 0 && total) *total = tot;
}

size_t scan_tmp_bytes(int64_t n)
{
    int64_t tiles = (n + kScanTile - 1) / kScanTile;
    return (size_t)(tiles + 1) * sizeof(int32_t) + 256;
}

// out may alias in.  *total (device) receives the sum when non-null.
void scan_exclusive(const int32_t *in, int32_t *out, int64_t n, int32_t *total, void *tmp,
                    hipStream_t s)
{
    if (n <= kScanSmall) {
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, s, in, out, n, total);
        return;
    }
    int64_t tiles = (n + kScanTile - 1) / kScanTile;
    int32_t *sums = (int32_t *)tmp;
    hipLaunchKernelGGL(k_scan_tile_sums, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, n,
                       sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, sums, tiles, total);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, out, n,
                       sums);
}

// ------------------------------------------------------------------ radix
// Digits of W bits (7..10); a key of B bits takes ceil(B/10) passes, the
// digits split evenly, so keys up to 20 bits sort in two passes.
constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 8;
constexpr int kRadixTile = kRadixThreads * kRadixItems;   // striped rounds of 256
constexpr int kRadixMaxBins = 1024;

template <int W>
__global__ __launch_bounds__(kRadixThreads) void k_radix_count(const uint32_t *__restrict__ keys, int64_t n,
                                                               int shift, int32_t *__restrict__ counts,
                                                               int ntiles)
{
    constexpr int NB = 1 << W;
    __shared__ int32_t hist[NB];
    for (int b = threadIdx.x; b < NB; b += kRadixThreads) hist[b] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    uint32_t kk[kRadixItems];   // all loads in flight before the first atomic
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
        const int64_t i = base + (int64_t)k * kRadixThreads + threadIdx.x;
        kk[k] = i < n ? keys[i] : 0xffffffffu;
    }
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
        const int64_t i = base + (int64_t)k * kRadixThreads + threadIdx.x;
        if (i < n) atomicAdd(&hist[(kk[k] >> shift) & (NB - 1)], 1);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < NB; b += kRadixThreads) counts[(int64_t)b * ntiles + blockIdx.x] = hist[b];
}

template <int W>
__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                                 const int32_t *__restrict__ vin,
                                                                 uint32_t *__restrict__ kout,
                                                                 int32_t *__restrict__ vout, int64_t n,
                                                                 int shift, const int32_t *__restrict__ offs,
                                                                 int ntiles)
{
    constexpr int NB = 1 << W;
    __shared__ int32_t run[NB];        // elements of each digit already placed
    __shared__ int32_t wcnt[4][NB];    // per-wave digit counts of this round
    __shared__ int32_t goff[NB];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int b = t; b < NB; b += kRadixThreads) {
        goff[b] = offs[(int64_t)b * ntiles + blockIdx.x];
        run[b] = 0;
    }
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    uint32_t kk[kRadixItems];   // the tile's loads all in flight before the first round
    int32_t vv[kRadixItems];
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
        const int64_t i = base + (int64_t)k * kRadixThreads + t;
        kk[k] = i < n ? kin[i] : 0u;
        vv[k] = i < n ? vin[i] : 0;
    }
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
        for (int b = t; b < NB; b += kRadixThreads)
            for (int q = 0; q < 4; ++q) wcnt[q][b] = 0;
        __syncthreads();
        const int64_t i = base + (int64_t)k * kRadixThreads + t;
        const bool valid = i < n;
        const uint32_t key = kk[k];
        const int32_t val = vv[k];
        const uint32_t d = (key >> shift) & (NB - 1);
        // lanes of this wave with the same digit: W ballots
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int b = 0; b < W; ++b) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            match &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const int rank_w = __popcll(match & lt_mask);
        if (valid && rank_w == 0) wcnt[w][d] = __popcll(match);
        __syncthreads();
        if (valid) {
            int32_t before = 0;
            for (int q = 0; q < w; ++q) before += wcnt[q][d];
            const int64_t pos = (int64_t)goff[d] + run[d] + before + rank_w;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        for (int b = t; b < NB; b += kRadixThreads) run[b] += wcnt[0][b] + wcnt[1][b] + wcnt[2][b] + wcnt[3][b];
    }
}

size_t radix_tmp_bytes(int64_t n)
{
    int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
    if (ntiles == 0) ntiles = 1;
    size_t counts = (size_t)kRadixMaxBins * ntiles * sizeof(int32_t);
    size_t bufs = (size_t)n * (sizeof(uint32_t) + sizeof(int32_t));
    return counts + scan_tmp_bytes(kRadixMaxBins * ntiles) + bufs + 1024;
}

static char *align256(char *p) { return (char *)(((uintptr_t)p + 255) & ~(uintptr_t)255); }

template <int W>
static void radix_pass(const uint32_t *ka, const int32_t *va, uint32_t *kb, int32_t *vb, int64_t n, int shift,
                       int32_t *counts, void *stmp, int ntiles, hipStream_t s)
{
    hipLaunchKernelGGL((k_radix_count<W>), dim3(ntiles), dim3(kRadixThreads), 0, s, ka, n, shift, counts,
                       ntiles);
    scan_exclusive(counts, counts, ((int64_t)1 << W) * ntiles, nullptr, stmp, s);
    hipLaunchKernelGGL((k_radix_scatter<W>), dim3(ntiles), dim3(kRadixThreads), 0, s, ka, va, kb, vb, n,
                       shift, counts, ntiles);
}

void radix_sort(uint32_t *keys, int32_t *vals, int64_t n, int bits, void *tmp, hipStream_t s)
{
    if (n <= 1 || bits <= 0) return;
    int ntiles = (int)((n + kRadixTile - 1) / kRadixTile);
    char *p = align256((char *)tmp);
    int32_t *counts = (int32_t *)p;
    p = align256(p + (size_t)kRadixMaxBins * ntiles * sizeof(int32_t));
    void *stmp = p;
    p = align256(p + scan_tmp_bytes(kRadixMaxBins * (int64_t)ntiles));
    uint32_t *k2 = (uint32_t *)p;
    p = align256(p + (size_t)n * sizeof(uint32_t));
    int32_t *v2 = (int32_t *)p;
    uint32_t *ka = keys, *kb = k2;
    int32_t *va = vals, *vb = v2;
    const int passes = (bits + 9) / 10;
    const int wd = std::max(7, (bits + passes - 1) / passes);   // 7..10
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = wd * ps;
        switch (wd) {
        case 7: radix_pass<7>(ka, va, kb, vb, n, shift, counts, stmp, ntiles, s); break;
        case 8: radix_pass<8>(ka, va, kb, vb, n, shift, counts, stmp, ntiles, s); break;
        case 9: radix_pass<9>(ka, va, kb, vb, n, shift, counts, stmp, ntiles, s); break;
        default: radix_pass<10>(ka, va, kb, vb, n, shift, counts, stmp, ntiles, s); break;
        }
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        hipMemcpyAsync(keys, ka, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        hipMemcpyAsync(vals, va, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
    }
}

}  // namespace fmm
