// m2l_mixed.hip -- M2L as BF16x3 split products on MFMA (gfx950).
//
// Greengard & Rokhlin (1987) Lemma 2.4, radius-scaled.  For one (level,
// target group) every target cell sees the same E4 offsets, so for each
// slot s the translation is one real matrix M_s (rows: Re/Im of b~_0..b~_p;
// columns: Re/Im of a~_1..a~_p) applied to the gathered source columns:
//     B[:, T] += sum_s  M_s * A[:, src(T, s)]     (a dense contraction).
// The entries of M_s are T_0k = (-1/delta)^k and
// T_mk = C(m+k-1, k-1) (-1/delta)^k delta^-m (complex, 2x2 real blocks).
// Every FP32 operand x is split into three bfloat16 parts x = h + m + l
// (24 significand bits); the six products with weight >= 2^-16
// (hh, hm, mh, hl, lh, mm) run on v_mfma_f32_16x16x32_bf16 with FP32
// accumulation, and each slot's FP32 result is folded into FP64
// accumulators.  The monopole terms a_0 Log(c_T - c_S) and -a_0 delta^-m / m
// are added in FP64.  M_s is pre-split into the MFMA lane layout at plan
// time; it depends on the level only for the septree (whose offsets rotate
// by arctan(sqrt3/2) per level), so quadtree and triangle-quadtree tables
// are shared by all levels.
//
// MFMA 16x16x32 bf16 operand layout (lane l, j = 0..7 / 0..3):
//   A[i = l%16][k = 8(l/16)+j], B[k = 8(l/16)+j][n = l%16],
//   C[i = 4(l/16)+j][n = l%16].
#include <vector>

#include "eval.h"

namespace fmm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kTileT = 64;   // mixed: targets per workgroup (4 waves x 16 columns)
constexpr int kTileT64 = 16; // FP64: targets per workgroup (4 waves share 16 columns)

// Targets per M2L tile of a plan's form.
static int tile_targets(const Plan &P) { return P.precision == FMM_PREC_MIXED ? kTileT : kTileT64; }

struct MixedLayout {
    int MT, KB;          // 16-row M tiles, 32-deep K blocks
    int tab_levels;      // 1 (level-invariant) or L+1 (septree)
    int G, S, pm;
    size_t tab_elems;    // bf16 elements per (level, group, slot) table
    int n_tiles;
    size_t off_tab, off_tiles, off_list, off_cnt, off_b;   // byte offsets in P.mixed
};

// The M2L area of a plan: target tiles grouped by (level, group) for both
// forms; the split matrices and split multipoles only for the mixed form.
static MixedLayout layout_of(const Plan &P)
{
    const bool mixed = P.precision == FMM_PREC_MIXED;
    MixedLayout m;
    m.MT = (2 * (P.p + 1) + 15) / 16;
    m.KB = (2 * P.p + 31) / 32;
    m.tab_levels = P.geo.tiling == kSept ? P.geo.L + 1 : 1;
    m.G = P.tables.n_groups;
    m.S = P.tables.e4_width;
    m.pm = P.m2l_pm;
    m.tab_elems = (size_t)m.MT * m.KB * 3 * 64 * 8;
    m.n_tiles = 0;
    size_t o = 0;
    m.off_tab = o;
    if (mixed) o += (size_t)m.tab_levels * m.G * m.S * m.tab_elems * 2;
    o = (o + 255) & ~(size_t)255;
    m.off_cnt = o;   // cell counts/offsets, cursors, tile offsets: 256 each
    o += 3 * 256 * sizeof(int32_t);
    m.off_tiles = o;
    int64_t ncell = P.n_cells;
    o += (size_t)(ncell / tile_targets(P) + 2 * (kMaxL + 1) * kMaxGroups + 2) * 4 * sizeof(int32_t);
    o = (o + 255) & ~(size_t)255;
    m.off_list = o;
    o += (size_t)(ncell + 1) * sizeof(int32_t);
    o = (o + 255) & ~(size_t)255;
    m.off_b = o;   // split multipoles: [cell][kb][split][q] bf16x8
    return m;
}

size_t mixed_bytes(const Plan &P)
{
    if (P.m2l_pm == 0) return 256;
    MixedLayout m = layout_of(P);
    const size_t splits = P.precision == FMM_PREC_MIXED ? (size_t)P.n_cells * m.KB * 12 * 16 : 0;
    return m.off_b + splits + 256;
}

struct CellOffsets {
    int64_t v[kMaxL + 2];
};
struct SlotCounts {
    int v[kMaxGroups];
};

// Build the split matrices: block per (table level, group, slot, mt, kb),
// lane per MFMA lane.
__global__ __launch_bounds__(64) void k_build_mixed_tables(int p, int MT, int KB, int G, int S, int pm,
                                                           int sept, SlotCounts counts,
                                                           const double *__restrict__ pwt,
                                                           const double *__restrict__ binom,
                                                           __bf16 *__restrict__ tab)
{
    const int lane = threadIdx.x;
    int id = blockIdx.x;
    const int kb = id % KB;
    id /= KB;
    const int mt = id % MT;
    id /= MT;
    const int s = id % S;
    id /= S;
    const int g = id % G;
    const int tl = id / G;                 // table level
    const int lev = sept ? tl : 1;         // FP64 power table level to read
    const size_t tidx = ((size_t)tl * G + g) * S + s;
    __bf16 *out = tab + tidx * (size_t)MT * KB * 3 * 512 + ((size_t)(mt * KB + kb) * 3) * 512;
    const bool used = s < counts.v[g] && (!sept || tl >= 1);
    const double *pw = pwt + 2 * (((size_t)lev * G + g) * S + s) * (pm + 1);
    const int row = 16 * mt + (lane % 16);
    for (int j = 0; j < 8; ++j) {
        const int col = 32 * kb + 8 * (lane / 16) + j;
        double v = 0.0;
        const int m = row / 2, k = col / 2 + 1;
        if (used && m <= p && k <= p) {
            // T_mk = C(m+k-1, k-1) (-1/delta)^k delta^-m ; T_0k = (-1/delta)^k
            double tr = pw[2 * k], ti = pw[2 * k + 1];
            if (m > 0) {
                double dr = pw[2 * m], di = pw[2 * m + 1];
                if (m & 1) {
                    dr = -dr;
                    di = -di;
                }
                const double c = binom[(m + k - 1) * kBinomStride + (k - 1)];
                const double nr = (tr * dr - ti * di) * c, ni = (tr * di + ti * dr) * c;
                tr = nr;
                ti = ni;
            }
            const bool re_out = (row & 1) == 0, re_in = (col & 1) == 0;
            v = re_out ? (re_in ? tr : -ti) : (re_in ? ti : tr);
        }
        __bf16 h, mm, l;
        split3((float)v, h, mm, l);
        out[0 * 512 + lane * 8 + j] = h;
        out[1 * 512 + lane * 8 + j] = mm;
        out[2 * 512 + lane * 8 + j] = l;
    }
}

// Group target cells of levels >= 1 by (level, group): per-block LDS
// histograms, one global atomic per (block, key).
__global__ void k_group_count(int64_t first, int64_t n_cells, int L, int G, CellOffsets cell_off,
                              const uint8_t *__restrict__ occ,
                              const uint8_t *__restrict__ group, int32_t *__restrict__ cnt)
{
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t gid = first + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid < n_cells && (occ[gid] & 2)) {
        int l = 1;
        while (l < L && gid >= cell_off.v[l + 1]) ++l;
        atomicAdd(&h[l * G + group[gid]], 1);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], h[threadIdx.x]);
}

__global__ void k_group_scatter(int64_t first, int64_t n_cells, int L, int G, CellOffsets cell_off,
                                const uint8_t *__restrict__ occ,
                                const uint8_t *__restrict__ group, const int32_t *__restrict__ off,
                                int32_t *__restrict__ cursor, int32_t *__restrict__ list)
{
    __shared__ int32_t h[256], base[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t gid = first + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int key = -1, rank = 0;
    if (gid < n_cells && (occ[gid] & 2)) {
        int l = 1;
        while (l < L && gid >= cell_off.v[l + 1]) ++l;
        key = l * G + group[gid];
        rank = atomicAdd(&h[key], 1);
    }
    __syncthreads();
    if (h[threadIdx.x]) base[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], h[threadIdx.x]);
    __syncthreads();
    if (key >= 0) list[off[key] + base[key] + rank] = (int32_t)gid;
}

// One block: turns the per-key cell counts into cell offsets (in place,
// off[K] = total), tile offsets toff[0..K] (ceil(count / T) tiles per key)
// and the tile total; clears the scatter cursors.
__global__ __launch_bounds__(256) void k_tile_plan(int K, int T, int32_t *__restrict__ cnt,
                                                   int32_t *__restrict__ cursor,
                                                   int32_t *__restrict__ toff,
                                                   int32_t *__restrict__ n_tiles)
{
    __shared__ int32_t sc[256], st[256];
    const int k = threadIdx.x;
    const int32_t c = k < K ? cnt[k] : 0;
    sc[k] = c;
    st[k] = (c + T - 1) / T;
    cursor[k] = 0;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {   // inclusive Hillis-Steele scans
        const int32_t a = k >= d ? sc[k - d] : 0, b = k >= d ? st[k - d] : 0;
        __syncthreads();
        sc[k] += a;
        st[k] += b;
        __syncthreads();
    }
    if (k <= K) {
        cnt[k] = k ? sc[k - 1] : 0;
        toff[k] = k ? st[k - 1] : 0;
    }
    if (k == 0) *n_tiles = st[255];
}

// Thread per tile t < n_tiles: key = the k with toff[k] <= t < toff[k+1];
// tile = {key, first list position, cell count (<= T), 0}.
__global__ void k_tile_fill(int K, int T, const int32_t *__restrict__ off, const int32_t *__restrict__ toff,
                            const int32_t *__restrict__ n_tiles, int32_t *__restrict__ tiles)
{
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= *n_tiles) return;
    int lo = 0, hi = K;   // toff[lo] <= t < toff[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (toff[mid] <= t) lo = mid;
        else hi = mid;
    }
    const int32_t j = t - toff[lo];
    const int32_t c = off[lo + 1] - off[lo];
    tiles[4 * t] = lo;
    tiles[4 * t + 1] = off[lo] + j * T;
    tiles[4 * t + 2] = min(T, c - j * T);
    tiles[4 * t + 3] = 0;
}

int mixed_setup(Plan &P)
{
    if (P.m2l_pm == 0 || P.geo.L < 1) return 0;
    MixedLayout m = layout_of(P);
    char *base = (char *)P.mixed;
    hipStream_t s = P.stream;
    const int G = m.G, L = P.geo.L;
    int32_t *cnt = (int32_t *)(base + m.off_cnt);
    int32_t *cursor = cnt + 256;
    int32_t *list = (int32_t *)(base + m.off_list);
    int32_t *tiles = (int32_t *)(base + m.off_tiles);
    CellOffsets coff;
    for (int l = 0; l < kMaxL + 2; ++l) coff.v[l] = P.n_cells;
    for (int l = 0; l <= L; ++l) coff.v[l] = P.lev[l].cell_off;
    int32_t *toff = cnt + 512;
    hipMemsetAsync(cnt, 0, 256 * sizeof(int32_t), s);
    const int64_t first = P.lev[1].cell_off, n = P.n_cells - first;
    const int K = L * G + G;   // keys l*G + g, l = 0..L (level 0 stays empty)
    if (n > 0)
        hipLaunchKernelGGL(k_group_count, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, first,
                           P.n_cells, L, G, coff, P.cell_occ, P.group, cnt);
    const int T = tile_targets(P);
    hipLaunchKernelGGL(k_tile_plan, dim3(1), dim3(256), 0, s, K, T, cnt, cursor, toff, P.counts + 1);
    // sum_k ceil(c_k / T) <= (sum_k c_k) / T + (keys of levels >= 1)
    P.mixed_tiles = (int)(n / T + (int64_t)L * G + 1);
    hipLaunchKernelGGL(k_tile_fill, dim3((unsigned)((P.mixed_tiles + 255) / 256)), dim3(256), 0, s,
                       K, T, cnt, toff, P.counts + 1, tiles);
    if (n > 0)
        hipLaunchKernelGGL(k_group_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, first,
                           P.n_cells, L, G, coff, P.cell_occ, P.group, cnt, cursor, list);
    if (P.precision != FMM_PREC_MIXED) return hipGetLastError() != hipSuccess;
    // Split translation matrices.
    SlotCounts counts;
    for (int g = 0; g < kMaxGroups; ++g) counts.v[g] = g < G ? P.tables.e4_count[g] : 0;
    const int nb = m.tab_levels * G * m.S * m.MT * m.KB;
    hipLaunchKernelGGL(k_build_mixed_tables, dim3(nb), dim3(64), 0, s, P.p, m.MT, m.KB, G, m.S, m.pm,
                       P.geo.tiling == kSept ? 1 : 0, counts, P.m2l_pw, P.binom,
                       (__bf16 *)(base + m.off_tab));
    return hipGetLastError() != hipSuccess;
}

// One workgroup (4 waves) per tile of up to 64 target cells of one (level,
// group); wave w owns target columns 16w..16w+15.  The slots with at least one
// source in the tile are listed first (E4 rows staged in LDS), then processed
// as a software pipeline: while the MFMAs of slot i read its split matrix
// from one LDS buffer, the matrix, monopole row and gathered source columns of
// slot i+1 are already in flight to registers and go to the other buffer
// after the MFMAs, so one barrier per slot and no load on the critical path.
template <int MT, int KB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_m2l_bf16x3(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    far_field_priority();
    constexpr int NA = MT * KB * 3 * 64;   // bf16x8 vectors of one slot's matrix
    constexpr int NR = 32 * MT;            // output rows (>= 2(p+1))
    constexpr int PER = (NA + 255) / 256;  // staging vectors per thread
    __shared__ bf16x8 Ash[2][NA];
    __shared__ double A0s[2][NR];
    __shared__ int32_t srcs[kMaxSlots][64];
    __shared__ int8_t act[kMaxSlots];
    __shared__ int32_t nact;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = lane % 16, q = lane / 16;
    const bf16x8 zero8 = {};
    // XCD-aware order: the 8 XCDs each take a contiguous eighth of the tiles
    // (workgroups are dealt to XCDs round-robin), so the tiles of one
    // (level, group) -- which share translation matrices -- stay on one L2.
    const int64_t total = bm.pre[bm.n];
    const int xcd = blockIdx.x % 8, lb = blockIdx.x / 8, nb = gridDim.x / 8;
    const int64_t t_beg = total * xcd / 8, t_end = total * (xcd + 1) / 8;
    for (int64_t item = t_beg + lb; item < t_end; item += nb) {
        const int e = batch_entry(bm, item);
        const EvalJob &J = jobs[bm.job[e]];
        if (item - bm.pre[e] >= J.counts[1]) continue;   // block-uniform
        const int32_t *tile = J.mix_tiles + 4 * (item - bm.pre[e]);
        const int key = tile[0], start = tile[1], count = tile[2];
        const int G = J.G, S = J.ew, p = J.p, pm = J.pm;
        const int l = key / G, g = key % G;
        const int P1 = p + 1;
        const int tl = J.sept ? l : 0;
        const bf16x8 *Tbase = (const bf16x8 *)J.mix_tab + ((size_t)tl * G + g) * S * (size_t)NA;
        const double *A0base = J.m2l_a0 + 2 * ((size_t)l * G + g) * S * (pm + 1);
        const bf16x8 *Bbase = (const bf16x8 *)J.mix_b + q;

        // E4 rows of the tile's targets -> srcs[slot][column] (4 threads per
        // target), then the list of slots that have any source.
        __syncthreads();   // the previous tile is done with the LDS
        {
            const int c = threadIdx.x >> 2, part = threadIdx.x & 3;
            const int32_t gc = c < count ? J.mix_list[start + c] : -1;
            for (int s = part; s < S; s += 4) srcs[s][c] = gc >= 0 ? J.e4[(int64_t)gc * S + s] : -1;
        }
        __syncthreads();
        if (threadIdx.x < S) {
            bool any = false;
            for (int c = 0; c < 64; ++c) any = any || srcs[threadIdx.x][c] >= 0;
            act[threadIdx.x] = any ? 1 : 0;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int k = 0;
            for (int s = 0; s < S; ++s)
                if (act[s]) act[k++] = (int8_t)s;
            nact = k;
        }
        __syncthreads();
        const int NS = nact;
        const int col = 16 * w + n;

        bf16x8 stage[PER];
        double a0row = 0.0;
        bf16x8 bcur[3 * KB], bnext[3 * KB];
        double a0cur = 0.0, a0next = 0.0;
        // Global loads of slot s: its matrix and monopole row into registers,
        // this lane's gathered source column into b.
        auto load_slot = [&](int s, bf16x8 *b, double &a0) {
            const bf16x8 *T = Tbase + (size_t)s * NA;
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int i = threadIdx.x + 256 * k;
                stage[k] = i < NA ? T[i] : zero8;
            }
            a0row = (threadIdx.x < NR && threadIdx.x < 2 * P1)
                        ? A0base[(size_t)s * 2 * (pm + 1) + threadIdx.x] : 0.0;
            const int32_t src = srcs[s][col];
            if (src >= 0) {
                const bf16x8 *Bs = Bbase + (int64_t)src * KB * 3 * 4;
#pragma unroll
                for (int k = 0; k < 3 * KB; ++k) b[k] = Bs[k * 4];
                a0 = J.mp[(int64_t)src * 2 * P1];
            } else {
#pragma unroll
                for (int k = 0; k < 3 * KB; ++k) b[k] = zero8;
                a0 = 0.0;
            }
        };
        auto store_slot = [&](int buf) {
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int i = threadIdx.x + 256 * k;
                if (i < NA) Ash[buf][i] = stage[k];
            }
            if (threadIdx.x < NR) A0s[buf][threadIdx.x] = a0row;
        };

        double acc[MT][4];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[mt][j] = 0.0;
        if (NS > 0) {
            load_slot(act[0], bcur, a0cur);
            store_slot(0);
        }
        __syncthreads();
        for (int i = 0; i < NS; ++i) {
            const int buf = i & 1;
            const bool more = i + 1 < NS;
            if (more) load_slot(act[i + 1], bnext, a0next);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    const bf16x8 *t3 = Ash[buf] + (mt * KB + kb) * 3 * 64;
                    const bf16x8 ah = t3[lane], am = t3[64 + lane], al = t3[128 + lane];
                    const bf16x8 bh = bcur[kb * 3 + 0], bmd = bcur[kb * 3 + 1], bl = bcur[kb * 3 + 2];
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bmd, c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bmd, c, 0, 0, 0);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    // monopole terms in FP64: a0 Log(c_T - c_S), -a0 delta^-m / m
                    const int row = 16 * mt + 4 * q + j;
                    acc[mt][j] += (double)c[j] + a0cur * A0s[buf][row];
                }
            }
            if (more) store_slot(buf ^ 1);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 3 * KB; ++k) bcur[k] = bnext[k];
            a0cur = a0next;
        }
        if (col < count) {
            const int32_t gid = J.mix_list[start + col];
            double *out = J.lc + (int64_t)gid * 2 * P1;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = 16 * mt + 4 * q + j;
                    if (row < 2 * P1) out[row] = acc[mt][j];
                }
        }
    }
}

void mixed_pointers(const Plan &P, const __bf16 **tab, const int32_t **tiles, const int32_t **list,
                    __bf16 **bsplit, int *MT, int *KB)
{
    MixedLayout m = layout_of(P);
    char *base = (char *)P.mixed;
    *bsplit = base ? (__bf16 *)(base + m.off_b) : nullptr;
    *tab = base ? (const __bf16 *)(base + m.off_tab) : nullptr;
    *tiles = base ? (const int32_t *)(base + m.off_tiles) : nullptr;
    *list = base ? (const int32_t *)(base + m.off_list) : nullptr;
    *MT = m.MT;
    *KB = m.KB;
}

// Split every multipole of levels >= 1 into three bfloat16 parts in the
// MFMA B-operand layout: thread per (cell, k-block, lane group q).
__global__ __launch_bounds__(256) void k_split_mp(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    far_field_priority();
    for (int64_t item = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; item < bm.pre[bm.n];
         item += (int64_t)gridDim.x * blockDim.x) {
        const int e = batch_entry(bm, item);
        const EvalJob &J = jobs[bm.job[e]];
        const int64_t it = item - bm.pre[e];
        const int q = (int)(it % 4), kb = (int)((it / 4) % J.KB);
        const int64_t cell = J.m2l_first + it / (4 * J.KB);
        const double *a = J.mp + cell * 2 * (J.p + 1);
        const bool src = (J.occ[cell] & 1) != 0;
        bf16x8 h, m, l;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int idx = 32 * kb + 8 * q + j;
            const float x = (src && idx < 2 * J.p) ? (float)a[2 + idx] : 0.0f;
            __bf16 hh, mm, ll;
            split3(x, hh, mm, ll);
            h[j] = hh;
            m[j] = mm;
            l[j] = ll;
        }
        bf16x8 *out = (bf16x8 *)J.mix_b + ((cell * J.KB + kb) * 3) * 4 + q;
        out[0] = h;
        out[4] = m;
        out[8] = l;
    }
}

void batch_split_mp(const EvalJob *jobs, const BatchMap &m, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    const int64_t threads = m.pre[m.n];
    const unsigned grid = (unsigned)std::min<int64_t>((threads + 255) / 256, 4096);
    hipLaunchKernelGGL(k_split_mp, dim3(grid), dim3(256), 0, s, jobs, m);
}

bool mixed_shape_supported(int MT, int KB)
{
    const int key = MT * 10 + KB;
    return key == 11 || key == 21 || key == 31 || key == 32 || key == 42 || key == 52 ||
           key == 53 || key == 63 || key == 73;
}

void batch_m2l_mixed(const EvalJob *jobs, const BatchMap &m, int MT, int KB, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    const dim3 grid((persistent_grid(m.pre[m.n], 16) + 7) / 8 * 8), block(256);
    switch (MT * 10 + KB) {
    case 11: hipLaunchKernelGGL((k_m2l_bf16x3<1, 1>), grid, block, 0, s, jobs, m); break;
    case 21: hipLaunchKernelGGL((k_m2l_bf16x3<2, 1>), grid, block, 0, s, jobs, m); break;
    case 31: hipLaunchKernelGGL((k_m2l_bf16x3<3, 1>), grid, block, 0, s, jobs, m); break;
    case 32: hipLaunchKernelGGL((k_m2l_bf16x3<3, 2>), grid, block, 0, s, jobs, m); break;
    case 42: hipLaunchKernelGGL((k_m2l_bf16x3<4, 2>), grid, block, 0, s, jobs, m); break;
    case 52: hipLaunchKernelGGL((k_m2l_bf16x3<5, 2>), grid, block, 0, s, jobs, m); break;
    case 53: hipLaunchKernelGGL((k_m2l_bf16x3<5, 3>), grid, block, 0, s, jobs, m); break;
    case 63: hipLaunchKernelGGL((k_m2l_bf16x3<6, 3>), grid, block, 0, s, jobs, m); break;
    case 73: hipLaunchKernelGGL((k_m2l_bf16x3<7, 3>), grid, block, 0, s, jobs, m); break;
    default: break;
    }
}

}  // namespace fmm
