// m2l_mixed.hip -- M2L target tiles (both forms) and the mixed form's M2L as
// BF16x3 split products on MFMA (gfx950).
//
// Greengard & Rokhlin (1987) Lemma 2.4, radius-scaled.  For one (level,
// target group) every target cell sees the same E4 offsets, so the M2L of a
// level runs per (level, group) over tiles of up to 16 target cells: the
// slot's offset-dependent scalings are staged once per tile and every
// target column of the tile shares them.  The tiles are built here at plan
// time for the FP64 MFMA kernel (m2l.hip) and the BF16x3 kernel below.
//
// MFMA 16x16x32 bf16 operand layout (lane l, j = 0..7 / 0..3):
//   A[i = l%16][k = 8(l/16)+j], B[k = 8(l/16)+j][n = l%16],
//   C[i = 4(l/16)+j][n = l%16].
#include <vector>

#include "eval.h"

namespace fmm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kTileT = 16;   // target cells per M2L tile (one MFMA column each)

struct TileLayout {
    int64_t max_tiles;   // bound on the tile count
    size_t off_tiles, off_order, off_list, off_cnt, off_keys, off_sort, bytes;   // byte offsets in P.mixed
};

// The M2L tile area of a plan: per-key counts and tile offsets, the tiles
// and their launch order, the cells of levels >= 1 sorted by (level, group),
// the sort keys and the sort's scratch.
static TileLayout layout_of(const Plan &P)
{
    TileLayout m;
    const int64_t ncell = P.n_cells;
    m.max_tiles = ncell / kTileT + 2 * (kMaxL + 1) * kMaxGroups + 2;
    const int64_t nsort = std::max(ncell + 1, m.max_tiles);
    size_t o = 0;
    m.off_cnt = o;   // cell counts/offsets and tile offsets: 256 each
    o += 2 * 256 * sizeof(int32_t);
    m.off_tiles = o;
    o += (size_t)m.max_tiles * 4 * sizeof(int32_t);
    o = (o + 255) & ~(size_t)255;
    m.off_order = o;
    o += (size_t)m.max_tiles * sizeof(int32_t);
    o = (o + 255) & ~(size_t)255;
    m.off_list = o;
    o += (size_t)(ncell + 1) * sizeof(int32_t);
    o = (o + 255) & ~(size_t)255;
    m.off_keys = o;   // sort keys: of the cells, then of the tiles
    o += (size_t)nsort * sizeof(uint32_t);
    o = (o + 255) & ~(size_t)255;
    m.off_sort = o;   // the radix sort's scratch
    o += radix_tmp_bytes(nsort);
    m.bytes = (o + 255) & ~(size_t)255;
    return m;
}

size_t mixed_bytes(const Plan &P)
{
    if (P.m2l_pm == 0) return 256;
    return layout_of(P).bytes + 256;
}

struct CellOffsets {
    int64_t v[kMaxL + 2];
};

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

// Sort key of every cell of levels >= 1: l G + g for cells with targets,
// 255 (after every real key) for the others; the value is the cell id.  A
// stable sort by this key lists each (level, group)'s target cells in cell
// order, i.e. in key order within the level, so a tile covers neighbouring
// cells and the tiles of one (level, group) walk the level in order (their
// E4 sources overlap, which keeps the gathered source rows in cache).
__global__ void k_group_keys(int64_t first, int64_t n_cells, int L, int G, CellOffsets cell_off,
                             const uint8_t *__restrict__ occ, const uint8_t *__restrict__ group,
                             uint32_t *__restrict__ keys, int32_t *__restrict__ vals)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t gid = first + i;
    if (gid >= n_cells) return;
    uint32_t key = 255;
    if (occ[gid] & 2) {
        int l = 1;
        while (l < L && gid >= cell_off.v[l + 1]) ++l;
        key = (uint32_t)(l * G + group[gid]);
    }
    keys[i] = key;
    vals[i] = (int32_t)gid;
}

// One block: turns the per-key cell counts into cell offsets (in place,
// off[K] = total), tile offsets toff[0..K] (ceil(count / T) tiles per key)
// and the tile total.
__global__ __launch_bounds__(256) void k_tile_plan(int K, int T, int32_t *__restrict__ cnt,
                                                   int32_t *__restrict__ toff,
                                                   int32_t *__restrict__ n_tiles)
{
    __shared__ int32_t sc[256], st[256];
    const int k = threadIdx.x;
    const int32_t c = k < K ? cnt[k] : 0;
    sc[k] = c;
    st[k] = (c + T - 1) / T;
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


// Launch order of the tiles: thread per tile slot t < bound; key = the
// tile's first cell (cell ids are level-major, and in key order within a
// level), slots past the device's tile count after every tile.
__global__ void k_tile_keys(int32_t bound, const int32_t *__restrict__ n_tiles, const int32_t *__restrict__ tiles,
                            const int32_t *__restrict__ list, uint32_t past, uint32_t *__restrict__ keys,
                            int32_t *__restrict__ order)
{
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= bound) return;
    keys[t] = t < *n_tiles ? (uint32_t)list[tiles[4 * t + 1]] : past;
    order[t] = t;
}

int mixed_setup(Plan &P)
{
    if (P.m2l_pm == 0 || P.geo.L < 1) return 0;
    const TileLayout m = layout_of(P);
    char *base = (char *)P.mixed;
    hipStream_t s = P.stream;
    const int G = P.tables.n_groups, L = P.geo.L;
    int32_t *cnt = (int32_t *)(base + m.off_cnt);
    int32_t *toff = cnt + 256;
    int32_t *list = (int32_t *)(base + m.off_list);
    int32_t *tiles = (int32_t *)(base + m.off_tiles);
    CellOffsets coff;
    for (int l = 0; l < kMaxL + 2; ++l) coff.v[l] = P.n_cells;
    for (int l = 0; l <= L; ++l) coff.v[l] = P.lev[l].cell_off;
    hipMemsetAsync(cnt, 0, 256 * sizeof(int32_t), s);
    const int64_t first = P.lev[1].cell_off, n = P.n_cells - first;
    const int K = L * G + G;   // keys l*G + g, l = 0..L (level 0 stays empty)
    if (n > 0)
        hipLaunchKernelGGL(k_group_count, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, first,
                           P.n_cells, L, G, coff, P.cell_occ, P.group, cnt);
    hipLaunchKernelGGL(k_tile_plan, dim3(1), dim3(256), 0, s, K, kTileT, cnt, toff, P.counts + 1);
    // sum_k ceil(c_k / T) <= (sum_k c_k) / T + (keys of levels >= 1)
    P.mixed_tiles = (int)(n / kTileT + (int64_t)L * G + 1);
    int32_t *order = (int32_t *)(base + m.off_order);
    uint32_t *keys = (uint32_t *)(base + m.off_keys);
    hipLaunchKernelGGL(k_tile_fill, dim3((unsigned)((P.mixed_tiles + 255) / 256)), dim3(256), 0, s,
                       K, kTileT, cnt, toff, P.counts + 1, tiles);
    if (n > 0) {
        hipLaunchKernelGGL(k_group_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, first, P.n_cells, L, G,
                           coff, P.cell_occ, P.group, keys, list);
        radix_sort(keys, list, n, 8, base + m.off_sort, s);
    }
    // Tiles ordered by their first cell: the tiles of every group of one
    // region of a level run together, so a source cell's multipole, read by
    // the E4 targets of all groups around it, is fetched once into the L2
    // rather than once per group.
    const int nt = P.mixed_tiles;
    int bits = 1;
    while (bits < 32 && ((uint64_t)1 << bits) <= (uint64_t)P.n_cells) ++bits;
    hipLaunchKernelGGL(k_tile_keys, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, nt, P.counts + 1, tiles, list,
                       (uint32_t)P.n_cells, keys, order);
    radix_sort(keys, order, nt, bits, base + m.off_sort, s);
    return hipGetLastError() != hipSuccess;
}


// ------------------------------------------------------------ factored form
// The mixed M2L as the FP64 MFMA kernel factors it (m2l.hip): for every E4
// pair b~ += D_out (H g - a_0 [0, 1/1, ..., 1/p]) + a_0 Log(c_T - c_S) e_0
// with g = D_in a, D_in = diag((-1/delta)^k), D_out = diag(delta^-m) and the
// offset-free binomial matrix H[m][k'] = C(m + k', k').  Here H g runs on
// v_mfma_f32_16x16x32_bf16 as BF16x3 split products with FP32 accumulation:
// H is split once into three bfloat16 parts and held in the A-operand
// registers for the whole kernel; each pair's scaled column g (formed in FP64
// from the FP64 multipole and the slot's D_in, then rounded to FP32) is split
// into three parts as the B operand, its Re and Im parts as two column sets.
// The six products with weight >= 2^-16 (hh, hm, mh, hl, lh, mm) are
// accumulated in FP32; the slot's result is scaled by D_out and added in
// FP64.  Only the gathered multipole rows travel per pair: no per-slot
// matrices.  A split by truncation, x = h + m + l with h the upper 16 bits of
// x, m those of x - h and l = x - h - m, is exact for every FP32 x (each part
// carries 8 of the 24 significand bits).  Tile and wave layout as in the FP64
// kernel: up to 16 target cells of one (level, group) per workgroup, the
// four waves taking the slots s = w mod 4, partial rows added in wave order.
//
// MFMA 16x16x32 bf16 layout (lane l, j = 0..7 / 0..3):
//   A[i = l%16][k = 8(l/16)+j], B[k = 8(l/16)+j][n = l%16],
//   C[i = 4(l/16)+j][n = l%16].

// Upper 16 bits of a and b as one bf16 pair (a in the low half).
__device__ __forceinline__ uint32_t hi_pair(float a, float b)
{
    return __builtin_amdgcn_perm(__float_as_uint(b), __float_as_uint(a), 0x07060302u);
}

__device__ __forceinline__ float trunc16(float x) { return __uint_as_float(__float_as_uint(x) & 0xFFFF0000u); }

// Three-way truncation split of eight FP32 values into bf16x8 parts.
__device__ __forceinline__ void split8(const float (&x)[8], bf16x8 &h, bf16x8 &m, bf16x8 &l)
{
    uint32_t ph[4], pm[4], pl[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float a = x[2 * j], b = x[2 * j + 1];
        const float ra = a - trunc16(a), rb = b - trunc16(b);
        const float sa = ra - trunc16(ra), sb = rb - trunc16(rb);
        ph[j] = hi_pair(a, b);
        pm[j] = hi_pair(ra, rb);
        pl[j] = hi_pair(sa, sb);
    }
    h = __builtin_bit_cast(bf16x8, ph);
    m = __builtin_bit_cast(bf16x8, pm);
    l = __builtin_bit_cast(bf16x8, pl);
}

template <int MT, int KB>
__global__ __launch_bounds__(256) void k_m2l_bf16x3f(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    far_field_priority();
    constexpr int W = 16 * MT > 32 * KB + 1 ? 16 * MT : 32 * KB + 1;   // table entries per slot
    constexpr int NR = 16 * MT;                                         // output rows per column
    constexpr int TAB_BYTES = kMaxSlots * W * 16, RED_BYTES = 4 * 16 * 2 * NR * 8;
    __shared__ __align__(16) char lds[TAB_BYTES > RED_BYTES ? TAB_BYTES : RED_BYTES];
    __shared__ double2 lgs[kMaxSlots];
    __shared__ int32_t srcs[kMaxSlots][16];
    double2 *tab = reinterpret_cast<double2 *>(lds);   // [slot][W]: (-1/delta)^k, zero beyond p
    double(*red)[16][2 * NR] = reinterpret_cast<double(*)[16][2 * NR]>(lds);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = lane & 15, q = lane >> 4;

    // H in the A-operand layout, split in three: rows m = 16 mt + n, columns
    // k' = 32 kb + 8 q + j.
    bf16x8 hh[MT][KB], hm[MT][KB], hl[MT][KB];
    {
        const double *binom = jobs[bm.job[0]].binom;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                float v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int m = 16 * mt + n, kp = 32 * kb + 8 * q + j;
                    v[j] = (m <= kMaxP && kp < kMaxP) ? (float)binom[(m + kp) * kBinomStride + kp] : 0.0f;
                }
                split8(v, hh[mt][kb], hm[mt][kb], hl[mt][kb]);
            }
    }
    // 1/m for the output rows (0 for m = 0); the sign (-1)^m of D_out is
    // (-1)^j, row m = 16 mt + 4 q + j.
    __shared__ double invm[NR];
    for (int i = threadIdx.x; i < NR; i += 256) invm[i] = i ? 1.0 / (double)i : 0.0;

    const int64_t total = bm.pre[bm.n];
    const int xcd = blockIdx.x % 8, lb = blockIdx.x / 8, nb = gridDim.x / 8;
    const int64_t t_beg = total * xcd / 8, t_end = total * (xcd + 1) / 8;
    for (int64_t item = t_beg + lb; item < t_end; item += nb) {
        const int e = batch_entry(bm, item);
        const EvalJob &J = jobs[bm.job[e]];
        if (item - bm.pre[e] >= J.counts[1]) continue;   // block-uniform
        const int32_t *tile = J.mix_tiles + 4 * J.mix_order[item - bm.pre[e]];
        const int key = tile[0], start = tile[1], count = tile[2];
        const int G = J.G, S = J.ew, p = J.p, pm = J.pm;
        const int l = key / G, g = key % G;
        const int P1 = p + 1;
        const size_t tab0 = ((size_t)l * G + g) * S;

        __syncthreads();   // the previous tile is done with the LDS
        for (int i = threadIdx.x; i < S * W; i += 256) {
            const int sl = i / W, k = i - sl * W;
            double2 v = make_double2(0.0, 0.0);
            if (k <= p) {
                const double *pw = J.m2l_pw + 2 * ((tab0 + sl) * (pm + 1) + k);
                v = make_double2(pw[0], pw[1]);
            }
            tab[i] = v;
        }
        for (int i = threadIdx.x; i < S; i += 256)
            lgs[i] = make_double2(J.m2l_lg[2 * (tab0 + i)], J.m2l_lg[2 * (tab0 + i) + 1]);
        for (int i = threadIdx.x; i < S * 16; i += 256) {
            const int c = i / S, sl = i - c * S;
            srcs[sl][c] = c < count ? J.e4[(int64_t)J.mix_list[start + c] * S + sl] : -1;
        }
        __syncthreads();

        double accr[MT][4], acci[MT][4];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) accr[mt][j] = acci[mt][j] = 0.0;
        for (int sl = w; sl < S; sl += 4) {
            const int32_t src = srcs[sl][n];
            if (!__any(src >= 0)) continue;
            const double2 *ts = tab + sl * W;
            const double *a = J.mp + (int64_t)(src >= 0 ? src : 0) * 2 * P1;
            const double a0 = src >= 0 ? a[0] : 0.0;
            bf16x8 brh[KB], brm[KB], brl[KB], bih[KB], bim[KB], bil[KB];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                float gr[8], gi[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int k = 32 * kb + 8 * q + j + 1;
                    double2 c = make_double2(0.0, 0.0);
                    if (src >= 0 && k <= p) c = *reinterpret_cast<const double2 *>(a + 2 * k);
                    const double2 d = ts[k];
                    gr[j] = (float)(c.x * d.x - c.y * d.y);
                    gi[j] = (float)(c.x * d.y + c.y * d.x);
                }
                split8(gr, brh[kb], brm[kb], brl[kb]);
                split8(gi, bih[kb], bim[kb], bil[kb]);
            }
            const double2 lg = lgs[sl];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                floatx4 yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    yr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hh[mt][kb], brh[kb], yr, 0, 0, 0);
                    yi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hh[mt][kb], bih[kb], yi, 0, 0, 0);
                    yr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hh[mt][kb], brm[kb], yr, 0, 0, 0);
                    yi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hh[mt][kb], bim[kb], yi, 0, 0, 0);
                    yr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hm[mt][kb], brh[kb], yr, 0, 0, 0);
                    yi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hm[mt][kb], bih[kb], yi, 0, 0, 0);
                    yr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hh[mt][kb], brl[kb], yr, 0, 0, 0);
                    yi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hh[mt][kb], bil[kb], yi, 0, 0, 0);
                    yr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hl[mt][kb], brh[kb], yr, 0, 0, 0);
                    yi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hl[mt][kb], bih[kb], yi, 0, 0, 0);
                    yr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hm[mt][kb], brm[kb], yr, 0, 0, 0);
                    yi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hm[mt][kb], bim[kb], yi, 0, 0, 0);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int m = 16 * mt + 4 * q + j;
                    const double2 d = ts[m];
                    const double dr = (j & 1) ? -d.x : d.x, di = (j & 1) ? -d.y : d.y;
                    const double y = fma(-a0, invm[m], (double)yr[j]);
                    const double z = (double)yi[j];
                    accr[mt][j] = fma(y, dr, fma(-z, di, accr[mt][j]));
                    acci[mt][j] = fma(y, di, fma(z, dr, acci[mt][j]));
                }
            }
            if (q == 0) {   // row 0 (register 0 of lane group 0): the log term
                accr[0][0] = fma(a0, lg.x, accr[0][0]);
                acci[0][0] = fma(a0, lg.y, acci[0][0]);
            }
        }
        __syncthreads();   // every wave is done with the table
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = 16 * mt + 4 * q + j;
                red[w][n][2 * m] = accr[mt][j];
                red[w][n][2 * m + 1] = acci[mt][j];
            }
        __syncthreads();
        for (int i = threadIdx.x; i < count * 2 * P1; i += 256) {
            const int c = i / (2 * P1), r = i - c * 2 * P1;
            const double v = ((red[0][c][r] + red[1][c][r]) + red[2][c][r]) + red[3][c][r];
            J.lc[(int64_t)J.mix_list[start + c] * 2 * P1 + r] = v;
        }
    }
}

// (MT, KB) of the factored form for order p: MT = ceil((p+1)/16), KB = ceil(p/32).
int m2l_bf16x3f_class(int p) { return (p >= 1 && p <= 47) ? ((p + 1 + 15) / 16) * 10 + (p + 31) / 32 : 0; }

void batch_m2l_bf16x3f(const EvalJob *jobs, const BatchMap &m, int p, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    const dim3 grid((persistent_grid(m.pre[m.n], 12) + 7) / 8 * 8), block(256);
    switch (m2l_bf16x3f_class(p)) {
    case 11: hipLaunchKernelGGL((k_m2l_bf16x3f<1, 1>), grid, block, 0, s, jobs, m); break;
    case 21: hipLaunchKernelGGL((k_m2l_bf16x3f<2, 1>), grid, block, 0, s, jobs, m); break;
    case 31: hipLaunchKernelGGL((k_m2l_bf16x3f<3, 1>), grid, block, 0, s, jobs, m); break;
    case 32: hipLaunchKernelGGL((k_m2l_bf16x3f<3, 2>), grid, block, 0, s, jobs, m); break;
    default: break;
    }
}
void tile_pointers(const Plan &P, const int32_t **tiles, const int32_t **order, const int32_t **list)
{
    const TileLayout m = layout_of(P);
    char *base = (char *)P.mixed;
    *tiles = base ? (const int32_t *)(base + m.off_tiles) : nullptr;
    *order = base ? (const int32_t *)(base + m.off_order) : nullptr;
    *list = base ? (const int32_t *)(base + m.off_list) : nullptr;
}

}  // namespace fmm
