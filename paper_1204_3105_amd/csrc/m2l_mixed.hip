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

constexpr int kTileT = 64;   // targets per workgroup (4 waves x 16 columns)

struct MixedLayout {
    int MT, KB;          // 16-row M tiles, 32-deep K blocks
    int tab_levels;      // 1 (level-invariant) or L+1 (septree)
    int G, S, pm;
    size_t tab_elems;    // bf16 elements per (level, group, slot) table
    int n_tiles;
    size_t off_tab, off_tiles, off_list, off_cnt;   // byte offsets in P.mixed
};

static MixedLayout layout_of(const Plan &P)
{
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
    o += (size_t)m.tab_levels * m.G * m.S * m.tab_elems * 2;
    o = (o + 255) & ~(size_t)255;
    m.off_cnt = o;
    o += 2 * 256 * sizeof(int32_t);
    m.off_tiles = o;
    int64_t ncell = P.n_cells;
    o += (size_t)(ncell / kTileT + 2 * (kMaxL + 1) * kMaxGroups + 2) * 4 * sizeof(int32_t);
    o = (o + 255) & ~(size_t)255;
    m.off_list = o;
    o += (size_t)(ncell + 1) * sizeof(int32_t);
    m.tab_elems = m.tab_elems;
    return m;
}

size_t mixed_bytes(const Plan &P)
{
    if (P.m2l_pm == 0) return 256;
    MixedLayout m = layout_of(P);
    return m.off_list + (size_t)(P.n_cells + 1) * sizeof(int32_t) + 256;
}

struct CellOffsets {
    int64_t v[kMaxL + 2];
};
struct SlotCounts {
    int v[kMaxGroups];
};

__device__ __forceinline__ void split3(float x, __bf16 &h, __bf16 &m, __bf16 &l)
{
    h = (__bf16)x;
    const float r1 = x - (float)h;
    m = (__bf16)r1;
    const float r2 = r1 - (float)m;
    l = (__bf16)r2;
}

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

// Group target cells of levels >= 1 by (level, group).
__global__ void k_group_count(int64_t first, int64_t n_cells, int L, int G, CellOffsets cell_off,
                              const uint8_t *__restrict__ occ,
                              const uint8_t *__restrict__ group, int32_t *__restrict__ cnt)
{
    const int64_t gid = first + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid >= n_cells || !(occ[gid] & 2)) return;
    int l = 1;
    while (l < L && gid >= cell_off.v[l + 1]) ++l;
    atomicAdd(&cnt[l * G + group[gid]], 1);
}

__global__ void k_group_scatter(int64_t first, int64_t n_cells, int L, int G, CellOffsets cell_off,
                                const uint8_t *__restrict__ occ,
                                const uint8_t *__restrict__ group, const int32_t *__restrict__ off,
                                int32_t *__restrict__ cursor, int32_t *__restrict__ list)
{
    const int64_t gid = first + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid >= n_cells || !(occ[gid] & 2)) return;
    int l = 1;
    while (l < L && gid >= cell_off.v[l + 1]) ++l;
    const int key = l * G + group[gid];
    list[off[key] + atomicAdd(&cursor[key], 1)] = (int32_t)gid;
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
    hipMemsetAsync(cnt, 0, 2 * 256 * sizeof(int32_t), s);
    const int64_t first = P.lev[1].cell_off, n = P.n_cells - first;
    if (n > 0)
        hipLaunchKernelGGL(k_group_count, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, first,
                           P.n_cells, L, G, coff, P.cell_occ, P.group, cnt);
    std::vector<int32_t> hc(256, 0);
    hipMemcpyAsync(hc.data(), cnt, 256 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    hipStreamSynchronize(s);
    std::vector<int32_t> off(256, 0), ht;
    int32_t acc = 0;
    for (int k = 0; k < (L + 1) * G; ++k) {
        off[k] = acc;
        for (int st = 0; st < hc[k]; st += kTileT) {
            ht.push_back(k);
            ht.push_back(acc + st);
            ht.push_back(std::min(kTileT, hc[k] - st));
            ht.push_back(0);
        }
        acc += hc[k];
    }
    P.mixed_tiles = (int)(ht.size() / 4);
    hipMemcpy(cnt, off.data(), 256 * sizeof(int32_t), hipMemcpyHostToDevice);
    hipMemsetAsync(cursor, 0, 256 * sizeof(int32_t), s);
    if (!ht.empty()) hipMemcpy(tiles, ht.data(), ht.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (n > 0)
        hipLaunchKernelGGL(k_group_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, first,
                           P.n_cells, L, G, coff, P.cell_occ, P.group, cnt, cursor, list);
    // Split translation matrices.
    SlotCounts counts;
    for (int g = 0; g < kMaxGroups; ++g) counts.v[g] = g < G ? P.tables.e4_count[g] : 0;
    const int nb = m.tab_levels * G * m.S * m.MT * m.KB;
    hipLaunchKernelGGL(k_build_mixed_tables, dim3(nb), dim3(64), 0, s, P.p, m.MT, m.KB, G, m.S, m.pm,
                       P.geo.tiling == kSept ? 1 : 0, counts, P.m2l_pw, P.binom,
                       (__bf16 *)(base + m.off_tab));
    return hipGetLastError() != hipSuccess;
}

template <int MT, int KB>
__global__ __launch_bounds__(256) void k_m2l_bf16x3(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = lane % 16, q = lane / 16;
    for (int64_t item = blockIdx.x; item < bm.pre[bm.n]; item += gridDim.x) {
        const int e = batch_entry(bm, item);
        const EvalJob &J = jobs[bm.job[e]];
        const int32_t *tile = J.mix_tiles + 4 * (item - bm.pre[e]);
        const int key = tile[0], start = tile[1], count = tile[2];
        const int G = J.G, S = J.ew, p = J.p, pm = J.pm;
        const int l = key / G, g = key % G;
        const int col = 16 * w + n;
        const bool valid = col < count;
        const int32_t gid = valid ? J.mix_list[start + col] : -1;
        const int P1 = p + 1, twoP = 2 * p;
        const int tl = J.sept ? l : 0;
        double acc[MT][4];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[mt][j] = 0.0;
        const size_t tab_elems = (size_t)MT * KB * 3 * 512;
        for (int s = 0; s < S; ++s) {
            const int32_t src = valid ? J.e4[(int64_t)gid * S + s] : -1;
            // Wave-uniform skip when no lane has a source in this slot.
            if (__ballot(src >= 0) == 0ull) continue;
            const double *a = src >= 0 ? J.mp + (int64_t)src * 2 * P1 : nullptr;
            bf16x8 bh[KB], bmd[KB], bl[KB];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int idx = 32 * kb + 8 * q + j;
                    float x = 0.0f;
                    if (a && idx < twoP) x = (float)a[2 + idx];
                    __bf16 h, m, lo;
                    split3(x, h, m, lo);
                    bh[kb][j] = h;
                    bmd[kb][j] = m;
                    bl[kb][j] = lo;
                }
            }
            const bf16x8 *T = (const bf16x8 *)(J.mix_tab + (((size_t)tl * G + g) * S + s) * tab_elems);
            const size_t pidx = ((size_t)l * G + g) * S + s;
            const double *pw = J.m2l_pw + 2 * pidx * (pm + 1);
            const double a0 = a ? a[0] : 0.0;
            const double lgr = J.m2l_lg[2 * pidx], lgi = J.m2l_lg[2 * pidx + 1];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    const bf16x8 *t3 = T + (size_t)((mt * KB + kb) * 3) * 64;
                    const bf16x8 ah = t3[lane], am = t3[64 + lane], al = t3[128 + lane];
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[kb], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bmd[kb], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh[kb], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[kb], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[kb], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bmd[kb], c, 0, 0, 0);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = 16 * mt + 4 * q + j;
                    const int m = row >> 1;
                    double t0 = 0.0;
                    if (a && m <= p) {
                        if (m == 0) {
                            t0 = a0 * ((row & 1) ? lgi : lgr);
                        } else {
                            // -a0/m delta^-m, delta^-m = (-1)^m (-1/delta)^m
                            double d = pw[2 * m + (row & 1)];
                            if (m & 1) d = -d;
                            t0 = -a0 / (double)m * d;
                        }
                    }
                    acc[mt][j] += (double)c[j] + t0;
                }
            }
        }
        if (valid) {
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
                    int *MT, int *KB)
{
    MixedLayout m = layout_of(P);
    const char *base = (const char *)P.mixed;
    *tab = base ? (const __bf16 *)(base + m.off_tab) : nullptr;
    *tiles = base ? (const int32_t *)(base + m.off_tiles) : nullptr;
    *list = base ? (const int32_t *)(base + m.off_list) : nullptr;
    *MT = m.MT;
    *KB = m.KB;
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
    const dim3 grid(persistent_grid(m.pre[m.n], 16)), block(256);
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
