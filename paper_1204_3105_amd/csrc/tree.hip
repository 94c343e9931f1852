// tree.hip -- per-level occupied cells, centres and interaction lists.
//
// Hierarchical addressing (paper Sec. 4): the level-l key of a leaf key is
// its first l digits (Parent = drop a digit, Children = append one).  The
// occupied cells of every level are found from the sorted leaf keys; each
// gets a global id, a source range, a target range and its centre
// (CellCenter: quadtree cell centre; septree Sec. 5 zero-extended GBT
// components summed as integer lattice vectors; triangle-quadtree Sec. 6
// translations F(t, i) summed in integer units).
//
// Interaction lists (Sec. 4, Neighbors and NeighborsE4; the E4 set is the
// children of the parent's closed neighbourhood minus the cell's own closed
// neighbourhood) are built from per-tiling offset tables: a cell's
// neighbourhood is the same configuration of relative positions for every
// cell of one group (quadtree: child digit; septree: child digit; triangle-
// quadtree: child type and orientation).  A relative position is turned
// back into a key by the tiling's exact integer encoder (Morton, GBT digits
// by division by beta, triangle descent by integer nearest centroid), and a
// position outside the root gives no cell, as the paper drops neighbours
// beyond the root (Sec. 5 septree "less than 7^l"; Sec. 6 no ancestor with a
// sibling).  This file is compiled with -ffp-contract=off so the centres
// are the exact products of the integer coordinates with the scale.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "fmm_internal.h"

namespace fmm {

struct Levels {
    LevelInfo l[kMaxL + 1];
    uint32_t div[kMaxL + 1];   // septree: 7^(L-l)
    int L;
};

static Levels make_levels(const GeoParams &g, const LevelInfo *lev)
{
    Levels s;
    s.L = g.L;
    for (int l = 0; l <= g.L; ++l) {
        s.l[l] = lev[l];
        uint32_t d = 1;
        for (int k = 0; k < g.L - l; ++k) d *= 7u;
        s.div[l] = d;
    }
    return s;
}

__device__ __forceinline__ uint32_t level_key(int tiling, const Levels &s, uint32_t leaf, int l)
{
    if (tiling == kSept) return leaf / s.div[l];
    return leaf >> (2 * (s.L - l));
}

// ------------------------------------------------------------ occupancy
__global__ void k_mark_cells(int tiling, Levels s, const uint32_t *__restrict__ key, int64_t n,
                             int32_t bit, int32_t *__restrict__ flags)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t k = key[i];
    uint32_t kp = i > 0 ? key[i - 1] : 0xffffffffu;
    if (i > 0 && kp == k) return;   // same leaf, so the same cell at every level
    for (int l = 0; l <= s.L; ++l) {
        uint32_t lk = level_key(tiling, s, k, l);
        bool start = (i == 0) || level_key(tiling, s, kp, l) != lk;
        if (start) atomicOr(&flags[s.l[l].dense_off + lk], bit);
    }
}

void launch_mark_cells(const GeoParams &g, const LevelInfo *lev, const uint32_t *key, int64_t n,
                       uint8_t bit, int32_t *flags, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mark_cells, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g.tiling,
                       make_levels(g, lev), key, n, (int32_t)bit, flags);
}

__global__ void k_flags_to_ones(const int32_t *__restrict__ flags, int64_t n, int32_t *__restrict__ ones)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) ones[i] = flags[i] != 0;
}

void launch_flags_to_ids(int32_t *flags_ones, int64_t n, hipStream_t s)
{
    // flags_ones[0..n) = flags, flags_ones[n..2n) receives 0/1
    if (n <= 0) return;
    hipLaunchKernelGGL(k_flags_to_ones, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       flags_ones, n, flags_ones + n);
}

__device__ __forceinline__ int level_of_dense(const Levels &s, int64_t j)
{
    int l = 0;
    while (l < s.L && j >= s.l[l + 1].dense_off) ++l;
    return l;
}

__device__ __forceinline__ int level_of_cell(const Levels &s, int64_t gid)
{
    int l = 0;
    while (l < s.L && gid >= s.l[l + 1].cell_off) ++l;
    return l;
}

__global__ void k_compact(Levels s, const int32_t *__restrict__ flags, const int32_t *__restrict__ ids,
                          int64_t n, int32_t *__restrict__ dense, uint32_t *__restrict__ cell_key,
                          uint8_t *__restrict__ occ, int32_t *__restrict__ sb, int32_t *__restrict__ se,
                          int32_t *__restrict__ tb, int32_t *__restrict__ te, double *__restrict__ zero,
                          int n_zero)
{
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j < n_zero) zero[j] = 0.0;   // cleared on the way (see launch_compact)
    if (j >= n) return;
    int32_t f = flags[j];
    if (!f) {
        dense[j] = -1;
        return;
    }
    int l = level_of_dense(s, j);
    int32_t gid = ids[j];
    dense[j] = gid;
    cell_key[gid] = (uint32_t)(j - s.l[l].dense_off);
    occ[gid] = (uint8_t)f;
    sb[gid] = se[gid] = 0;   // ranges of absent kinds stay empty
    if (tb) tb[gid] = te[gid] = 0;
}

void launch_compact(const GeoParams &g, const LevelInfo *lev, int64_t dense_total,
                    const int32_t *flags, const int32_t *ids, int32_t *dense, uint32_t *cell_key,
                    uint8_t *occ, int32_t *sb, int32_t *se, int32_t *tb, int32_t *te, double *zero,
                    int n_zero, hipStream_t s)
{
    const int64_t m = dense_total > n_zero ? dense_total : n_zero;
    hipLaunchKernelGGL(k_compact, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                       make_levels(g, lev), flags, ids, dense_total, dense, cell_key, occ, sb, se,
                       tb, te, zero, n_zero);
}

// out[l] = first cell id of level l (l = 0..L), out[L+1] = cell count,
// out[L+2] = points outside the root.
__global__ void k_gather_bounds(Levels s, const int32_t *__restrict__ ids,
                                const int32_t *__restrict__ total, const int32_t *__restrict__ bad,
                                int32_t *__restrict__ out)
{
    const int l = threadIdx.x;
    if (l <= s.L) out[l] = ids[s.l[l].dense_off];
    if (l == 0) {
        out[s.L + 1] = *total;
        out[s.L + 2] = *bad;
    }
}

void launch_gather_bounds(const LevelInfo *lev, int L, const int32_t *ids, const int32_t *total,
                          const int32_t *bad, int32_t *out, hipStream_t s)
{
    Levels lv;
    lv.L = L;
    for (int l = 0; l <= L; ++l) lv.l[l] = lev[l];
    hipLaunchKernelGGL(k_gather_bounds, dim3(1), dim3(64), 0, s, lv, ids, total, bad, out);
}

__global__ void k_ranges(int tiling, Levels s, const uint32_t *__restrict__ key, int64_t n,
                         const int32_t *__restrict__ dense, int32_t *__restrict__ b,
                         int32_t *__restrict__ e)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t k = key[i];
    uint32_t kp = i > 0 ? key[i - 1] : 0u;
    uint32_t kn = i + 1 < n ? key[i + 1] : 0u;
    // inside a leaf's run (same leaf key on both sides): no cell starts or
    // ends here at any level
    if (i > 0 && i + 1 < n && kp == k && kn == k) return;
    for (int l = 0; l <= s.L; ++l) {
        uint32_t lk = level_key(tiling, s, k, l);
        int32_t gid = dense[s.l[l].dense_off + lk];
        if (i == 0 || level_key(tiling, s, kp, l) != lk) b[gid] = (int32_t)i;
        if (i + 1 == n || level_key(tiling, s, kn, l) != lk) e[gid] = (int32_t)(i + 1);
    }
}

void launch_cell_ranges(const GeoParams &g, const LevelInfo *lev, const uint32_t *key, int64_t n,
                        const int32_t *dense, int32_t *b, int32_t *e, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g.tiling,
                       make_levels(g, lev), key, n, dense, b, e);
}

// ------------------------------------------------------------ positions
__device__ __forceinline__ void quad_split(uint32_t key, int l, int64_t &ix, int64_t &iy)
{
    uint32_t x = 0, y = 0;
    for (int b = 0; b < l; ++b) {
        x |= ((key >> (2 * b)) & 1u) << b;
        y |= ((key >> (2 * b + 1)) & 1u) << b;
    }
    ix = x;
    iy = y;
}

__device__ __forceinline__ uint32_t quad_join(int64_t ix, int64_t iy, int l)
{
    uint32_t k = 0;
    for (int b = 0; b < l; ++b) {
        k |= (uint32_t)((ix >> b) & 1) << (2 * b);
        k |= (uint32_t)((iy >> b) & 1) << (2 * b + 1);
    }
    return k;
}

// Eisenstein value a + b w of a level-l septree key in level-l units:
// sum_i digit_i beta^i, least significant digit first (|a|, |b| < 2^16 for
// the 11 levels a 32-bit key holds).
__device__ __forceinline__ void sept_value(uint32_t key, int l, int64_t &a, int64_t &b)
{
    const int da[7] = {0, 1, 0, -1, -1, 0, 1};
    const int db[7] = {0, 0, 1, 1, 0, -1, -1};
    int32_t va = 0, vb = 0, qa = 1, qb = 0;   // q = beta^i
    for (int i = 0; i < l; ++i) {
        const int d = (int)(key % 7u);
        key /= 7u;
        // v += q * digit; (qa + qb w)(x + y w) = (qa x - qb y) + (qa y + qb x + qb y) w
        va += qa * da[d] - qb * db[d];
        vb += qa * db[d] + qb * da[d] + qb * db[d];
        // q *= beta, beta (a + b w) = (a - 2b) + (2a + 3b) w
        const int32_t na = qa - 2 * qb, nb = 2 * qa + 3 * qb;
        qa = na;
        qb = nb;
    }
    a = va;
    b = vb;
}

// GBT digits of a + b w (level-l units, ndig digits), -1 if it needs more.
// After the digit is removed, (a + b w)(3 - 2w) is divisible by 7 = beta
// conj(beta); the exact quotient is the product with 7^-1 mod 2^32.
__device__ __forceinline__ int64_t sept_encode(int32_t a, int32_t b, int ndig)
{
    const int rdig[7] = {0, 1, 3, 2, 5, 6, 4};
    const int da[7] = {0, 1, 0, -1, -1, 0, 1};
    const int db[7] = {0, 0, 1, 1, 0, -1, -1};
    constexpr uint32_t kInv7 = 0xB6DB6DB7u;
    uint32_t key = 0, pw = 1;
    for (int i = 0; i < ndig; ++i) {
        int32_t r = (a + 3 * b) % 7;
        if (r < 0) r += 7;
        const int d = rdig[r];
        a -= da[d];
        b -= db[d];
        const uint32_t na = (uint32_t)(3 * a + 2 * b), nb = (uint32_t)(b - 2 * a);
        a = (int32_t)(na * kInv7);
        b = (int32_t)(nb * kInv7);
        key += (uint32_t)d * pw;
        pw *= 7u;
    }
    if (a != 0 || b != 0) return -1;
    return key;
}

// Triangle centre in integer units (x = U sqrt3/2 r, y = V r/2), orientation.
__device__ __forceinline__ void tri_units(uint32_t key, int l, int L, int64_t &U, int64_t &V, int &o)
{
    int64_t u = 0, v = 0;
    int up = 1;
    for (int i = 1; i <= l; ++i) {
        int t = (int)((key >> (2 * (l - i))) & 3u);
        int64_t R = (int64_t)1 << (L - i);
        if (t == 0) {
            up = -up;
        } else if (t == 1) {
            v += 2 * up * R;
        } else if (t == 2) {
            u -= R;
            v -= up * R;
        } else {
            u += R;
            v -= up * R;
        }
    }
    U = u;
    V = v;
    o = up;
}

// Key of the level-l triangle whose centroid is (U, V); -1 if outside the
// root.  Descent by the lines that split a triangle into its children: with
// du = U - c_u, dv = o (V - c_v) and R the child offset unit, the apex child
// (type 1) holds dv > R, the two base corners (types 2, 3) hold
// 3 du + dv < -2R and -3 du + dv < -2R, and the inverted centre (type 0) the
// rest.  Centroids of finer cells never lie on these lines.
__device__ __forceinline__ int64_t tri_encode(int32_t U, int32_t V, int l, int L)
{
    const int32_t lim = 1 << (L + 1);
    if (!(V > -(1 << L) && 3 * U + V < lim && -3 * U + V < lim)) return -1;
    int32_t cu = 0, cv = 0;
    uint32_t key = 0;
    int up = 1;
    for (int i = 1; i <= l; ++i) {
        const int32_t R = 1 << (L - i);
        const int32_t du = U - cu, dv = up * (V - cv);
        uint32_t t;
        if (dv > R) {
            t = 1;
            cv += 2 * up * R;
        } else if (3 * du + dv < -2 * R) {
            t = 2;
            cu -= R;
            cv -= up * R;
        } else if (-3 * du + dv < -2 * R) {
            t = 3;
            cu += R;
            cv -= up * R;
        } else {
            t = 0;
            up = -up;
        }
        key = key * 4u + t;
    }
    if (cu != U || cv != V) return -1;
    return key;
}

// ------------------------------------------------------------ centres
__global__ void k_cell_geometry(GeoParams g, Levels s, int64_t n_cells,
                                const uint32_t *__restrict__ cell_key,
                                const int32_t *__restrict__ dense, double *__restrict__ cx,
                                double *__restrict__ cy, int32_t *__restrict__ parent,
                                uint8_t *__restrict__ group)
{
    int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid >= n_cells) return;
    int l = level_of_cell(s, gid);
    uint32_t key = cell_key[gid];
    double x, y;
    uint8_t grp = 0;
    if (g.tiling == kQuad) {
        int64_t ix, iy;
        quad_split(key, l, ix, iy);
        double h = ldexp(g.size, -l);
        x = g.ox + ((double)ix + 0.5) * h;
        y = g.oy + ((double)iy + 0.5) * h;
        grp = (uint8_t)(key & 3u);
    } else if (g.tiling == kSept) {
        int64_t a, b;
        sept_value(key, l, a, b);
        // level-l units -> leaf units: multiply by beta^(L-l)
        for (int k = 0; k < g.L - l; ++k) {
            int64_t na = a - 2 * b, nb = 2 * a + 3 * b;
            a = na;
            b = nb;
        }
        const double r = g.size;
        x = g.ox + (3.0 * r * (double)a) / 2.0;
        y = g.oy + (r * g.s3 * (2.0 * (double)b + (double)a)) / 2.0;
        grp = (uint8_t)(key % 7u);
    } else {
        int64_t U, V;
        int o;
        tri_units(key, l, g.L, U, V, o);
        const double r = g.size;
        double ax = (g.s3 * r) / 2.0, ay = r / 2.0;
        x = g.ox + (double)U * ax;
        y = g.oy + (double)V * ay;
        grp = (uint8_t)((key & 3u) + (o < 0 ? 4 : 0));
    }
    if (l == 0) grp = 0;
    cx[gid] = x;
    cy[gid] = y;
    group[gid] = grp;
    if (l == 0) {
        parent[gid] = -1;
    } else {
        uint32_t pk = key / (uint32_t)base_of(g.tiling);
        parent[gid] = dense[s.l[l - 1].dense_off + pk];
    }
}

void launch_cell_geometry(const GeoParams &g, const LevelInfo *lev, int64_t n_cells,
                          const uint32_t *cell_key, const int32_t *dense, const int32_t *sb,
                          const int32_t *se, const int32_t *tb, const int32_t *te, double *cx,
                          double *cy, int32_t *parent, uint8_t *group, uint8_t *occ,
                          hipStream_t s)
{
    (void)sb;
    (void)se;
    (void)tb;
    (void)te;
    (void)occ;
    if (n_cells <= 0) return;
    hipLaunchKernelGGL(k_cell_geometry, dim3((unsigned)((n_cells + 255) / 256)), dim3(256), 0, s, g,
                       make_levels(g, lev), n_cells, cell_key, dense, cx, cy, parent, group);
}

// ------------------------------------------------------------ lists
struct DevTables {
    int e4_width, near_width;
    int e4[kMaxGroups][kMaxSlots][2];
    int e4_count[kMaxGroups];
    int near[2][kNearSlots][2];
    int near_count[2];
};

// Global id of the source-occupied cell at relative position `off` from a
// cell at (pa, pb) on level l; -1 if none.
__device__ __forceinline__ int32_t lookup(const GeoParams &g, const Levels &s,
                                          const int32_t *__restrict__ dense,
                                          const uint8_t *__restrict__ occ, int l, int32_t pa,
                                          int32_t pb, int da, int db)
{
    int64_t key;
    if (g.tiling == kQuad) {
        const int32_t x = pa + da, y = pb + db, n = 1 << l;
        if (x < 0 || y < 0 || x >= n || y >= n) return -1;
        key = quad_join(x, y, l);
    } else if (g.tiling == kSept) {
        key = sept_encode(pa + da, pb + db, l);
    } else {
        const int32_t R = 1 << (g.L - l);
        key = tri_encode(pa + da * R, pb + db * R, l, g.L);
    }
    if (key < 0) return -1;
    int32_t gid = dense[s.l[l].dense_off + key];
    if (gid < 0 || !(occ[gid] & 1)) return -1;
    return gid;
}

// Position of a cell in lattice units of its level (quadtree cell indices,
// septree Eisenstein value, triangle centroid units) and its orientation.
__device__ __forceinline__ void cell_position(const GeoParams &g, uint32_t key, int l, int32_t &pa,
                                              int32_t &pb, int &orient)
{
    int64_t qa, qb;
    orient = 1;
    if (g.tiling == kQuad) quad_split(key, l, qa, qb);
    else if (g.tiling == kSept) sept_value(key, l, qa, qb);
    else tri_units(key, l, g.L, qa, qb, orient);
    pa = (int32_t)qa;
    pb = (int32_t)qb;
}

// One thread per (cell, E4 slot): slot k of a target cell on level >= 1 is
// the source-occupied cell at the group's k-th offset, or -1 (every other
// slot and every other cell's row is -1).  Threads are
// many and independent, so the dependent dense-map loads of all slots are in
// flight together.
__global__ void k_lists_e4(GeoParams g, Levels s, DevTables t, int64_t first, int64_t n_slots,
                           const uint32_t *__restrict__ cell_key, const uint8_t *__restrict__ group,
                           const uint8_t *__restrict__ occ, const int32_t *__restrict__ dense,
                           int32_t *__restrict__ e4)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_slots) return;
    const int64_t gid = first + i / t.e4_width;
    const int k = (int)(i % t.e4_width);
    const int grp = group[gid];
    int32_t v = -1;
    const int l = level_of_cell(s, gid);
    if (l >= 1 && (occ[gid] & 2) && k < t.e4_count[grp]) {
        int32_t pa, pb;
        int orient;
        cell_position(g, cell_key[gid], l, pa, pb, orient);
        v = lookup(g, s, dense, occ, l, pa, pb, t.e4[grp][k][0], t.e4[grp][k][1]);
    }
    e4[gid * (int64_t)t.e4_width + k] = v;
}

// One thread per (leaf, near slot): the closed neighbourhood of each target
// leaf, slot 0 the leaf itself, restricted to source-occupied cells.
__global__ void k_lists_near(GeoParams g, Levels s, DevTables t, int64_t n_slots,
                             const uint32_t *__restrict__ cell_key, const uint8_t *__restrict__ occ,
                             const int32_t *__restrict__ dense, int32_t *__restrict__ near)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_slots) return;
    const int64_t li = i / t.near_width;
    const int k = (int)(i % t.near_width);
    const int64_t gid = s.l[s.L].cell_off + li;
    int32_t v = -1;
    if (occ[gid] & 2) {
        int32_t pa, pb;
        int orient;
        cell_position(g, cell_key[gid], s.L, pa, pb, orient);
        const int oi = orient < 0 ? 1 : 0;
        if (k < t.near_count[oi])
            v = lookup(g, s, dense, occ, s.L, pa, pb, t.near[oi][k][0], t.near[oi][k][1]);
    }
    near[i] = v;
}

void launch_lists(const GeoParams &g, const LevelInfo *lev, const ListTables &tab, int64_t n_cells,
                  const uint32_t *cell_key, const uint8_t *group, const uint8_t *occ,
                  const int32_t *dense, int32_t *e4, int32_t *near, hipStream_t s)
{
    if (n_cells <= 0) return;
    DevTables t;
    t.e4_width = tab.e4_width;
    t.near_width = tab.near_width;
    for (int a = 0; a < kMaxGroups; ++a) {
        t.e4_count[a] = tab.e4_count[a];
        for (int k = 0; k < kMaxSlots; ++k) {
            t.e4[a][k][0] = tab.e4[a][k][0];
            t.e4[a][k][1] = tab.e4[a][k][1];
        }
    }
    for (int a = 0; a < 2; ++a) {
        t.near_count[a] = tab.near_count[a];
        for (int k = 0; k < kNearSlots; ++k) {
            t.near[a][k][0] = tab.near[a][k][0];
            t.near[a][k][1] = tab.near[a][k][1];
        }
    }
    const Levels lv = make_levels(g, lev);
    const int64_t ne = n_cells * (int64_t)t.e4_width;
    hipLaunchKernelGGL(k_lists_e4, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, g, lv, t,
                       (int64_t)0, ne, cell_key, group, occ, dense, e4);
    const int64_t nn = lev[g.L].n * (int64_t)t.near_width;
    if (nn > 0)
        hipLaunchKernelGGL(k_lists_near, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, g, lv,
                           t, nn, cell_key, occ, dense, near);
}

// ------------------------------------------------------------ local coords
__global__ void k_local_coords(const double *__restrict__ x, const double *__restrict__ y,
                               const uint32_t *__restrict__ key, int64_t n, int32_t leaf_dense_off,
                               const int32_t *__restrict__ dense, const double *__restrict__ cx,
                               const double *__restrict__ cy, float *__restrict__ xl,
                               float *__restrict__ yl)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t gid = dense[leaf_dense_off + key[i]];
    xl[i] = (float)(x[i] - cx[gid]);
    yl[i] = (float)(y[i] - cy[gid]);
}

void launch_local_coords(const double *x, const double *y, const uint32_t *key, int64_t n,
                         const GeoParams &g, const LevelInfo *lev, const int32_t *dense,
                         const double *cx, const double *cy, float *xl, float *yl, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_local_coords, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, key,
                       n, (int32_t)lev[g.L].dense_off, dense, cx, cy, xl, yl);
}

// ------------------------------------------------------------ near items
__global__ void k_near_counts(int64_t off, int64_t n, const int32_t *__restrict__ tb,
                              const int32_t *__restrict__ te, int32_t *__restrict__ counts)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t nt = te[off + i] - tb[off + i];
    counts[i] = (nt + kChunk - 1) / kChunk;
}

void launch_near_items(const LevelInfo *lev, int L, const int32_t *tb, const int32_t *te,
                       int32_t *counts, hipStream_t s)
{
    int64_t n = lev[L].n;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_near_counts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       lev[L].cell_off, n, tb, te, counts);
}

__global__ void k_near_fill(int64_t off, int64_t n, const int32_t *__restrict__ tb,
                            const int32_t *__restrict__ te, const int32_t *__restrict__ offs,
                            int32_t *__restrict__ items)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t b = tb[off + i], e = te[off + i];
    int32_t o = offs[i];
    for (int32_t st = b; st < e; st += kChunk, ++o) {
        items[2 * o] = (int32_t)i;     // leaf index within the leaf level
        items[2 * o + 1] = st;         // first target of the item
    }
}

void launch_near_items_fill(const LevelInfo *lev, int L, const int32_t *tb, const int32_t *te,
                            const int32_t *offs, int32_t *items, hipStream_t s)
{
    int64_t n = lev[L].n;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_near_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       lev[L].cell_off, n, tb, te, offs, items);
}

// Near-field items in decreasing order of their estimated cost, so that the
// launch ends on its cheapest items (a persistent grid otherwise ends on
// whichever items happen to come last).  The estimate is the item's rounds
// times its target blocks, in units of sixteen sources: with a leaf's whole
// near list of `srcs` sources and m targets, 2 ceil(m / 8) srcs for the
// eight-row tile, max(2, ceil(m / 4)) srcs for the four-row tile (items of at most
// `small` targets; 0 = never).  A leaf of at most `wide` targets is one item,
// its first; the other items of such a leaf cost nothing.  The key of item
// i < *count is 255 minus the estimate as an 8-bit float (5-bit exponent,
// 3-bit mantissa), so one radix pass sorts them; items past the count key
// 255 (after every item); the value is the item's index.
__global__ void k_near_cost(int64_t leaf_off, int nw, int wide, int small, int32_t cap,
                            const int32_t *__restrict__ count, const int32_t *__restrict__ items,
                            const int32_t *__restrict__ tb, const int32_t *__restrict__ te,
                            const int32_t *__restrict__ near, const int32_t *__restrict__ sb,
                            const int32_t *__restrict__ se, uint32_t *__restrict__ keys,
                            int32_t *__restrict__ vals)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    uint32_t key = 255u;
    if (i < *count) {
        const int32_t li = items[2 * i], st = items[2 * i + 1];
        const int32_t b = tb[leaf_off + li], e = te[leaf_off + li];
        const bool one = e - b <= wide;
        if (!one || st == b) {
            const int32_t m = one ? e - b : min(kChunk, e - st);
            int64_t srcs = 0;
            for (int k = 0; k < nw; ++k) {
                const int32_t c = near[(int64_t)li * nw + k];
                if (c >= 0) srcs += se[c] - sb[c];
            }
            const uint64_t blocks = m <= small ? (uint64_t)max(2, (m + 3) / 4) : 2 * (uint64_t)((m + 7) / 8);
            const uint64_t cost = blocks * (uint64_t)srcs + 1;
            const int x = 63 - __builtin_clzll(cost);   // cost in [2^x, 2^(x+1))
            const uint32_t mant = x >= 3 ? (uint32_t)(cost >> (x - 3)) & 7u : (uint32_t)(cost << (3 - x)) & 7u;
            key = 255u - min(255u, ((uint32_t)min(x, 31) << 3) | mant);
        }
    }
    keys[i] = key;
    vals[i] = i;
}

__global__ void k_items_gather(int32_t cap, const int32_t *__restrict__ order, const int32_t *__restrict__ items,
                               int32_t *__restrict__ out)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    const int32_t j = order[i];
    out[2 * i] = items[2 * j];
    out[2 * i + 1] = items[2 * j + 1];
}

void launch_near_items_order(int64_t leaf_off, int nw, int wide, int small, int32_t cap, const int32_t *count,
                             const int32_t *items, const int32_t *tb, const int32_t *te, const int32_t *near,
                             const int32_t *sb, const int32_t *se, uint32_t *keys, int32_t *vals, void *tmp,
                             int32_t *out, hipStream_t s)
{
    if (cap <= 0) return;
    const unsigned g = (unsigned)((cap + 255) / 256);
    hipLaunchKernelGGL(k_near_cost, dim3(g), dim3(256), 0, s, leaf_off, nw, wide, small, cap, count, items, tb, te,
                       near, sb, se, keys, vals);
    radix_sort(keys, vals, cap, 8, tmp, s);
    hipLaunchKernelGGL(k_items_gather, dim3(g), dim3(256), 0, s, cap, vals, items, out);
}

// ------------------------------------------------------------ pair counts
__global__ void k_count_pairs(int64_t leaf_off, int64_t n_cells, int64_t n_leaf, int e4w, int nw,
                              const int32_t *__restrict__ e4, const int32_t *__restrict__ near,
                              const int32_t *__restrict__ sb, const int32_t *__restrict__ se,
                              const int32_t *__restrict__ tb, const int32_t *__restrict__ te,
                              unsigned long long *__restrict__ out)
{
    int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid >= n_cells) return;
    unsigned long long m2l = 0, np = 0;
    for (int k = 0; k < e4w; ++k) m2l += e4[gid * e4w + k] >= 0;
    if (gid >= leaf_off && gid - leaf_off < n_leaf) {
        int64_t li = gid - leaf_off;
        unsigned long long ns = 0;
        for (int k = 0; k < nw; ++k) {
            int32_t c = near[li * nw + k];
            if (c >= 0) ns += (unsigned long long)(se[c] - sb[c]);
        }
        np = ns * (unsigned long long)(te[gid] - tb[gid]);
    }
    if (m2l) atomicAdd(&out[0], m2l);
    if (np) atomicAdd(&out[1], np);
}

void launch_count_pairs(const LevelInfo *lev, int L, int e4w, int nw, const int32_t *e4,
                        const int32_t *near, const uint8_t *occ, const int32_t *sb,
                        const int32_t *se, const int32_t *tb, const int32_t *te,
                        unsigned long long *out2, hipStream_t s)
{
    (void)occ;
    int64_t n_cells = lev[L].cell_off + lev[L].n;
    if (n_cells <= 0) return;
    hipLaunchKernelGGL(k_count_pairs, dim3((unsigned)((n_cells + 255) / 256)), dim3(256), 0, s,
                       lev[L].cell_off, n_cells, lev[L].n, e4w, nw, e4, near, sb, se, tb, te, out2);
}

// ------------------------------------------------------------ host tables
namespace {

struct Tri {
    int U, V, o;
    bool operator==(const Tri &b) const { return U == b.U && V == b.V && o == b.o; }
};

void tri_vertices(const Tri &t, int vu[3], int vv[3])
{
    if (t.o > 0) {
        vu[0] = t.U;     vv[0] = t.V + 2;
        vu[1] = t.U - 1; vv[1] = t.V - 1;
        vu[2] = t.U + 1; vv[2] = t.V - 1;
    } else {
        vu[0] = t.U;     vv[0] = t.V - 2;
        vu[1] = t.U - 1; vv[1] = t.V + 1;
        vu[2] = t.U + 1; vv[2] = t.V + 1;
    }
}

// The 12 triangles sharing a vertex with t (same size, unit circumradius).
std::vector<Tri> tri_neighbors(const Tri &t)
{
    int vu[3], vv[3];
    tri_vertices(t, vu, vv);
    std::vector<Tri> out;
    const int up_du[3] = {1, -1, 0}, up_dv[3] = {1, 1, -2};
    const int dn_du[3] = {0, 1, -1}, dn_dv[3] = {2, -1, -1};
    for (int k = 0; k < 3; ++k) {
        for (int m = 0; m < 3; ++m) {
            Tri a{vu[k] + up_du[m], vv[k] + up_dv[m], 1};
            Tri b{vu[k] + dn_du[m], vv[k] + dn_dv[m], -1};
            for (const Tri &c : {a, b}) {
                if (c == t) continue;
                if (std::find(out.begin(), out.end(), c) == out.end()) out.push_back(c);
            }
        }
    }
    return out;
}

// Children in the child level's units (coordinates doubled).
Tri tri_child(const Tri &p, int type)
{
    int U = 2 * p.U, V = 2 * p.V;
    switch (type) {
    case 0: return Tri{U, V, -p.o};
    case 1: return Tri{U, V + 2 * p.o, p.o};
    case 2: return Tri{U - 1, V - p.o, p.o};
    default: return Tri{U + 1, V - p.o, p.o};
    }
}

}  // namespace

ListTables build_tables(int tiling)
{
    ListTables t;
    memset(&t, 0, sizeof(t));
    if (tiling == kQuad) {
        t.n_groups = 4;
        t.e4_width = 27;
        t.near_width = 9;
        for (int c = 0; c < 4; ++c) {
            int cx = c & 1, cy = c >> 1, n = 0;
            for (int ey = -1; ey <= 1; ++ey)
                for (int ex = -1; ex <= 1; ++ex)
                    for (int dy = 0; dy <= 1; ++dy)
                        for (int dx = 0; dx <= 1; ++dx) {
                            int ox = 2 * ex + dx - cx, oy = 2 * ey + dy - cy;
                            if (std::max(std::abs(ox), std::abs(oy)) <= 1) continue;
                            t.e4[c][n][0] = ox;
                            t.e4[c][n][1] = oy;
                            ++n;
                        }
            t.e4_count[c] = n;
        }
        for (int oi = 0; oi < 2; ++oi) {
            int n = 0;
            t.near[oi][n][0] = 0;
            t.near[oi][n][1] = 0;
            ++n;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (!dx && !dy) continue;
                    t.near[oi][n][0] = dx;
                    t.near[oi][n][1] = dy;
                    ++n;
                }
            t.near_count[oi] = n;
        }
    } else if (tiling == kSept) {
        const int ua[7] = {0, 1, 0, -1, -1, 0, 1};
        const int ub[7] = {0, 0, 1, 1, 0, -1, -1};
        t.n_groups = 7;
        t.e4_width = 42;
        t.near_width = 7;
        for (int c = 0; c < 7; ++c) {
            int n = 0;
            for (int e = 0; e < 7; ++e) {
                // beta * unit(e): (a - 2b) + (2a + 3b) w
                int ba = ua[e] - 2 * ub[e], bb = 2 * ua[e] + 3 * ub[e];
                for (int c2 = 0; c2 < 7; ++c2) {
                    int oa = ba + ua[c2] - ua[c], ob = bb + ub[c2] - ub[c];
                    bool own = false;
                    for (int k = 0; k < 7; ++k) own |= (oa == ua[k] && ob == ub[k]);
                    if (own) continue;
                    t.e4[c][n][0] = oa;
                    t.e4[c][n][1] = ob;
                    ++n;
                }
            }
            t.e4_count[c] = n;
        }
        for (int oi = 0; oi < 2; ++oi) {
            for (int k = 0; k < 7; ++k) {
                t.near[oi][k][0] = ua[k];
                t.near[oi][k][1] = ub[k];
            }
            t.near_count[oi] = 7;
        }
    } else {
        t.n_groups = 8;
        t.e4_width = 39;
        t.near_width = 13;
        for (int oi = 0; oi < 2; ++oi) {
            int oT = oi == 0 ? 1 : -1;
            for (int c = 0; c < 4; ++c) {
                int oP = (c == 0) ? -oT : oT;
                Tri P{0, 0, oP};
                std::vector<Tri> cp = tri_neighbors(P);
                cp.insert(cp.begin(), P);
                Tri T = tri_child(P, c);
                std::vector<Tri> ct = tri_neighbors(T);
                ct.push_back(T);
                int g = c + 4 * oi, n = 0;
                for (const Tri &q : cp)
                    for (int ty = 0; ty < 4; ++ty) {
                        Tri ch = tri_child(q, ty);
                        if (std::find(ct.begin(), ct.end(), ch) != ct.end()) continue;
                        t.e4[g][n][0] = ch.U - T.U;
                        t.e4[g][n][1] = ch.V - T.V;
                        ++n;
                    }
                t.e4_count[g] = n;
            }
            Tri S{0, 0, oT};
            std::vector<Tri> nb = tri_neighbors(S);
            int n = 0;
            t.near[oi][n][0] = 0;
            t.near[oi][n][1] = 0;
            ++n;
            for (const Tri &q : nb) {
                t.near[oi][n][0] = q.U;
                t.near[oi][n][1] = q.V;
                ++n;
            }
            t.near_count[oi] = n;
        }
    }
    return t;
}

}  // namespace fmm
