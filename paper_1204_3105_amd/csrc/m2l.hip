// m2l.hip -- multipole-to-local translation in FP64: the per-plan offset
// tables, the dense contraction on FP64 MFMA (orders up to 48), and the lane
// form (one target cell per lane) for plans without target tiles.
//
// Greengard & Rokhlin (1987) Lemma 2.4 in radius-scaled form.  For a source
// cell S and target cell T on level l with delta = (c_S - c_T)/ell_l and
// g_k = a~_k (-1/delta)^k (k = 1..p):
//     b~_0 += a_0 Log(c_T - c_S) + sum_k g_k
//     b~_m += delta^(-m) [ -a_0/m + sum_k C(m+k-1, k-1) g_k ],  m = 1..p.
// The matrix C(m+k-1, k-1) is the same for every offset, so it is read from
// uniform (scalar) memory, and the offset enters only through the powers
// (-1/delta)^k and the log term.  Those depend on (level, target group,
// slot) alone -- the E4 list of every cell of one group is the same set of
// relative positions -- and are tabulated once per plan.  Each lane keeps
// its target's p+1 local coefficients and the scaled source vector in
// registers; the order is a compile-time bound PM >= p.
#include <math.h>

#include "eval.h"

namespace fmm {

int m2l_pm_for(int p)
{
    const int pms[] = {8, 16, 24, 32, 40, 48};
    for (int v : pms)
        if (p <= v) return v;
    return 0;
}

struct SlotTable {
    int off[kMaxGroups][kMaxSlots][2];   // E4 offsets per group, lattice units
    int count[kMaxGroups];
};

// Offset of slot s of group g on level l in Cartesian units, c_S - c_T.
__device__ void slot_offset(const GeoParams &G, const SlotTable &T, int l, int g, int s, double scale,
                            double &dx, double &dy)
{
    const int da = T.off[g][s][0], db = T.off[g][s][1];
    if (G.tiling == kQuad) {
        dx = da * scale;
        dy = db * scale;
    } else if (G.tiling == kSept) {
        int64_t a = da, b = db;
        for (int k = 0; k < G.L - l; ++k) {   // times beta = 1 + 2w
            const int64_t na = a - 2 * b, nb = 2 * a + 3 * b;
            a = na;
            b = nb;
        }
        const double r = G.size;
        dx = (3.0 * r * (double)a) / 2.0;
        dy = (r * G.s3 * (2.0 * (double)b + (double)a)) / 2.0;
    } else {
        const double r = G.size;
        const int64_t R = (int64_t)1 << (G.L - l);
        dx = (double)(da * R) * ((G.s3 * r) / 2.0);
        dy = (double)(db * R) * (r / 2.0);
    }
}

struct LevelScales {
    double v[kMaxL + 1];
};

// Thread per (level, group, slot) entry idx = (l G + g) S + s:
//   pw[idx (PM+1) + k] = (-1/delta)^k for k <= p (zero beyond p and for
//   unused entries), lg[idx] = Log(c_T - c_S), and the monopole row
//   a0[idx (PM+1) + k] = Log(c_T - c_S) for k = 0, -delta^-k / k =
//   (-1)^(k+1) (-1/delta)^k / k otherwise.
__global__ void k_m2l_tables(GeoParams geo, SlotTable T, LevelScales sc, int G, int S, int p, int pm,
                             double *__restrict__ pw, double *__restrict__ lg,
                             double *__restrict__ a0)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (geo.L + 1) * G * S) return;
    const int s = idx % S, g = (idx / S) % G, l = idx / (S * G);
    double *pr = pw + 2 * (size_t)idx * (pm + 1), *ar = a0 + 2 * (size_t)idx * (pm + 1);
    if (l < 1 || s >= T.count[g]) {
        for (int k = 0; k <= pm; ++k) pr[2 * k] = pr[2 * k + 1] = ar[2 * k] = ar[2 * k + 1] = 0.0;
        lg[2 * idx] = lg[2 * idx + 1] = 0.0;
        return;
    }
    double dx, dy;
    slot_offset(geo, T, l, g, s, sc.v[l], dx, dy);
    const double lx = -dx, ly = -dy + 0.0;   // a -0 imaginary part counts as +0
    const double lr = log(hypot(lx, ly)), li = atan2(ly, lx);
    lg[2 * idx] = lr;
    lg[2 * idx + 1] = li;
    const double ex = dx / sc.v[l], ey = dy / sc.v[l];
    const double d2 = ex * ex + ey * ey;
    const double qx = -ex / d2, qy = ey / d2;   // -1/delta
    double cr = 1.0, ci = 0.0;
    for (int k = 0; k <= pm; ++k) {
        const bool in = k <= p;
        pr[2 * k] = in ? cr : 0.0;
        pr[2 * k + 1] = in ? ci : 0.0;
        if (k == 0) {
            ar[0] = lr;
            ar[1] = li;
        } else {
            const double sg = (k & 1) ? 1.0 : -1.0;
            ar[2 * k] = in ? sg * cr / (double)k : 0.0;
            ar[2 * k + 1] = in ? sg * ci / (double)k : 0.0;
        }
        const double nr = cr * qx - ci * qy, ni = cr * qy + ci * qx;
        cr = nr;
        ci = ni;
    }
}

size_t m2l_table_doubles(const Plan &P, int pm)
{
    const size_t n = (size_t)(P.geo.L + 1) * P.tables.n_groups * P.tables.e4_width;
    return n * (pm + 1) * 2 * 2 + n * 2;
}

void launch_m2l_tables(Plan &P, int pm, double *base, hipStream_t s)
{
    const int G = P.tables.n_groups, S = P.tables.e4_width;
    const size_t n = (size_t)(P.geo.L + 1) * G * S;
    P.m2l_pw = base;
    P.m2l_lg = base + n * (pm + 1) * 2;
    P.m2l_a0 = P.m2l_lg + n * 2;
    SlotTable T;
    for (int g = 0; g < kMaxGroups; ++g) {
        T.count[g] = g < G ? P.tables.e4_count[g] : 0;
        for (int k = 0; k < kMaxSlots; ++k) {
            T.off[g][k][0] = P.tables.e4[g][k][0];
            T.off[g][k][1] = P.tables.e4[g][k][1];
        }
    }
    LevelScales sc;
    for (int l = 0; l <= kMaxL; ++l) sc.v[l] = l <= P.geo.L ? P.scale[l] : 0.0;
    hipLaunchKernelGGL(k_m2l_tables, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, P.geo, T, sc, G, S,
                       P.p, pm, P.m2l_pw, P.m2l_lg, P.m2l_a0);
}

template <int PM>
__global__ __launch_bounds__(64) void k_m2l_lanes(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    far_field_priority();
    constexpr int CH = 8;   // outputs per pass over the slots
    __shared__ double H[PM * PM];   // H[(m-1)*PM + (k-1)] = C(m+k-1, k-1)
    __shared__ double invm[PM + 1];
    {
        const double *binom = jobs[bm.job[0]].binom;
        for (int i = threadIdx.x; i < PM * PM; i += 64) {
            int m = i / PM + 1, k = i % PM + 1;
            H[i] = binom[(m + k - 1) * kBinomStride + (k - 1)];
        }
        for (int i = threadIdx.x; i <= PM; i += 64) invm[i] = i ? 1.0 / (double)i : 0.0;
    }
    __syncthreads();
    // One item = 64 consecutive cells of levels >= 1 (one per lane).
    for (int64_t item = blockIdx.x; item < bm.pre[bm.n]; item += gridDim.x) {
        const int e = batch_entry(bm, item);
        const EvalJob &J = jobs[bm.job[e]];
        const int64_t gid = J.m2l_first + (item - bm.pre[e]) * 64 + threadIdx.x;
        if (gid >= J.n_cells) continue;
        const int p = J.p, P1 = p + 1;
        double *out = J.lc + gid * 2 * P1;
        if (!(J.occ[gid] & 2)) {
            for (int m = 0; m <= p; ++m) out[2 * m] = out[2 * m + 1] = 0.0;
            continue;
        }
        const int l = level_of(J, gid);
        const int g = J.group[gid];
        const int32_t *row_e4 = J.e4 + gid * (int64_t)J.ew;
        const size_t tab0 = ((size_t)l * J.G + g) * J.ew;
        const double *pwt = J.m2l_pw, *lgt = J.m2l_lg, *mp = J.mp;
        const int nch = (p + CH - 1) / CH;
        for (int c = 0; c < nch; ++c) {
            double ar[CH], ai[CH];
            double b0r = 0.0, b0i = 0.0;
#pragma unroll
            for (int j = 0; j < CH; ++j) ar[j] = ai[j] = 0.0;
            for (int s = 0; s < J.ew; ++s) {
                const int32_t src = row_e4[s];
                if (src < 0) continue;
                const double *tb = pwt + 2 * (tab0 + s) * (PM + 1);
                const double *a = mp + (int64_t)src * 2 * P1;
                const double a0 = a[0];
                double gr[PM + 1], gi[PM + 1];
#pragma unroll
                for (int k = 1; k <= PM; ++k) {
                    double xr = 0.0, xi = 0.0;
                    if (k <= p) {
                        xr = a[2 * k];
                        xi = a[2 * k + 1];
                    }
                    const double tr = tb[2 * k], ti = tb[2 * k + 1];
                    gr[k] = xr * tr - xi * ti;
                    gi[k] = xr * ti + xi * tr;
                }
                if (c == 0) {
                    double s0r = a0 * lgt[2 * (tab0 + s)], s0i = a0 * lgt[2 * (tab0 + s) + 1];
#pragma unroll
                    for (int k = 1; k <= PM; ++k) {
                        s0r += gr[k];
                        s0i += gi[k];
                    }
                    b0r += s0r;
                    b0i += s0i;
                }
                // An opaque zero keeps the LDS reads of H inside the slot loop.
                int hoff = (c * CH) * PM;
                asm volatile("" : "+v"(hoff));
#pragma unroll
                for (int j = 0; j < CH; ++j) {
                    const int m = c * CH + 1 + j;
                    double hr = -a0 * invm[m < PM ? m : PM], hi = 0.0;
                    const double *Hr = H + hoff + j * PM;
#pragma unroll
                    for (int k = 1; k <= PM; ++k) {
                        const double cf = Hr[k - 1];
                        hr += cf * gr[k];
                        hi += cf * gi[k];
                    }
                    double dr = tb[2 * m], di = tb[2 * m + 1];
                    if (m & 1) {
                        dr = -dr;
                        di = -di;
                    }
                    ar[j] += hr * dr - hi * di;
                    ai[j] += hr * di + hi * dr;
                }
            }
            if (c == 0) {
                out[0] = b0r;
                out[1] = b0i;
            }
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int m = c * CH + 1 + j;
                if (m <= p) {
                    out[2 * m] = ar[j];
                    out[2 * m + 1] = ai[j];
                }
            }
        }
    }
}

// ------------------------------------------------------------ FP64 MFMA form
// The same translation as a dense contraction on v_mfma_f64_16x16x4f64.
// With g = D_in a (D_in = diag((-1/delta)^k), k = 1..p) and the offset-free
// matrix H[m][k'] = C(m + k', k') (m = 0..p, k' = k - 1), every E4 pair is
//     b~ += D_out (H g - a_0 [0, 1/1, 1/2, ..., 1/p]) + a_0 Log(c_T - c_S) e_0,
// D_out = diag(delta^-m) = diag((-1)^m (-1/delta)^m).  H is the same for every
// pair of every level and tiling, so it sits in the MFMA A-operand registers
// for the whole kernel; each pair contributes two real columns (Re g, Im g)
// to the B operand.  One workgroup takes a tile of up to 16 target cells of
// one (level, group) -- they share the slot offsets, so the slot's D_in and
// D_out are read from a table staged in LDS -- and its four waves split the
// E4 slots (wave w takes the slots s = w mod 4, so a target's sums do not
// depend on which cells share its tile); the waves' partial rows are added
// in wave order through LDS and written as contiguous rows.  Accumulation is
// FP64 throughout (the MFMA accumulates in FP64).
//
// MFMA 16x16x4 f64 operand layout (lane l, register j):
//   A[i = l%16][k = l/16], B[k = l/16][n = l%16], D[i = l/16 + 4j][n = l%16].
typedef double doublex4 __attribute__((ext_vector_type(4)));

// Output row of register j of lane group q in row tile mt.
__device__ __forceinline__ constexpr int f64_out_row(int mt, int q, int j) { return 16 * mt + q + 4 * j; }

template <int MT, int KT>
__global__ __launch_bounds__(256) void k_m2l_f64_mfma(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    far_field_priority();
    constexpr int W = 16 * MT > 4 * KT + 1 ? 16 * MT : 4 * KT + 1;   // table entries per slot
    constexpr int NR = 16 * MT;                                       // output rows per column
    constexpr int TAB_BYTES = kMaxSlots * W * 16, RED_BYTES = 4 * 16 * 2 * NR * 8;
    __shared__ __align__(16) char lds[TAB_BYTES > RED_BYTES ? TAB_BYTES : RED_BYTES];
    __shared__ double2 lgs[kMaxSlots];
    __shared__ int32_t srcs[kMaxSlots][16];
    double2 *tab = reinterpret_cast<double2 *>(lds);        // [slot][W]: (-1/delta)^k, zero beyond p
    double(*red)[16][2 * NR] = reinterpret_cast<double(*)[16][2 * NR]>(lds);   // after the slots
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = lane & 15, q = lane >> 4;

    // H in the A-operand layout: h[mt][t] = C(m + k', k'), m = 16 mt + n,
    // k' = 4 t + q (rows beyond p meet zero D_out entries, columns beyond p
    // meet zero B entries; the bounds keep the binomial table in range).
    double h[MT][KT];
    {
        const double *binom = jobs[bm.job[0]].binom;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int t = 0; t < KT; ++t) {
                const int m = 16 * mt + n, kp = 4 * t + q;
                h[mt][t] = (m <= kMaxP && kp < kMaxP) ? binom[(m + kp) * kBinomStride + kp] : 0.0;
            }
    }
    // 1/m for the output rows (0 for m = 0); every row m = 16 mt + q + 4 j of
    // this lane has the parity of q, so the sign (-1)^m of D_out is one value.
    __shared__ double invm[NR];
    for (int i = threadIdx.x; i < NR; i += 256) invm[i] = i ? 1.0 / (double)i : 0.0;
    const double sgn = (q & 1) ? -1.0 : 1.0;

    // XCD-aware order: each XCD takes a contiguous range of the tiles in
    // their launch order (by first cell), so the tiles of one region of a
    // level, of every group, share an L2 and its source multipoles.
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
            // B operand: g_k = a~_k (-1/delta)^k, k = 4 t + q + 1
            double br[KT], bi[KT];
            double a0 = 0.0;
            const double *a = J.mp + (int64_t)(src >= 0 ? src : 0) * 2 * P1;
            if (src >= 0) a0 = a[0];
#pragma unroll
            for (int t = 0; t < KT; ++t) {
                const int k = 4 * t + q + 1;
                double2 c = make_double2(0.0, 0.0);
                if (src >= 0 && k <= p) c = *reinterpret_cast<const double2 *>(a + 2 * k);
                const double2 d = ts[k];
                br[t] = c.x * d.x - c.y * d.y;
                bi[t] = c.x * d.y + c.y * d.x;
            }
            const double2 lg = lgs[sl];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                doublex4 yr = {0.0, 0.0, 0.0, 0.0}, yi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int t = 0; t < KT; ++t) {
                    yr = __builtin_amdgcn_mfma_f64_16x16x4f64(h[mt][t], br[t], yr, 0, 0, 0);
                    yi = __builtin_amdgcn_mfma_f64_16x16x4f64(h[mt][t], bi[t], yi, 0, 0, 0);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int m = f64_out_row(mt, q, j);
                    const double2 d = ts[m];
                    const double dr = sgn * d.x, di = sgn * d.y;
                    const double y = fma(-a0, invm[m], yr[j]);
                    accr[mt][j] = fma(y, dr, fma(-yi[j], di, accr[mt][j]));
                    acci[mt][j] = fma(y, di, fma(yi[j], dr, acci[mt][j]));
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
                const int m = f64_out_row(mt, q, j);
                red[w][n][2 * m] = accr[mt][j];
                red[w][n][2 * m + 1] = acci[mt][j];
            }
        __syncthreads();
        // Rows of the tile's targets, the waves' partial sums added in order.
        for (int i = threadIdx.x; i < count * 2 * P1; i += 256) {
            const int c = i / (2 * P1), r = i - c * 2 * P1;
            const double v = ((red[0][c][r] + red[1][c][r]) + red[2][c][r]) + red[3][c][r];
            J.lc[(int64_t)J.mix_list[start + c] * 2 * P1 + r] = v;
        }
    }
}

// (MT, KT) of the FP64 MFMA form for order p: MT = ceil((p+1)/16),
// KT = ceil(p/4).
static int f64_mfma_key(int p) { return ((p + 1 + 15) / 16) * 100 + (p + 3) / 4; }

bool m2l_f64_mfma_supported(int p) { return p >= 1 && p <= 48; }

void batch_m2l_f64_mfma(const EvalJob *jobs, const BatchMap &m, int p, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    const dim3 grid((persistent_grid(m.pre[m.n], 12) + 7) / 8 * 8), block(256);
#define F64_MFMA_CASE(MT, KT)                                                                         \
    case MT * 100 + KT: hipLaunchKernelGGL((k_m2l_f64_mfma<MT, KT>), grid, block, 0, s, jobs, m); break;
    switch (f64_mfma_key(p)) {
        F64_MFMA_CASE(1, 1) F64_MFMA_CASE(1, 2) F64_MFMA_CASE(1, 3) F64_MFMA_CASE(1, 4)
        F64_MFMA_CASE(2, 4) F64_MFMA_CASE(2, 5) F64_MFMA_CASE(2, 6) F64_MFMA_CASE(2, 7) F64_MFMA_CASE(2, 8)
        F64_MFMA_CASE(3, 8) F64_MFMA_CASE(3, 9) F64_MFMA_CASE(3, 10) F64_MFMA_CASE(3, 11) F64_MFMA_CASE(3, 12)
        F64_MFMA_CASE(4, 12)
    default: break;
    }
#undef F64_MFMA_CASE
}

int m2l_f64_mfma_class(int p) { return m2l_f64_mfma_supported(p) ? f64_mfma_key(p) : 0; }

void batch_m2l_lanes(const EvalJob *jobs, const BatchMap &m, int pm, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    const dim3 grid(persistent_grid(m.pre[m.n], 32));
    switch (pm) {
    case 8: hipLaunchKernelGGL(k_m2l_lanes<8>, grid, dim3(64), 0, s, jobs, m); break;
    case 16: hipLaunchKernelGGL(k_m2l_lanes<16>, grid, dim3(64), 0, s, jobs, m); break;
    case 24: hipLaunchKernelGGL(k_m2l_lanes<24>, grid, dim3(64), 0, s, jobs, m); break;
    case 32: hipLaunchKernelGGL(k_m2l_lanes<32>, grid, dim3(64), 0, s, jobs, m); break;
    case 40: hipLaunchKernelGGL(k_m2l_lanes<40>, grid, dim3(64), 0, s, jobs, m); break;
    case 48: hipLaunchKernelGGL(k_m2l_lanes<48>, grid, dim3(64), 0, s, jobs, m); break;
    default: break;
    }
}

}  // namespace fmm
