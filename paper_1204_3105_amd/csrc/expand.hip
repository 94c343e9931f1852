// expand.hip -- multipole and local expansions (FP64).
//
// Operators: Greengard & Rokhlin (1987) Lemma 2.1 (P2M), 2.3 (M2M),
// 2.4 (M2L), 2.5 (L2L); the paper cites them and omits them (end of
// Sec. 2).  Coefficients are radius-scaled per level with the real length
// ell_l of the level (quadtree: cell side; septree: lattice spacing
// r sqrt3 sqrt7^(L-l); triangle-quadtree: circumradius 2^(L-l) r):
//     multipole  phi(z) = a_0 log(z - c) + sum_k a~_k ((z - c)/ell)^(-k),
//     local      psi(z) = sum_m b~_m ((z - c)/ell)^m,
// so every stored coefficient is O(1) and the translation formulas carry
// only the dimensionless offsets.  Rows are 2(p+1) doubles, (re, im)
// interleaved, one row per cell.
#include <map>
#include <mutex>
#include <vector>

#include "fmm_internal.h"

namespace fmm {

struct cd {
    double x, y;
};
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return {a.x * s, a.y * s}; }
__device__ __forceinline__ cd cinv(cd a)
{
    double d = a.x * a.x + a.y * a.y;
    return {a.x / d, -a.y / d};
}

constexpr int kBinomN = 2 * kMaxP + 2;   // table C(n, k) for n, k < kBinomN

// Pascal's triangle C(n, k), n, k < kBinomN, built once per device on the
// host (exact integers below 2^53, correctly rounded sums above).
const double *device_binom(int *err)
{
    static std::mutex mu;
    static std::map<int, double *> tabs;
    int dev = 0;
    hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    auto it = tabs.find(dev);
    if (it != tabs.end()) return it->second;
    std::vector<double> t((size_t)kBinomN * kBinomN, 0.0);
    for (int n = 0; n < kBinomN; ++n) {
        t[(size_t)n * kBinomN] = 1.0;
        for (int k = 1; k <= n; ++k)
            t[(size_t)n * kBinomN + k] = t[(size_t)(n - 1) * kBinomN + k - 1] + t[(size_t)(n - 1) * kBinomN + k];
    }
    double *d = nullptr;
    if (hipMalloc(&d, t.size() * sizeof(double)) != hipSuccess ||
        hipMemcpy(d, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        if (err) *err = 1;
        return nullptr;
    }
    tabs[dev] = d;
    return d;
}

struct ExpParams {
    int p, L, tiling, base;
    double scale[kMaxL + 1];
    int64_t cell_off[kMaxL + 2];
    int64_t dense_off[kMaxL + 1];
};

static ExpParams exp_params(const Plan &P)
{
    ExpParams e;
    e.p = P.p;
    e.L = P.geo.L;
    e.tiling = P.geo.tiling;
    e.base = base_of(P.geo.tiling);
    for (int l = 0; l <= P.geo.L; ++l) {
        e.scale[l] = P.scale[l];
        e.cell_off[l] = P.lev[l].cell_off;
        e.dense_off[l] = P.lev[l].dense_off;
    }
    e.cell_off[P.geo.L + 1] = P.n_cells;
    return e;
}

// ------------------------------------------------------------------ P2M
// One wave per leaf: lane i holds one source, builds w^k incrementally and
// the wave reduces each term; lane k keeps coefficient k.
__global__ __launch_bounds__(64) void k_p2m(ExpParams e, const double *__restrict__ sx,
                                            const double *__restrict__ sy,
                                            const double *__restrict__ su,
                                            const int32_t *__restrict__ sb,
                                            const int32_t *__restrict__ se,
                                            const double *__restrict__ cx,
                                            const double *__restrict__ cy,
                                            double *__restrict__ mp)
{
    int64_t gid = e.cell_off[e.L] + blockIdx.x;
    int lane = threadIdx.x;
    int32_t b = sb[gid], en = se[gid];
    const int P1 = e.p + 1;
    double *row = mp + gid * 2 * P1;
    if (en <= b) {
        if (lane < P1) {
            row[2 * lane] = 0.0;
            row[2 * lane + 1] = 0.0;
        }
        return;
    }
    const double inv = 1.0 / e.scale[e.L];
    const double c0 = cx[gid], c1 = cy[gid];
    double acc_re = 0.0, acc_im = 0.0;
    for (int32_t base = b; base < en; base += 64) {
        int32_t i = base + lane;
        bool ok = i < en;
        double u = ok ? su[i] : 0.0;
        cd w = ok ? cd{(sx[i] - c0) * inv, (sy[i] - c1) * inv} : cd{0.0, 0.0};
        // a_0 = sum u
        double s0 = u;
        for (int o = 32; o > 0; o >>= 1) s0 += __shfl_xor(s0, o);
        if (lane == 0) acc_re += s0;
        cd pw = {1.0, 0.0};
        for (int k = 1; k <= e.p; ++k) {
            pw = cmul(pw, w);
            double f = -u / (double)k;
            double tr = pw.x * f, ti = pw.y * f;
            for (int o = 32; o > 0; o >>= 1) {
                tr += __shfl_xor(tr, o);
                ti += __shfl_xor(ti, o);
            }
            if (lane == k) {
                acc_re += tr;
                acc_im += ti;
            }
        }
    }
    if (lane < P1) {
        row[2 * lane] = acc_re;
        row[2 * lane + 1] = acc_im;
    }
}

void launch_p2m(const Plan &P, hipStream_t s)
{
    int64_t n = P.lev[P.geo.L].n;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_p2m, dim3((unsigned)n), dim3(64), 0, s, exp_params(P), P.sx, P.sy, P.su,
                       P.sb, P.se, P.cx, P.cy, P.mp);
}

// ------------------------------------------------------------------ M2M
// Block per level-l cell, thread m: sum over source-occupied children of
//   b~_m = -a_0 w^m / m + sum_{k=1..m} a~_k rho^k w^(m-k) C(m-1, k-1),
// w = (c_child - c_parent)/ell_l, rho = ell_(l+1)/ell_l.
__global__ __launch_bounds__(64) void k_m2m(ExpParams e, int l, const uint8_t *__restrict__ occ,
                                            const int32_t *__restrict__ dense,
                                            const uint32_t *__restrict__ cell_key,
                                            const double *__restrict__ cx,
                                            const double *__restrict__ cy,
                                            const double *__restrict__ binom,
                                            double *__restrict__ mp)
{
    __shared__ cd wp[kMaxP + 1];
    __shared__ cd ac[kMaxP + 1];
    __shared__ double rp[kMaxP + 1];
    int64_t gid = e.cell_off[l] + blockIdx.x;
    const int m = threadIdx.x, P1 = e.p + 1;
    double *row = mp + gid * 2 * P1;
    if (!(occ[gid] & 1)) {
        if (m < P1) {
            row[2 * m] = 0.0;
            row[2 * m + 1] = 0.0;
        }
        return;
    }
    const double inv = 1.0 / e.scale[l];
    const double rho = e.scale[l + 1] * inv;
    if (m == 0) {
        double r = 1.0;
        for (int k = 0; k <= e.p; ++k) {
            rp[k] = r;
            r *= rho;
        }
    }
    cd acc = {0.0, 0.0};
    uint32_t key = cell_key[gid];
    for (int d = 0; d < e.base; ++d) {
        uint32_t ck = key * (uint32_t)e.base + (uint32_t)d;
        int32_t c = dense[e.dense_off[l + 1] + ck];
        __syncthreads();
        if (c < 0 || !(occ[c] & 1)) continue;   // uniform across the block
        if (m < P1) ac[m] = cd{mp[(int64_t)c * 2 * P1 + 2 * m], mp[(int64_t)c * 2 * P1 + 2 * m + 1]};
        if (m == 0) {
            cd w = {(cx[c] - cx[gid]) * inv, (cy[c] - cy[gid]) * inv};
            cd q = {1.0, 0.0};
            for (int k = 0; k <= e.p; ++k) {
                wp[k] = q;
                q = cmul(q, w);
            }
        }
        __syncthreads();
        if (m < P1) {
            if (m == 0) {
                acc = cadd(acc, ac[0]);
            } else {
                cd s = cscale(wp[m], -ac[0].x / (double)m);
                for (int k = 1; k <= m; ++k) {
                    double cf = rp[k] * binom[(m - 1) * kBinomN + (k - 1)];
                    s = cadd(s, cscale(cmul(ac[k], wp[m - k]), cf));
                }
                acc = cadd(acc, s);
            }
        }
    }
    if (m < P1) {
        row[2 * m] = acc.x;
        row[2 * m + 1] = acc.y;
    }
}

void launch_m2m(const Plan &P, int level, hipStream_t s)
{
    int64_t n = P.lev[level].n;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_m2m, dim3((unsigned)n), dim3(64), 0, s, exp_params(P), level, P.cell_occ,
                       P.dense, P.cell_key, P.cx, P.cy, P.binom, P.mp);
}

// ------------------------------------------------------------------ M2L
// Block per target-occupied cell at levels >= 1, thread m.  For a source
// cell S with delta = (c_S - c_T)/ell and g_k = a~_k (-1/delta)^k:
//   b~_0 += a_0 Log(c_T - c_S) + sum_k g_k
//   b~_m += delta^(-m) [ -a_0/m + sum_k C(m+k-1, k-1) g_k ]
__global__ __launch_bounds__(64) void k_m2l_fp64(ExpParams e, int ew, const uint8_t *__restrict__ occ,
                                                 const int32_t *__restrict__ e4,
                                                 const double *__restrict__ cx,
                                                 const double *__restrict__ cy,
                                                 const double *__restrict__ binom,
                                                 const double *__restrict__ mp,
                                                 double *__restrict__ lc)
{
    __shared__ cd gk[kMaxP + 1];
    __shared__ cd np[kMaxP + 1];   // (-1/delta)^k
    __shared__ double a0s;
    __shared__ cd lg;
    int64_t gid = e.cell_off[1] + blockIdx.x;
    int l = 1;
    while (l < e.L && gid >= e.cell_off[l + 1]) ++l;
    const int m = threadIdx.x, P1 = e.p + 1;
    double *row = lc + gid * 2 * P1;
    cd acc = {0.0, 0.0};
    if (occ[gid] & 2) {
        const double inv = 1.0 / e.scale[l];
        const double tx = cx[gid], ty = cy[gid];
        for (int k = 0; k < ew; ++k) {
            int32_t s = e4[gid * ew + k];
            if (s < 0) continue;   // uniform across the block
            __syncthreads();
            const double *src = mp + (int64_t)s * 2 * P1;
            if (m == 0) {
                double dx = cx[s] - tx, dy = cy[s] - ty;   // c_S - c_T
                cd d = {dx * inv, dy * inv};
                cd q = cinv(d);
                q = cd{-q.x, -q.y};
                cd pw = {1.0, 0.0};
                for (int j = 0; j <= e.p; ++j) {
                    np[j] = pw;
                    pw = cmul(pw, q);
                }
                double lx = tx - cx[s], ly = (ty - cy[s]) + 0.0;   // c_T - c_S, -0 -> +0
                lg = cd{log(hypot(lx, ly)), atan2(ly, lx)};
                a0s = src[0];
            }
            __syncthreads();
            if (m >= 1 && m < P1) gk[m] = cmul(cd{src[2 * m], src[2 * m + 1]}, np[m]);
            __syncthreads();
            if (m == 0) {
                cd s0 = cscale(lg, a0s);
                for (int k2 = 1; k2 <= e.p; ++k2) s0 = cadd(s0, gk[k2]);
                acc = cadd(acc, s0);
            } else if (m < P1) {
                cd s1 = {-a0s / (double)m, 0.0};
                const double *bc = binom + (int64_t)(m) * 0;
                (void)bc;
                for (int k2 = 1; k2 <= e.p; ++k2)
                    s1 = cadd(s1, cscale(gk[k2], binom[(m + k2 - 1) * kBinomN + (k2 - 1)]));
                // delta^(-m) = (-1)^m (-1/delta)^m
                cd dm = np[m];
                if (m & 1) dm = cd{-dm.x, -dm.y};
                acc = cadd(acc, cmul(s1, dm));
            }
        }
    }
    if (m < P1) {
        row[2 * m] = acc.x;
        row[2 * m + 1] = acc.y;
    }
}

void launch_m2l_fp64(const Plan &P, hipStream_t s)
{
    int64_t n = P.n_cells - P.lev[1 <= P.geo.L ? 1 : 0].cell_off;
    if (P.geo.L < 1 || n <= 0) return;
    hipLaunchKernelGGL(k_m2l_fp64, dim3((unsigned)n), dim3(64), 0, s, exp_params(P),
                       P.tables.e4_width, P.cell_occ, P.e4, P.cx, P.cy, P.binom, P.mp, P.lc);
}

// ------------------------------------------------------------------ L2L
// Block per target-occupied cell at level l (>= 2), thread m:
//   b~'_m += sum_{k>=m} b~_k C(k, m) w^(k-m) rho^m,
// w = (c_child - c_parent)/ell_(l-1), rho = ell_l/ell_(l-1).
__global__ __launch_bounds__(64) void k_l2l(ExpParams e, int l, const uint8_t *__restrict__ occ,
                                            const int32_t *__restrict__ parent,
                                            const double *__restrict__ cx,
                                            const double *__restrict__ cy,
                                            const double *__restrict__ binom,
                                            double *__restrict__ lc)
{
    __shared__ cd wp[kMaxP + 1];
    __shared__ cd bp[kMaxP + 1];
    int64_t gid = e.cell_off[l] + blockIdx.x;
    if (!(occ[gid] & 2)) return;
    const int m = threadIdx.x, P1 = e.p + 1;
    int32_t par = parent[gid];
    const double inv = 1.0 / e.scale[l - 1];
    const double rho = e.scale[l] * inv;
    if (m < P1) bp[m] = cd{lc[(int64_t)par * 2 * P1 + 2 * m], lc[(int64_t)par * 2 * P1 + 2 * m + 1]};
    if (m == 0) {
        cd w = {(cx[gid] - cx[par]) * inv, (cy[gid] - cy[par]) * inv};
        cd q = {1.0, 0.0};
        for (int k = 0; k <= e.p; ++k) {
            wp[k] = q;
            q = cmul(q, w);
        }
    }
    __syncthreads();
    if (m < P1) {
        cd s = {0.0, 0.0};
        for (int k = m; k <= e.p; ++k) s = cadd(s, cscale(cmul(bp[k], wp[k - m]), binom[k * kBinomN + m]));
        double rm = 1.0;
        for (int j = 0; j < m; ++j) rm *= rho;
        double *row = lc + gid * 2 * P1;
        row[2 * m] += s.x * rm;
        row[2 * m + 1] += s.y * rm;
    }
}

void launch_l2l(const Plan &P, int level, hipStream_t s)
{
    int64_t n = P.lev[level].n;
    if (n <= 0 || level < 2) return;
    hipLaunchKernelGGL(k_l2l, dim3((unsigned)n), dim3(64), 0, s, exp_params(P), level, P.cell_occ,
                       P.parent, P.cx, P.cy, P.binom, P.lc);
}

// ------------------------------------------------------------------ gather u
__global__ void k_gather_u(const double *__restrict__ u, const int32_t *__restrict__ perm, int64_t n,
                           double *__restrict__ su, float *__restrict__ suf)
{
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    double v = u[perm[j]];
    su[j] = v;
    if (suf) suf[j] = (float)v;
}

void launch_gather_u(const double *u, const int32_t *perm, int64_t n, double *su, float *suf,
                     hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_u, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, u, perm, n, su,
                       suf);
}

}  // namespace fmm
