// expand.hip -- multipole and local expansions (FP64): P2M, M2M, L2L, and
// the general-order M2L fallback.
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
// interleaved, one row per cell.  All kernels walk a batch of plans (see
// eval.h) with a persistent grid.
#include <map>
#include <mutex>
#include <vector>

#include "eval.h"

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

// Pascal's triangle C(n, k), n, k < kBinomStride, built once per device on
// the host (exact integers below 2^53, correctly rounded sums above).
const double *device_binom(int *err)
{
    static std::mutex mu;
    static std::map<int, double *> tabs;
    int dev = 0;
    hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    auto it = tabs.find(dev);
    if (it != tabs.end()) return it->second;
    std::vector<double> t((size_t)kBinomStride * kBinomStride, 0.0);
    for (int n = 0; n < kBinomStride; ++n) {
        t[(size_t)n * kBinomStride] = 1.0;
        for (int k = 1; k <= n; ++k)
            t[(size_t)n * kBinomStride + k] =
                t[(size_t)(n - 1) * kBinomStride + k - 1] + t[(size_t)(n - 1) * kBinomStride + k];
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

void batch_gather_u(const EvalJob *jobs_d, const EvalJob &J, const double *u, hipStream_t s)
{
    (void)jobs_d;
    if (J.n_src <= 0) return;
    hipLaunchKernelGGL(k_gather_u, dim3((unsigned)((J.n_src + 255) / 256)), dim3(256), 0, s, u,
                       J.sperm, J.n_src, J.su, J.prec == FMM_PREC_MIXED ? J.suf : nullptr);
}

// ------------------------------------------------------------------ P2M
// One wave per leaf.  The leaf's sources are loaded 64 at a time, one per
// lane, all loads in flight together; they are then taken 16 at a time: the
// wave's four 16-lane quarters read the same 16 sources from their owner
// lanes (cross-lane reads), and quarter q writes the terms -u w^k / k of the
// coefficients k = q (mod 4) (w^k stepped by w^4) to an LDS table with a
// row per Re/Im coefficient and a column per source; then lane r sums row r
// (and r + 64) over the 16 columns in source order.  With bm.u_in (a single
// plan) the strengths are gathered here from the caller's order,
// u = u_in[sperm[i]], and stored in sorted order (FP64, and FP32 for the
// mixed near field) for the near-field kernels.
constexpr int kP2MChunk = 16;
constexpr int kP2MStride = kP2MChunk + 1;   // odd stride: conflict-free row reads

__device__ __forceinline__ double lane_read(double v, int src)
{
    const int lo = __shfl(__double2loint(v), src), hi = __shfl(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

__global__ __launch_bounds__(64) void k_p2m(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    extern __shared__ double tab[];          // 2 (pmax + 1) rows of kP2MStride
    __shared__ double invk[kMaxP + 1];       // 1/k
    const int lane = threadIdx.x;
    const int src_lane = lane & (kP2MChunk - 1), q = lane / kP2MChunk;
    for (int k = lane; k <= kMaxP; k += 64) invk[k] = k ? 1.0 / (double)k : 0.0;
    for (int64_t item = blockIdx.x; item < bm.pre[bm.n]; item += gridDim.x) {
        const int e = batch_entry(bm, item);
        const EvalJob &J = jobs[bm.job[e]];
        const int64_t gid = J.leaf_off + (item - bm.pre[e]);
        const int32_t b = J.sb[gid], en = J.se[gid];
        const int p = J.p, P1 = p + 1, R = 2 * P1;
        double *row = J.mp + gid * 2 * P1;
        const double inv = 1.0 / J.scale[J.L];
        const double c0 = J.cx[gid], c1 = J.cy[gid];
        const bool gather = bm.u_in != nullptr, mixed = J.prec == FMM_PREC_MIXED;
        double acc = 0.0, acc2 = 0.0;   // rows lane and lane + 64
        for (int32_t blk = b; blk < en; blk += 64) {
            // this lane's source of the 64-block
            const int32_t i = blk + lane;
            double ul = 0.0, wxl = 0.0, wyl = 0.0;
            if (i < en) {
                if (gather) {
                    ul = bm.u_in[J.sperm[i]];
                    J.su[i] = ul;
                    if (mixed) J.suf[i] = (float)ul;
                } else {
                    ul = J.su[i];
                }
                wxl = (J.sx[i] - c0) * inv;
                wyl = (J.sy[i] - c1) * inv;
            }
            const int nb = en - blk < 64 ? en - blk : 64;
            for (int c = 0; c < nb; c += kP2MChunk) {
                const int from = c + src_lane;
                const double u = lane_read(ul, from);
                const cd w = {lane_read(wxl, from), lane_read(wyl, from)};   // zero past the end
                const cd w2 = cmul(w, w);
                const cd w4 = cmul(w2, w2);
                __syncthreads();
                if (q == 0) {
                    tab[0 * kP2MStride + src_lane] = u;
                    tab[1 * kP2MStride + src_lane] = 0.0;
                }
                cd pw = q == 0 ? w4 : (q == 1 ? w : (q == 2 ? w2 : cmul(w2, w)));   // w^q, w^4 for q = 0
                for (int k = q == 0 ? 4 : q; k <= p; k += 4) {
                    const double f = -u * invk[k];
                    tab[(2 * k) * kP2MStride + src_lane] = pw.x * f;
                    tab[(2 * k + 1) * kP2MStride + src_lane] = pw.y * f;
                    pw = cmul(pw, w4);
                }
                __syncthreads();
                const int n = nb - c < kP2MChunk ? nb - c : kP2MChunk;
                if (lane < R) {
                    double s = 0.0;
                    for (int j = 0; j < n; ++j) s += tab[lane * kP2MStride + j];
                    acc += s;
                }
                if (lane + 64 < R) {
                    double s = 0.0;
                    for (int j = 0; j < n; ++j) s += tab[(lane + 64) * kP2MStride + j];
                    acc2 += s;
                }
            }
        }
        if (lane < R) row[lane] = acc;
        if (lane + 64 < R) row[lane + 64] = acc2;
    }
}

void batch_p2m(const EvalJob *jobs, const BatchMap &m, int pmax, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    const size_t lds = (size_t)2 * (pmax + 1) * kP2MStride * sizeof(double);
    hipLaunchKernelGGL(k_p2m, dim3(persistent_grid(m.pre[m.n], 64)), dim3(64), lds, s, jobs, m);
}

// ------------------------------------------------------------------ M2M
// Block per level-l cell (l = aux of the entry), thread m: sum over
// source-occupied children of
//   b~_m = -a_0 w^m / m + sum_{k=1..m} a~_k rho^k w^(m-k) C(m-1, k-1),
// w = (c_child - c_parent)/ell_l, rho = ell_(l+1)/ell_l.
__global__ __launch_bounds__(64) void k_m2m(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    far_field_priority();
    __shared__ cd wp[kMaxP + 1];
    __shared__ cd ac[kMaxP + 1];
    __shared__ double rp[kMaxP + 1];
    const int m = threadIdx.x;
    for (int64_t item = blockIdx.x; item < bm.pre[bm.n]; item += gridDim.x) {
        const int e = batch_entry(bm, item);
        const EvalJob &J = jobs[bm.job[e]];
        const int l = bm.aux[e];
        const int64_t gid = J.cell_off[l] + (item - bm.pre[e]);
        const int P1 = J.p + 1;
        double *row = J.mp + gid * 2 * P1;
        if (!(J.occ[gid] & 1)) {
            if (m < P1) row[2 * m] = row[2 * m + 1] = 0.0;
            continue;
        }
        const double inv = 1.0 / J.scale[l];
        const double rho = J.scale[l + 1] * inv;
        __syncthreads();
        if (m == 0) {
            double r = 1.0;
            for (int k = 0; k <= J.p; ++k) {
                rp[k] = r;
                r *= rho;
            }
        }
        cd acc = {0.0, 0.0};
        const uint32_t key = J.cell_key[gid];
        for (int d = 0; d < J.base; ++d) {
            const uint32_t ck = key * (uint32_t)J.base + (uint32_t)d;
            const int32_t c = J.dense[J.dense_off[l + 1] + ck];
            __syncthreads();
            if (c < 0 || !(J.occ[c] & 1)) continue;   // uniform across the block
            if (m < P1) ac[m] = cd{J.mp[(int64_t)c * 2 * P1 + 2 * m], J.mp[(int64_t)c * 2 * P1 + 2 * m + 1]};
            if (m == 0) {
                const cd w = {(J.cx[c] - J.cx[gid]) * inv, (J.cy[c] - J.cy[gid]) * inv};
                cd q = {1.0, 0.0};
                for (int k = 0; k <= J.p; ++k) {
                    wp[k] = q;
                    q = cmul(q, w);
                }
            }
            __syncthreads();
            if (m < P1) {
                if (m == 0) {
                    acc = cadd(acc, ac[0]);
                } else {
                    cd sm = cscale(wp[m], -ac[0].x / (double)m);
                    for (int k = 1; k <= m; ++k) {
                        const double cf = rp[k] * J.binom[(m - 1) * kBinomStride + (k - 1)];
                        sm = cadd(sm, cscale(cmul(ac[k], wp[m - k]), cf));
                    }
                    acc = cadd(acc, sm);
                }
            }
        }
        if (m < P1) {
            row[2 * m] = acc.x;
            row[2 * m + 1] = acc.y;
        }
        __syncthreads();
    }
}

void batch_m2m(const EvalJob *jobs, const BatchMap &m, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    hipLaunchKernelGGL(k_m2m, dim3(persistent_grid(m.pre[m.n], 64)), dim3(64), 0, s, jobs, m);
}

// ------------------------------------------------------------------ L2L
// Block per target-occupied cell at level l (>= 2, aux of the entry),
// thread m:  b~'_m += sum_{k>=m} b~_k C(k, m) w^(k-m) rho^m,
// w = (c_child - c_parent)/ell_(l-1), rho = ell_l/ell_(l-1).
__global__ __launch_bounds__(64) void k_l2l(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    far_field_priority();
    __shared__ cd wp[kMaxP + 1];
    __shared__ cd bp[kMaxP + 1];
    const int m = threadIdx.x;
    for (int64_t item = blockIdx.x; item < bm.pre[bm.n]; item += gridDim.x) {
        const int e = batch_entry(bm, item);
        const EvalJob &J = jobs[bm.job[e]];
        const int l = bm.aux[e];
        const int64_t gid = J.cell_off[l] + (item - bm.pre[e]);
        if (!(J.occ[gid] & 2)) continue;
        const int P1 = J.p + 1;
        const int32_t par = J.parent[gid];
        const double inv = 1.0 / J.scale[l - 1];
        const double rho = J.scale[l] * inv;
        __syncthreads();
        if (m < P1) bp[m] = cd{J.lc[(int64_t)par * 2 * P1 + 2 * m], J.lc[(int64_t)par * 2 * P1 + 2 * m + 1]};
        if (m == 0) {
            const cd w = {(J.cx[gid] - J.cx[par]) * inv, (J.cy[gid] - J.cy[par]) * inv};
            cd q = {1.0, 0.0};
            for (int k = 0; k <= J.p; ++k) {
                wp[k] = q;
                q = cmul(q, w);
            }
        }
        __syncthreads();
        if (m < P1) {
            cd sm = {0.0, 0.0};
            for (int k = m; k <= J.p; ++k)
                sm = cadd(sm, cscale(cmul(bp[k], wp[k - m]), J.binom[k * kBinomStride + m]));
            double rm = 1.0;
            for (int j = 0; j < m; ++j) rm *= rho;
            double *row = J.lc + gid * 2 * P1;
            row[2 * m] += sm.x * rm;
            row[2 * m + 1] += sm.y * rm;
        }
    }
}

void batch_l2l(const EvalJob *jobs, const BatchMap &m, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    hipLaunchKernelGGL(k_l2l, dim3(persistent_grid(m.pre[m.n], 64)), dim3(64), 0, s, jobs, m);
}

// ------------------------------------------------------------------ M2M / L2L, lane form
// The same translations with one lane per (parent, child) pair (M2M) or per
// child (L2L), coefficients in registers (orders padded to PM with zeros),
// and the binomial sums done as Horner-style triangles with no division:
//   M2M: x_k = a~_k rho^k; passes j = 1..PM-1 of x_k += w x_(k-1)
//        (k = PM down to j+1) leave x_m = sum_k C(m-1, k-1) w^(m-k) x_k;
//        then b~_m = x_m - a_0 w^m / m and b~_0 = a_0.
//   L2L: passes j = 0..PM-1 of y_k += w y_(k+1) (k = PM-1 down to j) leave
//        y_m = sum_(k>=m) C(k, m) w^(k-m) b~_k; then b~'_m += y_m rho^m.
// The children of one parent occupy GS consecutive lanes (GS >= base) and
// are summed by an xor butterfly, which leaves the same sum in every lane.
template <int PM, int GS>
__global__ __launch_bounds__(256) void k_m2m_lanes(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    far_field_priority();
    const int64_t total = bm.pre[bm.n] * GS;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t item = t / GS;
        const int d = (int)(t % GS);
        const int e = batch_entry(bm, item);
        const EvalJob &J = jobs[bm.job[e]];
        const int l = bm.aux[e];
        const int64_t gid = J.cell_off[l] + (item - bm.pre[e]);
        const int p = J.p, P1 = p + 1;
        double xr[PM + 1], xi[PM + 1];
#pragma unroll
        for (int k = 0; k <= PM; ++k) xr[k] = xi[k] = 0.0;
        int32_t c = -1;
        if ((J.occ[gid] & 1) && d < J.base) {
            c = J.dense[J.dense_off[l + 1] + (int64_t)J.cell_key[gid] * J.base + d];
            if (c >= 0 && !(J.occ[c] & 1)) c = -1;
        }
        if (c >= 0) {
            const double inv = 1.0 / J.scale[l];
            const double rho = J.scale[l + 1] * inv;
            const double wr = (J.cx[c] - J.cx[gid]) * inv, wi = (J.cy[c] - J.cy[gid]) * inv;
            const double *a = J.mp + (int64_t)c * 2 * P1;
            double r = rho;
#pragma unroll
            for (int k = 1; k <= PM; ++k) {
                if (k <= p) {
                    xr[k] = a[2 * k] * r;
                    xi[k] = a[2 * k + 1] * r;
                }
                r *= rho;
            }
#pragma unroll
            for (int j = 1; j < PM; ++j)
#pragma unroll
                for (int k = PM; k > j; --k) {
                    xr[k] += wr * xr[k - 1] - wi * xi[k - 1];
                    xi[k] += wr * xi[k - 1] + wi * xr[k - 1];
                }
            const double a0 = a[0];
            double pr = 1.0, pi = 0.0;
#pragma unroll
            for (int m = 1; m <= PM; ++m) {
                const double nr = pr * wr - pi * wi, ni = pr * wi + pi * wr;
                pr = nr;
                pi = ni;
                const double f = -a0 / (double)m;
                xr[m] += f * pr;
                xi[m] += f * pi;
            }
            xr[0] = a[0];
            xi[0] = a[1];
        }
#pragma unroll
        for (int o = 1; o < GS; o <<= 1)
#pragma unroll
            for (int k = 0; k <= PM; ++k) {
                xr[k] += __shfl_xor(xr[k], o);
                xi[k] += __shfl_xor(xi[k], o);
            }
        double *row = J.mp + gid * 2 * P1;
#pragma unroll
        for (int m = 0; m <= PM; ++m)
            if (m <= p && m % GS == d) {
                row[2 * m] = xr[m];
                row[2 * m + 1] = xi[m];
            }
    }
}

template <int PM>
__global__ __launch_bounds__(256) void k_l2l_lanes(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    far_field_priority();
    for (int64_t item = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; item < bm.pre[bm.n];
         item += (int64_t)gridDim.x * blockDim.x) {
        const int e = batch_entry(bm, item);
        const EvalJob &J = jobs[bm.job[e]];
        const int l = bm.aux[e];
        const int64_t gid = J.cell_off[l] + (item - bm.pre[e]);
        if (!(J.occ[gid] & 2)) continue;
        const int p = J.p, P1 = p + 1;
        const int32_t par = J.parent[gid];
        const double inv = 1.0 / J.scale[l - 1];
        const double rho = J.scale[l] * inv;
        const double wr = (J.cx[gid] - J.cx[par]) * inv, wi = (J.cy[gid] - J.cy[par]) * inv;
        const double *b = J.lc + (int64_t)par * 2 * P1;
        double yr[PM + 1], yi[PM + 1];
#pragma unroll
        for (int k = 0; k <= PM; ++k) {
            yr[k] = k <= p ? b[2 * k] : 0.0;
            yi[k] = k <= p ? b[2 * k + 1] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < PM; ++j)
#pragma unroll
            for (int k = PM - 1; k >= j; --k) {
                yr[k] += wr * yr[k + 1] - wi * yi[k + 1];
                yi[k] += wr * yi[k + 1] + wi * yr[k + 1];
            }
        double *row = J.lc + gid * 2 * P1;
        double r = 1.0;
#pragma unroll
        for (int m = 0; m <= PM; ++m) {
            if (m <= p) {
                row[2 * m] += yr[m] * r;
                row[2 * m + 1] += yi[m] * r;
            }
            r *= rho;
        }
    }
}

template <int PM>
static void launch_m2m_lanes(const EvalJob *jobs, const BatchMap &m, int gs, hipStream_t s)
{
    const unsigned grid = persistent_grid((m.pre[m.n] * gs + 255) / 256, 16);
    if (gs == 4) hipLaunchKernelGGL((k_m2m_lanes<PM, 4>), dim3(grid), dim3(256), 0, s, jobs, m);
    else hipLaunchKernelGGL((k_m2m_lanes<PM, 8>), dim3(grid), dim3(256), 0, s, jobs, m);
}

void batch_m2m_lanes(const EvalJob *jobs, const BatchMap &m, int pm, int gs, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    switch (pm) {
    case 8: launch_m2m_lanes<8>(jobs, m, gs, s); break;
    case 16: launch_m2m_lanes<16>(jobs, m, gs, s); break;
    case 24: launch_m2m_lanes<24>(jobs, m, gs, s); break;
    case 32: launch_m2m_lanes<32>(jobs, m, gs, s); break;
    case 40: launch_m2m_lanes<40>(jobs, m, gs, s); break;
    case 48: launch_m2m_lanes<48>(jobs, m, gs, s); break;
    default: break;
    }
}

void batch_l2l_lanes(const EvalJob *jobs, const BatchMap &m, int pm, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    const dim3 grid(persistent_grid((m.pre[m.n] + 255) / 256, 16)), block(256);
    switch (pm) {
    case 8: hipLaunchKernelGGL((k_l2l_lanes<8>), grid, block, 0, s, jobs, m); break;
    case 16: hipLaunchKernelGGL((k_l2l_lanes<16>), grid, block, 0, s, jobs, m); break;
    case 24: hipLaunchKernelGGL((k_l2l_lanes<24>), grid, block, 0, s, jobs, m); break;
    case 32: hipLaunchKernelGGL((k_l2l_lanes<32>), grid, block, 0, s, jobs, m); break;
    case 40: hipLaunchKernelGGL((k_l2l_lanes<40>), grid, block, 0, s, jobs, m); break;
    case 48: hipLaunchKernelGGL((k_l2l_lanes<48>), grid, block, 0, s, jobs, m); break;
    default: break;
    }
}

// ------------------------------------------------------------------ M2L
// General-order fallback (any p): block per target cell at levels >= 1,
// thread m.  For a source cell with delta = (c_S - c_T)/ell and
// g_k = a~_k (-1/delta)^k:
//   b~_0 += a_0 Log(c_T - c_S) + sum_k g_k
//   b~_m += delta^(-m) [ -a_0/m + sum_k C(m+k-1, k-1) g_k ]
__global__ __launch_bounds__(64) void k_m2l_block(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    far_field_priority();
    __shared__ cd gk[kMaxP + 1];
    __shared__ cd np[kMaxP + 1];   // (-1/delta)^k
    __shared__ double a0s;
    __shared__ cd lg;
    const int m = threadIdx.x;
    for (int64_t item = blockIdx.x; item < bm.pre[bm.n]; item += gridDim.x) {
        const int e = batch_entry(bm, item);
        const EvalJob &J = jobs[bm.job[e]];
        const int64_t gid = J.m2l_first + (item - bm.pre[e]);
        const int l = level_of(J, gid);
        const int P1 = J.p + 1;
        double *row = J.lc + gid * 2 * P1;
        cd acc = {0.0, 0.0};
        if (J.occ[gid] & 2) {
            const double inv = 1.0 / J.scale[l];
            const double tx = J.cx[gid], ty = J.cy[gid];
            for (int k = 0; k < J.ew; ++k) {
                const int32_t s = J.e4[gid * J.ew + k];
                if (s < 0) continue;   // uniform across the block
                __syncthreads();
                const double *src = J.mp + (int64_t)s * 2 * P1;
                if (m == 0) {
                    const cd d = {(J.cx[s] - tx) * inv, (J.cy[s] - ty) * inv};
                    cd q = cinv(d);
                    q = cd{-q.x, -q.y};
                    cd pw = {1.0, 0.0};
                    for (int j = 0; j <= J.p; ++j) {
                        np[j] = pw;
                        pw = cmul(pw, q);
                    }
                    const double lx = tx - J.cx[s], ly = (ty - J.cy[s]) + 0.0;
                    lg = cd{log(hypot(lx, ly)), atan2(ly, lx)};
                    a0s = src[0];
                }
                __syncthreads();
                if (m >= 1 && m < P1) gk[m] = cmul(cd{src[2 * m], src[2 * m + 1]}, np[m]);
                __syncthreads();
                if (m == 0) {
                    cd s0 = cscale(lg, a0s);
                    for (int k2 = 1; k2 <= J.p; ++k2) s0 = cadd(s0, gk[k2]);
                    acc = cadd(acc, s0);
                } else if (m < P1) {
                    cd s1 = {-a0s / (double)m, 0.0};
                    for (int k2 = 1; k2 <= J.p; ++k2)
                        s1 = cadd(s1, cscale(gk[k2], J.binom[(m + k2 - 1) * kBinomStride + (k2 - 1)]));
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
        __syncthreads();
    }
}

void batch_m2l_block(const EvalJob *jobs, const BatchMap &m, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    hipLaunchKernelGGL(k_m2l_block, dim3(persistent_grid(m.pre[m.n], 64)), dim3(64), 0, s, jobs, m);
}

}  // namespace fmm
