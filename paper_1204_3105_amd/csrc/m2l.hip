// m2l.hip -- multipole-to-local translation, FP64, one target cell per lane.
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
