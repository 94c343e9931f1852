// near_mixed.hip -- the P2P near field in FP32 with compensated (Kahan)
// sums; the FP64 L2P is added afterwards (near.hip).
//
// Points are held as FP32 offsets from their own leaf centre, so a pair's
// separation y - x = (t_loc - (c_S - c_T)) - s_loc is formed from small
// numbers and the leaf offset c_S - c_T, without the cancellation that
// absolute FP32 coordinates would suffer.  Per pair:
//   Re += u * ln|y - x|  = (u ln2 / 2) * log2(dx^2 + dy^2)   (hardware log2)
//   Im += u * atan2(dy, dx)                                   (own atan2)
// Both sums are compensated in FP32 (Kahan steps on blocks of eight plainly
// summed pairs) and stored in FP64 for the far field to be added to.
// A pair with a zero separation is skipped (bitwise-equal points).
#include "eval.h"

namespace fmm {

// atan(t) = t * sum_k c_k t^(2k) for 0 <= t <= 1: weighted least-squares
// fit on Chebyshev nodes (gen_atan_poly.py); max abs error 1.8e-7 in FP32.
static constexpr float kAtanPoly[8] = {9.999999114e-01f, -3.333209348e-01f, 1.997137453e-01f,
                                       -1.402941598e-01f, 9.942748199e-02f, -5.990455402e-02f,
                                       2.455700589e-02f, -4.780421207e-03f};
static constexpr float kPi = 3.14159265358979324f, kPi2 = 1.57079632679489662f;

// atan2 on the principal branch (-pi, pi]; y = -0 is treated as +0 and
// (0, 0) gives 0.  t = min/max of |x|, |y| (the max floored so that t stays
// finite), then the octant is restored.
__device__ __forceinline__ float atan2_f32(float y, float x)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const float mn = fminf(ax, ay), mx = fmaxf(fmaxf(ax, ay), 1e-30f);
    const float t = mn * __builtin_amdgcn_rcpf(mx);
    const float z = t * t;
    float p = kAtanPoly[7];
#pragma unroll
    for (int k = 6; k >= 0; --k) p = fmaf(p, z, kAtanPoly[k]);
    float a = t * p;
    a = (ay > ax) ? kPi2 - a : a;
    a = (x < 0.0f) ? kPi - a : a;
    return (y < 0.0f) ? -a : a;
}

__device__ __forceinline__ float readlane_f(float v, int k)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

// One wave per work item (a target leaf and up to 64 of its targets, one per
// lane).  The item's near cells are described once, one lane per slot (cell,
// source range, FP32 offset from the target leaf), and read back with
// readlane; sources go through LDS in chunks of 64 with the next chunk's
// loads in flight while the current one is summed (double buffer, one
// barrier per chunk).
__global__ __launch_bounds__(64) void k_near_mixed(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    __shared__ float4 sh[2][64];
    const int lane = threadIdx.x;
    const float half_ln2 = 0.34657359027997264f;
    for (int64_t item = blockIdx.x; item < bm.pre[bm.n]; item += gridDim.x) {
        const int e = batch_entry(bm, item);
        const EvalJob &J = jobs[bm.job[e]];
        double *phi = bm.phi_override ? bm.phi_override : J.phi;
        const int64_t it = item - bm.pre[e];
        if (it >= J.counts[0]) continue;
        const int32_t li = J.work_near[2 * it], st = J.work_near[2 * it + 1];
        const int64_t gid = J.leaf_off + li;
        const int32_t t = st + lane;
        const bool ok = t < J.te[gid];
        const double tcx = J.cx[gid], tcy = J.cy[gid];
        const float tlx = ok ? J.txl[t] : 0.0f, tly = ok ? J.tyl[t] : 0.0f;

        // Near-cell table, lane k = slot k; an absent or empty cell has an
        // empty range.
        const int nw = J.nw;
        int32_t mc = -1, mb = 0, me = 0;
        float mdx = 0.0f, mdy = 0.0f;
        if (lane < nw) {
            mc = J.near[li * nw + lane];
            if (mc >= 0) {
                mb = J.sb[mc];
                me = J.se[mc];
                mdx = (float)(J.cx[mc] - tcx);
                mdy = (float)(J.cy[mc] - tcy);
            }
        }
        auto beg = [&](int k) { return __builtin_amdgcn_readlane(mb, k); };
        auto end = [&](int k) { return __builtin_amdgcn_readlane(me, k); };
        float4 pf = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        auto fetch = [&](int k, int32_t base) {
            const int32_t i = base + lane;
            if (i < end(k)) {
                const float u = J.suf[i];
                pf = make_float4(J.sxl[i], J.syl[i], u * half_ln2, u);
            }
        };

        float rs = 0.0f, rc = 0.0f, is = 0.0f, ic = 0.0f;
        // Kahan step for both sums.
        auto acc = [&](float vr, float vi) {
            const float yr = vr - rc;
            const float tr = rs + yr;
            rc = (tr - rs) - yr;
            rs = tr;
            const float yi = vi - ic;
            const float ti = is + yi;
            ic = (ti - is) - yi;
            is = ti;
        };
        int k = 0;
        while (k < nw && beg(k) == end(k)) ++k;
        int32_t base = k < nw ? beg(k) : 0;
        int buf = 0;
        if (k < nw) {
            fetch(k, base);
            sh[0][lane] = pf;
        }
        __syncthreads();
        while (k < nw) {
            // The chunk after this one: the rest of this cell, else the next
            // nonempty cell.
            int k2 = k;
            int32_t base2 = base + 64;
            if (base2 >= end(k)) {
                k2 = k + 1;
                while (k2 < nw && beg(k2) == end(k2)) ++k2;
                base2 = k2 < nw ? beg(k2) : 0;
            }
            if (k2 < nw) fetch(k2, base2);

            // Slot 0 is the target leaf itself: only there can a source have
            // the target's exact coordinates (equal points share a leaf key).
            const bool self = __builtin_amdgcn_readlane(mc, k) == gid;
            const float ax = tlx - readlane_f(mdx, k);
            const float ay = tly - readlane_f(mdy, k);
            const int nsrc = end(k) - base < 64 ? end(k) - base : 64;
            const float4 *src = sh[buf];
            if (self) {
                for (int j = 0; j < nsrc; ++j) {
                    const float4 sv = src[j];
                    const float dx = ax - sv.x, dy = ay - sv.y;
                    const float r2 = fmaf(dx, dx, dy * dy);
                    const bool live = r2 > 0.0f;
                    const float lg = __log2f(live ? r2 : 1.0f);
                    const float at = atan2_f32(dy, dx);
                    acc(live ? sv.z * lg : 0.0f, live ? sv.w * at : 0.0f);
                }
            } else {
                // Distinct leaves: separations are nonzero; the 1e-37 inside
                // r^2 only keeps a pair closer than FP32 resolution finite.
                // Eight pairs are summed plainly, then Kahan-added.
                int j = 0;
                for (; j + 8 <= nsrc; j += 8) {
                    float pr = 0.0f, pi = 0.0f;
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) {
                        const float4 sv = src[j + jj];
                        const float dx = ax - sv.x, dy = ay - sv.y;
                        const float r2 = fmaf(dx, dx, fmaf(dy, dy, 1e-37f));
                        pr = fmaf(sv.z, __log2f(r2), pr);
                        pi = fmaf(sv.w, atan2_f32(dy, dx), pi);
                    }
                    acc(pr, pi);
                }
                for (; j < nsrc; ++j) {
                    const float4 sv = src[j];
                    const float dx = ax - sv.x, dy = ay - sv.y;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, 1e-37f));
                    acc(sv.z * __log2f(r2), sv.w * atan2_f32(dy, dx));
                }
            }
            if (k2 < nw) sh[buf ^ 1][lane] = pf;
            __syncthreads();
            k = k2;
            base = base2;
            buf ^= 1;
        }
        if (ok) {
            const int64_t o = J.tperm[t];
            phi[2 * o] = (double)rs - (double)rc;
            phi[2 * o + 1] = (double)is - (double)ic;
        }
    }
}

void batch_near_mixed(const EvalJob *jobs, const BatchMap &m, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    hipLaunchKernelGGL(k_near_mixed, dim3(persistent_grid(m.pre[m.n], kNearWavesPerCU)), dim3(64), 0, s, jobs, m);
}

}  // namespace fmm
