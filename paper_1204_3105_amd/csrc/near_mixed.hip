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
// summed pairs) and stored in FP64 for the far field to be added to.  The
// 1e18 padding sources have zero strength: their terms are exact zeros.
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

// One wave per work item: a target leaf and up to 64 of its targets.  With m
// targets the wave runs g = min(near slots, 64/m) groups of m lanes (one
// target per lane); the item's sources, listed cell after cell, are cut into
// g equal slices, one per group, so an item with few targets still fills the
// wave.  Each round every group
// stages the next chunk of its slice (within one cell) in LDS (64/g sources rounded
// down to a multiple of 8, at least 8; padded to a multiple of 8 with
// zero-strength sources far away) and sums it; the groups' partial sums of a
// target are added in group order at the end.  With FIELD the kernel also
// sums u / (y - x) = u (dx - i dy) / r^2 into the field's near sums
// (bm.nfield): the separation is formed in FP64 from the absolute
// coordinates (staged beside the FP32 data), since 1/r amplifies the
// rounding of FP32 offsets for close pairs, then rounded to FP32 for r^2,
// the hardware reciprocal and the same compensated sums; a pair is skipped
// only when its FP64 coordinates are equal.
template <bool FIELD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(FIELD ? 5 : 7, 8))) void k_near_mixed(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    // g (cl + 1) <= 117 for every g: 64 (g = 1), 66, 51, 68, 45, ..., 117 (g = 13);
    // at least 128 entries so that the reduction (4 x 64 doubles) fits
    __shared__ float4 sh[kNearSlots * 9 > 128 ? kNearSlots * 9 : 128];
    __shared__ int32_t cbeg[kNearSlots], cend[kNearSlots], cum[kNearSlots + 1];
    __shared__ float cdx[kNearSlots], cdy[kNearSlots];
    __shared__ double2 shd[FIELD ? kNearSlots * 9 : 1];
    double(*red)[64] = reinterpret_cast<double(*)[64]>(sh);   // after the rounds
    const int lane = threadIdx.x;
    const float half_ln2 = 0.34657359027997264f;
    for (int64_t item = blockIdx.x; item < bm.pre[bm.n]; item += gridDim.x) {
        const int e = batch_entry(bm, item);
        const EvalJob &J = jobs[bm.job[e]];
        const int64_t it = item - bm.pre[e];
        if (it >= J.counts[0]) continue;
        const int32_t li = J.work_near[2 * it], st = J.work_near[2 * it + 1];
        const int64_t gid = J.leaf_off + li;
        const int nw = J.nw;
        const int m = min(kChunk, J.te[gid] - st);
        const int g = max(1, min(nw, 64 / m));
        const int cl = max(8, (64 / g) & ~7);
        const int stride = g == 1 ? 64 : cl + 1;
        const int grp = lane / m, tau = lane - grp * m;
        const bool in = grp < g;
        const int32_t t = st + tau;
        const float tlx = in ? J.txl[t] : 0.0f, tly = in ? J.tyl[t] : 0.0f;
        const double tx = FIELD && in ? J.tx[t] : 0.0, ty = FIELD && in ? J.ty[t] : 0.0;
        const double tcx = J.cx[gid], tcy = J.cy[gid];

        // Near-cell table (slot 0 is the leaf itself); an absent cell has an
        // empty range.
        __syncthreads();   // the previous item is done with the LDS
        if (lane < nw) {
            const int32_t c = J.near[li * nw + lane];
            int32_t b0 = 0, e0 = 0;
            float dx = 0.0f, dy = 0.0f;
            if (c >= 0) {
                b0 = J.sb[c];
                e0 = J.se[c];
                dx = (float)(J.cx[c] - tcx);
                dy = (float)(J.cy[c] - tcy);
            }
            cbeg[lane] = b0;
            cend[lane] = e0;
            cdx[lane] = dx;
            cdy[lane] = dy;
        }
        __syncthreads();
        if (lane == 0) {
            int32_t a = 0;
            for (int q = 0; q < nw; ++q) {
                cum[q] = a;
                a += cend[q] - cbeg[q];
            }
            cum[nw] = a;
        }
        __syncthreads();

        float rs = 0.0f, rc = 0.0f, is = 0.0f, ic = 0.0f;
        float frs = 0.0f, frc = 0.0f, fis = 0.0f, fic = 0.0f;
        // Kahan step for a sum s with compensation c.
        auto kahan = [](float &s, float &c, float v) {
            const float y = v - c;
            const float t = s + y;
            c = (t - s) - y;
            s = t;
        };
        auto acc = [&](float vr, float vi) {
            kahan(rs, rc, vr);
            kahan(is, ic, vi);
        };
        // This lane's group sums the slice [pos, hi) of the item's sources
        // listed cell after cell; k is the cell holding pos, base its index.
        const int32_t total = cum[nw];
        int32_t pos = in ? (int32_t)((int64_t)grp * total / g) : total;
        const int32_t hi = in ? (int32_t)((int64_t)(grp + 1) * total / g) : total;
        int k = 0;
        while (k + 1 < nw && cum[k + 1] <= pos) ++k;
        int32_t base = cbeg[k] + (pos - cum[k]);
        const float4 *gsh = sh + (in ? grp : 0) * stride;
        const double2 *gshd = shd + (FIELD && in ? grp * stride : 0);
        for (;;) {
            const bool busy = pos < hi;
            if (!__any(busy)) break;
            const int n = busy ? min(min(cl, cend[k] - base), hi - pos) : 0;
            // Only group 0 meets slot 0, the one cell where a source can sit
            // at the target's exact coordinates.
            const bool self_round = __any(busy && k == 0);
            int maxn = n;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) maxn = max(maxn, __shfl_xor(maxn, o));
            const int padn = (maxn + 7) & ~7;
            if (in) {
                float4 *w = sh + grp * stride;
                for (int j = tau; j < padn; j += m) {
                    float4 v = make_float4(1e18f, 1e18f, 0.0f, 0.0f);
                    if (j < n) {
                        const int32_t i = base + j;
                        const float u = J.suf[i];
                        v = make_float4(J.sxl[i], J.syl[i], u * half_ln2, u);
                    }
                    w[j] = v;
                    if (FIELD) {
                        double2 d = make_double2(1e18, 1e18);
                        if (j < n) d = make_double2(J.sx[base + j], J.sy[base + j]);
                        shd[grp * stride + j] = d;
                    }
                }
            }
            __syncthreads();
            const float ax = tlx - (busy ? cdx[k] : 0.0f);
            const float ay = tly - (busy ? cdy[k] : 0.0f);
            if (self_round) {
                for (int j = 0; j < padn; ++j) {
                    const float4 sv = gsh[j];
                    const float dx = ax - sv.x, dy = ay - sv.y;
                    const float r2 = fmaf(dx, dx, dy * dy);
                    const bool live = r2 > 0.0f;
                    const float lg = __log2f(live ? r2 : 1.0f);
                    const float at = atan2_f32(dy, dx);
                    acc(live ? sv.z * lg : 0.0f, live ? sv.w * at : 0.0f);
                    if (FIELD) {
                        const double2 sd = gshd[j];
                        const bool on = tx != sd.x || ty != sd.y;
                        const float ex = (float)(tx - sd.x), ey = (float)(ty - sd.y);
                        const float w = on ? sv.w * __builtin_amdgcn_rcpf(fmaf(ex, ex, fmaf(ey, ey, 1e-37f))) : 0.0f;
                        kahan(frs, frc, w * ex);
                        kahan(fis, fic, -w * ey);
                    }
                }
            } else {
                // Distinct leaves: separations are nonzero; the 1e-37 inside
                // r^2 only keeps a pair closer than FP32 resolution finite.
                // Eight pairs are summed plainly, then Kahan-added.
                for (int j = 0; j < padn; j += 8) {
                    float pr = 0.0f, pi = 0.0f, qr = 0.0f, qi = 0.0f;
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) {
                        const float4 sv = gsh[j + jj];
                        const float dx = ax - sv.x, dy = ay - sv.y;
                        const float r2 = fmaf(dx, dx, fmaf(dy, dy, 1e-37f));
                        pr = fmaf(sv.z, __log2f(r2), pr);
                        pi = fmaf(sv.w, atan2_f32(dy, dx), pi);
                        if (FIELD) {
                            const double2 sd = gshd[j + jj];
                            const float ex = (float)(tx - sd.x), ey = (float)(ty - sd.y);
                            const float w = sv.w * __builtin_amdgcn_rcpf(fmaf(ex, ex, fmaf(ey, ey, 1e-37f)));
                            qr = fmaf(w, ex, qr);
                            qi = fmaf(-w, ey, qi);
                        }
                    }
                    acc(pr, pi);
                    if (FIELD) {
                        kahan(frs, frc, qr);
                        kahan(fis, fic, qi);
                    }
                }
            }
            __syncthreads();
            if (busy) {
                pos += n;
                base += n;
                if (base >= cend[k] && pos < hi) {
                    ++k;
                    while (cbeg[k] == cend[k]) ++k;   // pos < hi: a nonempty cell follows
                    base = cbeg[k];
                }
            }
        }
        red[0][lane] = (double)rs - (double)rc;   // the last round's barrier freed sh
        red[1][lane] = (double)is - (double)ic;
        if (FIELD) {
            red[2][lane] = (double)frs - (double)frc;
            red[3][lane] = (double)fis - (double)fic;
        }
        __syncthreads();
        if (grp == 0) {
            double re = 0.0, im = 0.0, fre = 0.0, fim = 0.0;
            for (int q = 0; q < g; ++q) {
                re += red[0][q * m + tau];
                im += red[1][q * m + tau];
                if (FIELD) {
                    fre += red[2][q * m + tau];
                    fim += red[3][q * m + tau];
                }
            }
            J.nsum[2 * t] = re;   // sorted order: L2P adds the far field and un-permutes
            J.nsum[2 * t + 1] = im;
            if (FIELD) {
                bm.nfield[2 * t] = fre;
                bm.nfield[2 * t + 1] = fim;
            }
        }
    }
}

void batch_near_mixed(const EvalJob *jobs, const BatchMap &m, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    const dim3 grid(persistent_grid(m.pre[m.n], kNearWavesPerCU));
    if (m.nfield) hipLaunchKernelGGL(k_near_mixed<true>, grid, dim3(64), 0, s, jobs, m);
    else hipLaunchKernelGGL(k_near_mixed<false>, grid, dim3(64), 0, s, jobs, m);
}

}  // namespace fmm
