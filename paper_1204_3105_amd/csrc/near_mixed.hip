// near_mixed.hip -- L2P (FP64) and the P2P near field in FP32 with
// compensated (Kahan) sums, fused per target leaf.
//
// Points are held as FP32 offsets from their own leaf centre, so a pair's
// separation y - x = (t_loc - (c_S - c_T)) - s_loc is formed from small
// numbers and the leaf offset c_S - c_T, without the cancellation that
// absolute FP32 coordinates would suffer.  Per pair:
//   Re += u * ln|y - x|  = (u ln2 / 2) * log2(dx^2 + dy^2)   (hardware log2)
//   Im += u * atan2(dy, dx)                                   (own atan2)
// Both sums are compensated in FP32 (Kahan steps on blocks of four plainly
// summed pairs) and added to the FP64 far field.
// A pair with a zero separation is skipped (bitwise-equal points).
#include "eval.h"

namespace fmm {

// atan(t) = t * sum_k c_k t^(2k) for |t| <= tan(pi/8): weighted least-squares
// fit on Chebyshev nodes (gen_atan_poly.py); max abs error 2.8e-8 in FP32.
static constexpr float kAtan0 = 9.999999994e-01f, kAtan1 = -3.333330808e-01f,
                       kAtan2 = 1.999823819e-01f, kAtan3 = -1.424042995e-01f,
                       kAtan4 = 1.057579194e-01f, kAtan5 = -6.040182834e-02f;
static constexpr float kTanPi8 = 0.41421356237309503f;
static constexpr float kPi = 3.14159265358979324f, kPi2 = 1.57079632679489662f,
                       kPi4 = 0.78539816339744831f;

// atan2 on the principal branch (-pi, pi]; y = -0 is treated as +0.
__device__ __forceinline__ float atan2_f32(float y, float x)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const float mn = fminf(ax, ay), mx = fmaxf(ax, ay);
    const bool big = mn > kTanPi8 * mx;   // reduce by pi/4: t = (mn - mx)/(mn + mx)
    const float num = big ? mn - mx : mn;
    const float den = big ? mn + mx : mx;
    const float t = num * __builtin_amdgcn_rcpf(den);
    const float z = t * t;
    float p = kAtan5;
    p = fmaf(p, z, kAtan4);
    p = fmaf(p, z, kAtan3);
    p = fmaf(p, z, kAtan2);
    p = fmaf(p, z, kAtan1);
    p = fmaf(p, z, kAtan0);
    float a = fmaf(t, p, big ? kPi4 : 0.0f);
    a = (ay > ax) ? kPi2 - a : a;
    a = (x < 0.0f) ? kPi - a : a;
    return (y < 0.0f) ? -a : a;
}

__global__ __launch_bounds__(64) void k_near_mixed(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    __shared__ float4 sh[64];
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

        // L2P in FP64.
        double fr = 0.0, fi = 0.0;
        float tlx = 0.0f, tly = 0.0f;
        if (ok) {
            const int P1 = J.p + 1;
            const double *b = J.lc + gid * 2 * P1;
            const double inv = 1.0 / J.scale[J.L];
            const double zr = (J.tx[t] - tcx) * inv, zi = (J.ty[t] - tcy) * inv;
            fr = b[2 * J.p];
            fi = b[2 * J.p + 1];
            for (int m = J.p - 1; m >= 0; --m) {
                const double nr = fr * zr - fi * zi + b[2 * m];
                const double ni = fr * zi + fi * zr + b[2 * m + 1];
                fr = nr;
                fi = ni;
            }
            tlx = J.txl[t];
            tly = J.tyl[t];
        }

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
        for (int k = 0; k < J.nw; ++k) {
            // Slot 0 is the target leaf itself: only there can a source have
            // the target's exact coordinates (equal points share a leaf key).
            const int32_t c = __builtin_amdgcn_readfirstlane(J.near[li * J.nw + k]);
            if (c < 0) continue;
            const bool self = c == gid;
            const float ax = tlx - (float)(J.cx[c] - tcx);
            const float ay = tly - (float)(J.cy[c] - tcy);
            const int32_t b0 = __builtin_amdgcn_readfirstlane(J.sb[c]);
            const int32_t e0 = __builtin_amdgcn_readfirstlane(J.se[c]);
            for (int32_t base = b0; base < e0; base += 64) {
                __syncthreads();
                const int32_t i = base + lane;
                if (i < e0) {
                    const float u = J.suf[i];
                    sh[lane] = make_float4(J.sxl[i], J.syl[i], u * half_ln2, u);
                }
                __syncthreads();
                const int nsrc = e0 - base < 64 ? e0 - base : 64;
                if (self) {
                    for (int j = 0; j < nsrc; ++j) {
                        const float4 sv = sh[j];
                        const float dx = ax - sv.x, dy = ay - sv.y;
                        const float r2 = fmaf(dx, dx, dy * dy);
                        const bool live = r2 > 0.0f;
                        const float lg = __log2f(live ? r2 : 1.0f);
                        const float at = atan2_f32(dy, dx);
                        acc(live ? sv.z * lg : 0.0f, live ? sv.w * at : 0.0f);
                    }
                } else {
                    // Distinct leaves: separations are nonzero; the floor
                    // only keeps a pair closer than FP32 resolution finite.
                    // Four pairs are summed plainly, then Kahan-added.
                    int j = 0;
                    for (; j + 4 <= nsrc; j += 4) {
                        float pr = 0.0f, pi = 0.0f;
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) {
                            const float4 sv = sh[j + jj];
                            const float dx = ax - sv.x, dy = ay - sv.y;
                            const float r2 = fmaxf(fmaf(dx, dx, dy * dy), 1e-37f);
                            pr = fmaf(sv.z, __log2f(r2), pr);
                            pi = fmaf(sv.w, atan2_f32(dy, dx), pi);
                        }
                        acc(pr, pi);
                    }
                    for (; j < nsrc; ++j) {
                        const float4 sv = sh[j];
                        const float dx = ax - sv.x, dy = ay - sv.y;
                        const float r2 = fmaxf(fmaf(dx, dx, dy * dy), 1e-37f);
                        acc(sv.z * __log2f(r2), sv.w * atan2_f32(dy, dx));
                    }
                }
            }
        }
        if (ok) {
            const int64_t o = J.tperm[t];
            phi[2 * o] = fr + ((double)rs - (double)rc);
            phi[2 * o + 1] = fi + ((double)is - (double)ic);
        }
    }
}

void batch_near_mixed(const EvalJob *jobs, const BatchMap &m, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    hipLaunchKernelGGL(k_near_mixed, dim3(persistent_grid(m.pre[m.n], 128)), dim3(64), 0, s, jobs, m);
}

}  // namespace fmm
