// near_mixed.hip -- L2P (FP64) and the P2P near field in FP32 with
// compensated (Kahan) sums, fused per target leaf.
//
// Points are held as FP32 offsets from their own leaf centre, so a pair's
// separation y - x = (t_loc - (c_S - c_T)) - s_loc is formed from small
// numbers and the leaf offset c_S - c_T, without the cancellation that
// absolute FP32 coordinates would suffer.  Per pair:
//   Re += u * ln|y - x|  = (u ln2 / 2) * log2(dx^2 + dy^2)   (hardware log2)
//   Im += u * atan2(dy, dx)                                   (own atan2)
// Both sums are Kahan-compensated in FP32 and added to the FP64 far field.
// A pair with a zero separation is skipped (bitwise-equal points).
#include "fmm_internal.h"

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

struct NearMixedParams {
    int p;
    int nw;
    int64_t leaf_off;
    double inv_scale;
};

__global__ __launch_bounds__(64) void k_near_mixed(NearMixedParams q, const int32_t *__restrict__ items,
                                                   const int32_t *__restrict__ near,
                                                   const int32_t *__restrict__ sb,
                                                   const int32_t *__restrict__ se,
                                                   const int32_t *__restrict__ te,
                                                   const double *__restrict__ cx,
                                                   const double *__restrict__ cy,
                                                   const float *__restrict__ sxl,
                                                   const float *__restrict__ syl,
                                                   const float *__restrict__ suf,
                                                   const double *__restrict__ tx,
                                                   const double *__restrict__ ty,
                                                   const float *__restrict__ txl,
                                                   const float *__restrict__ tyl,
                                                   const int32_t *__restrict__ tperm,
                                                   const double *__restrict__ lc,
                                                   double *__restrict__ phi)
{
    __shared__ float4 sh[64];
    const int lane = threadIdx.x;
    const int32_t li = items[2 * blockIdx.x], st = items[2 * blockIdx.x + 1];
    const int64_t gid = q.leaf_off + li;
    const int32_t t = st + lane;
    const bool ok = t < te[gid];
    const double tcx = cx[gid], tcy = cy[gid];

    // L2P in FP64.
    double fr = 0.0, fi = 0.0;
    float tlx = 0.0f, tly = 0.0f;
    if (ok) {
        const int P1 = q.p + 1;
        const double *b = lc + gid * 2 * P1;
        const double zr = (tx[t] - tcx) * q.inv_scale, zi = (ty[t] - tcy) * q.inv_scale;
        fr = b[2 * q.p];
        fi = b[2 * q.p + 1];
        for (int m = q.p - 1; m >= 0; --m) {
            const double nr = fr * zr - fi * zi + b[2 * m];
            const double ni = fr * zi + fi * zr + b[2 * m + 1];
            fr = nr;
            fi = ni;
        }
        tlx = txl[t];
        tly = tyl[t];
    }

    float rs = 0.0f, rc = 0.0f, is = 0.0f, ic = 0.0f;
    const float half_ln2 = 0.34657359027997264f;
    for (int k = 0; k < q.nw; ++k) {
        const int32_t c = near[li * q.nw + k];
        if (c < 0) continue;
        const float ax = tlx - (float)(cx[c] - tcx);
        const float ay = tly - (float)(cy[c] - tcy);
        const int32_t b0 = sb[c], e0 = se[c];
        for (int32_t base = b0; base < e0; base += 64) {
            __syncthreads();
            const int32_t i = base + lane;
            if (i < e0) {
                const float u = suf[i];
                sh[lane] = make_float4(sxl[i], syl[i], u * half_ln2, u);
            }
            __syncthreads();
            const int n = e0 - base < 64 ? e0 - base : 64;
            for (int j = 0; j < n; ++j) {
                const float4 s = sh[j];
                const float dx = ax - s.x, dy = ay - s.y;
                const float r2 = fmaf(dx, dx, dy * dy);
                const bool live = r2 > 0.0f;
                const float lg = __log2f(live ? r2 : 1.0f);
                const float at = atan2_f32(dy, dx);
                const float vr = live ? s.z * lg : 0.0f;
                const float vi = live ? s.w * at : 0.0f;
                // Kahan steps
                const float yr = vr - rc;
                const float tr = rs + yr;
                rc = (tr - rs) - yr;
                rs = tr;
                const float yi = vi - ic;
                const float ti = is + yi;
                ic = (ti - is) - yi;
                is = ti;
            }
        }
    }
    if (ok) {
        const int64_t o = tperm[t];
        phi[2 * o] = fr + ((double)rs - (double)rc);
        phi[2 * o + 1] = fi + ((double)is - (double)ic);
    }
}

void launch_near_mixed(const Plan &P, double *phi, hipStream_t s)
{
    if (P.n_work_near <= 0) return;
    NearMixedParams q;
    q.p = P.p;
    q.nw = P.tables.near_width;
    q.leaf_off = P.lev[P.geo.L].cell_off;
    q.inv_scale = 1.0 / P.scale[P.geo.L];
    hipLaunchKernelGGL(k_near_mixed, dim3((unsigned)P.n_work_near), dim3(64), 0, s, q, P.work_near,
                       P.near, P.sb, P.se, P.te, P.cx, P.cy, P.sxl, P.syl, P.suf, P.tx, P.ty, P.txl,
                       P.tyl, P.tperm, P.lc, phi);
}

}  // namespace fmm
