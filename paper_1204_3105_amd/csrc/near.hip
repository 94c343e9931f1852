// near.hip -- L2P and the P2P near field, fused per target leaf (FP64).
//
// Each work item is one target leaf and up to 64 of its targets (one wave,
// one target per lane).  The lane evaluates the leaf's local expansion
// (Greengard-Rokhlin evaluation of sum_m b~_m ((y - c)/ell)^m, Horner) and
// then sums u_i Log(y - x_i) over the sources of the leaf and its
// neighbours ({T} u Neighbors(T), paper Sec. 4), staged through LDS 64 at a
// time.  Re = ln|y - x| = 0.5 ln(dx^2 + dy^2), Im = atan2(dy, dx) with a
// -0 dy read as +0; a source with the target's exact coordinates is
// skipped.  The result is written in the caller's target order.
#include "fmm_internal.h"

namespace fmm {

struct NearParams {
    int p;
    int nw;
    int64_t leaf_off;
    double inv_scale;
};

__global__ __launch_bounds__(64) void k_near_fp64(NearParams q, const int32_t *__restrict__ items,
                                                  const int32_t *__restrict__ near,
                                                  const int32_t *__restrict__ sb,
                                                  const int32_t *__restrict__ se,
                                                  const int32_t *__restrict__ tb,
                                                  const int32_t *__restrict__ te,
                                                  const double *__restrict__ cx,
                                                  const double *__restrict__ cy,
                                                  const double *__restrict__ sx,
                                                  const double *__restrict__ sy,
                                                  const double *__restrict__ su,
                                                  const double *__restrict__ tx,
                                                  const double *__restrict__ ty,
                                                  const int32_t *__restrict__ tperm,
                                                  const double *__restrict__ lc,
                                                  double *__restrict__ phi)
{
    __shared__ double shx[64], shy[64], shu[64];
    const int lane = threadIdx.x;
    const int32_t li = items[2 * blockIdx.x], st = items[2 * blockIdx.x + 1];
    const int64_t gid = q.leaf_off + li;
    const int32_t t = st + lane;
    const bool ok = t < te[gid];
    const double y0 = ok ? tx[t] : 0.0, y1 = ok ? ty[t] : 0.0;

    // L2P
    const int P1 = q.p + 1;
    const double *b = lc + gid * 2 * P1;
    double zr = (y0 - cx[gid]) * q.inv_scale, zi = (y1 - cy[gid]) * q.inv_scale;
    double fr = b[2 * q.p], fi = b[2 * q.p + 1];
    for (int m = q.p - 1; m >= 0; --m) {
        double nr = fr * zr - fi * zi + b[2 * m];
        double ni = fr * zi + fi * zr + b[2 * m + 1];
        fr = nr;
        fi = ni;
    }

    // P2P
    double re = 0.0, im = 0.0;
    for (int k = 0; k < q.nw; ++k) {
        int32_t c = near[li * q.nw + k];
        if (c < 0) continue;
        const int32_t b0 = sb[c], e0 = se[c];
        for (int32_t base = b0; base < e0; base += 64) {
            __syncthreads();
            int32_t i = base + lane;
            if (i < e0) {
                shx[lane] = sx[i];
                shy[lane] = sy[i];
                shu[lane] = su[i];
            }
            __syncthreads();
            int n = e0 - base < 64 ? e0 - base : 64;
            for (int j = 0; j < n; ++j) {
                double dx = y0 - shx[j], dy = y1 - shy[j];
                if (dx == 0.0 && dy == 0.0) continue;
                double u = shu[j];
                re += u * (0.5 * log(dx * dx + dy * dy));
                im += u * atan2(dy + 0.0, dx);
            }
        }
    }
    if (ok) {
        int64_t o = tperm[t];
        phi[2 * o] = fr + re;
        phi[2 * o + 1] = fi + im;
    }
}

void launch_near_fp64(const Plan &P, const double *dummy, double *phi, hipStream_t s)
{
    (void)dummy;
    if (P.n_work_near <= 0) return;
    NearParams q;
    q.p = P.p;
    q.nw = P.tables.near_width;
    q.leaf_off = P.lev[P.geo.L].cell_off;
    q.inv_scale = 1.0 / P.scale[P.geo.L];
    hipLaunchKernelGGL(k_near_fp64, dim3((unsigned)P.n_work_near), dim3(64), 0, s, q, P.work_near,
                       P.near, P.sb, P.se, P.tb, P.te, P.cx, P.cy, P.sx, P.sy, P.su, P.tx, P.ty,
                       P.tperm, P.lc, phi);
}

}  // namespace fmm
