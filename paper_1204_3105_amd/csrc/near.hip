// near.hip -- the P2P near field (FP64) and L2P.
//
// Each work item is one target leaf and up to 64 of its targets (one wave,
// one target per lane).  P2P sums u_i Log(y - x_i) over the sources of the
// leaf and its neighbours ({T} u Neighbors(T), paper Sec. 4), staged through
// LDS 64 at a time: Re = ln|y - x| = 0.5 ln(dx^2 + dy^2), Im = atan2(dy, dx)
// with a -0 dy read as +0; a source with the target's exact coordinates is
// skipped.  It writes the near sum in the caller's target order and runs
// beside the far-field passes; L2P then adds the leaf's local expansion
// (Greengard-Rokhlin evaluation of sum_m b~_m ((y - c)/ell)^m, Horner).
#include "eval.h"

namespace fmm {

__global__ __launch_bounds__(64) void k_near_fp64(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    __shared__ double shx[64], shy[64], shu[64];
    const int lane = threadIdx.x;
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
        const double y0 = ok ? J.tx[t] : 0.0, y1 = ok ? J.ty[t] : 0.0;

        // P2P
        double re = 0.0, im = 0.0;
        for (int k = 0; k < J.nw; ++k) {
            const int32_t c = J.near[li * J.nw + k];
            if (c < 0) continue;
            const int32_t b0 = J.sb[c], e0 = J.se[c];
            for (int32_t base = b0; base < e0; base += 64) {
                __syncthreads();
                const int32_t i = base + lane;
                if (i < e0) {
                    shx[lane] = J.sx[i];
                    shy[lane] = J.sy[i];
                    shu[lane] = J.su[i];
                }
                __syncthreads();
                const int nsrc = e0 - base < 64 ? e0 - base : 64;
                for (int j = 0; j < nsrc; ++j) {
                    const double dx = y0 - shx[j], dy = y1 - shy[j];
                    if (dx == 0.0 && dy == 0.0) continue;
                    const double u = shu[j];
                    re += u * (0.5 * log(dx * dx + dy * dy));
                    im += u * atan2(dy + 0.0, dx);
                }
            }
        }
        if (ok) {
            const int64_t o = J.tperm[t];
            phi[2 * o] = re;
            phi[2 * o + 1] = im;
        }
    }
}

// L2P: phi += the target leaf's local expansion, FP64 Horner (same items).
// The leaf's coefficient row is staged in LDS by the whole wave first, so the
// Horner loop reads broadcast LDS instead of a chain of dependent loads.
__global__ __launch_bounds__(64) void k_l2p(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    __shared__ double row[2 * (kMaxP + 1)];
    const int lane = threadIdx.x;
    for (int64_t item = blockIdx.x; item < bm.pre[bm.n]; item += gridDim.x) {
        const int e = batch_entry(bm, item);
        const EvalJob &J = jobs[bm.job[e]];
        double *phi = bm.phi_override ? bm.phi_override : J.phi;
        const int64_t it = item - bm.pre[e];
        if (it >= J.counts[0]) continue;   // uniform across the wave
        const int32_t li = J.work_near[2 * it], st = J.work_near[2 * it + 1];
        const int64_t gid = J.leaf_off + li;
        const int P1 = J.p + 1;
        const double *b = J.lc + gid * 2 * P1;
        __syncthreads();
        if (lane < 2 * P1) row[lane] = b[lane];
        if (lane + 64 < 2 * P1) row[lane + 64] = b[lane + 64];
        __syncthreads();
        const int32_t t = st + lane;
        if (t >= J.te[gid]) continue;
        const double inv = 1.0 / J.scale[J.L];
        const double zr = (J.tx[t] - J.cx[gid]) * inv, zi = (J.ty[t] - J.cy[gid]) * inv;
        double fr = row[2 * J.p], fi = row[2 * J.p + 1];
        for (int m = J.p - 1; m >= 0; --m) {
            const double nr = fr * zr - fi * zi + row[2 * m];
            const double ni = fr * zi + fi * zr + row[2 * m + 1];
            fr = nr;
            fi = ni;
        }
        const int64_t o = J.tperm[t];
        phi[2 * o] = phi[2 * o] + fr;
        phi[2 * o + 1] = phi[2 * o + 1] + fi;
    }
}

void batch_near_fp64(const EvalJob *jobs, const BatchMap &m, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    hipLaunchKernelGGL(k_near_fp64, dim3(persistent_grid(m.pre[m.n], kNearWavesPerCU)), dim3(64), 0, s, jobs, m);
}

void batch_l2p(const EvalJob *jobs, const BatchMap &m, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    hipLaunchKernelGGL(k_l2p, dim3(persistent_grid(m.pre[m.n], 64)), dim3(64), 0, s, jobs, m);
}

}  // namespace fmm
