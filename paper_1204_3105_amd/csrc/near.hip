// near.hip -- the P2P near field (FP64) and L2P.
//
// Each work item is one target leaf and up to 64 of its targets (one wave,
// one target per lane).  P2P sums u_i Log(y - x_i) over the sources of the
// leaf and its neighbours ({T} u Neighbors(T), paper Sec. 4), staged through
// LDS 64 at a time: Re = ln|y - x| = 0.5 ln(dx^2 + dy^2), Im = atan2(dy, dx)
// with a -0 dy read as +0; a source with the target's exact coordinates is
// skipped.  ln and atan2 are evaluated by the FP64 routines below.  It writes
// the near sums in sorted target order and runs beside the far-field passes;
// L2P then adds the leaf's local expansion (Greengard-Rokhlin evaluation of
// sum_m b~_m ((y - c)/ell)^m, Horner) and writes Phi in the caller's order.
#include <algorithm>

#include <type_traits>

#include "eval.h"

namespace fmm {

// ------------------------------------------------------------ FP64 math
// Constants from gen_f64_consts.py (series in 60-digit arithmetic).
static constexpr double kLn2Hi = 0.6931471803691238, kLn2Lo = 1.9082149292705877e-10;
static constexpr double kPiHi = 3.141592653589793, kPiLo = 1.2246467991473532e-16;
static constexpr double kPi2Hi = 1.5707963267948966, kPi2Lo = 6.123233995736766e-17;
static constexpr double kPi6Hi = 0.5235987755982989, kPi6Lo = -5.360408832255455e-17;
static constexpr double kInvSqrt3 = 0.5773502691896257, kTanPi12 = 0.2679491924311227;
static constexpr double kSqrtHalf = 0.7071067811865476;
// ln c for c = kSqrtHalf, the rounded sqrt(1/2).
static constexpr double kLnC = -0.3465735902799726;
// Series remainders on the reduced intervals, weighted minimax fits from
// gen_f64_poly.py: ln m = 2s (1 + z P(z)) with z = s^2 <= (3 - 2 sqrt2)^2
// (|z dP| <= 1.3e-18), atan t = t (1 + w Q(w)) with w = t^2 <= (2 - sqrt3)^2
// (|w dQ| <= 1.6e-17); coefficient k multiplies z^k (w^k).
static constexpr double kLnPoly[7] = {0.3333333333333367, 0.19999999999707335, 0.14285714371194552, 0.11111099286525694, 0.090917821661685105, 0.076570252032999594, 0.073979755249923215};
// kLnPoly scaled for the doubled variables s2 = 2s, z4 = s2^2 = 4z:
// z P(z) = z4 P4(z4) with coefficient k of P4 = that of P / 4^(k+1) (powers
// of two, so every Horner step is the same number scaled exactly).
static constexpr double kLnPoly4[7] = {kLnPoly[0] / 4, kLnPoly[1] / 16, kLnPoly[2] / 64, kLnPoly[3] / 256,
                                       kLnPoly[4] / 1024, kLnPoly[5] / 4096, kLnPoly[6] / 16384};
static constexpr double kAtanPoly64[8] = {-0.33333333333331033, 0.19999999998955142, -0.14285714123172341, 0.11111098862513553, -0.090903969460381456, 0.076797606015821029, -0.064863446745019704, 0.044493669821161291};

__device__ __forceinline__ double ln_poly(double z)
{
    double p = kLnPoly[6];
    p = fma(p, z, kLnPoly[5]);
    p = fma(p, z, kLnPoly[4]);
    p = fma(p, z, kLnPoly[3]);
    p = fma(p, z, kLnPoly[2]);
    p = fma(p, z, kLnPoly[1]);
    return fma(p, z, kLnPoly[0]);
}

__device__ __forceinline__ double ln_poly4(double z4)
{
    double p = kLnPoly4[6];
    p = fma(p, z4, kLnPoly4[5]);
    p = fma(p, z4, kLnPoly4[4]);
    p = fma(p, z4, kLnPoly4[3]);
    p = fma(p, z4, kLnPoly4[2]);
    p = fma(p, z4, kLnPoly4[1]);
    return fma(p, z4, kLnPoly4[0]);
}

__device__ __forceinline__ double atan_poly(double w)
{
    double q = kAtanPoly64[7];
    q = fma(q, w, kAtanPoly64[6]);
    q = fma(q, w, kAtanPoly64[5]);
    q = fma(q, w, kAtanPoly64[4]);
    q = fma(q, w, kAtanPoly64[3]);
    q = fma(q, w, kAtanPoly64[2]);
    q = fma(q, w, kAtanPoly64[1]);
    return fma(q, w, kAtanPoly64[0]);
}

// n / d for d in a safe range (no zero, infinity or denormal): hardware
// reciprocal, two Newton steps, one residual correction.
__device__ __forceinline__ double div_f64(double n, double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    const double q = n * r;
    return fma(r, fma(-d, q, n), q);
}

// ln x for a positive normal x (Cody & Waite): x = 2^e m, m in
// [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s), s = (m - 1)/(m + 1),
// |s| <= 3 - 2 sqrt(2); atanh(s)/s = 1 + z P(z), z = s^2 (ln_poly, error
// below 1.3e-18); e ln 2 in two parts.
__device__ __forceinline__ double ln_f64(double x)
{
    int e;
    double m = frexp(x, &e);   // m in [1/2, 1)
    const bool lo = m < kSqrtHalf;
    m = lo ? 2.0 * m : m;
    e = lo ? e - 1 : e;
    const double s = div_f64(m - 1.0, m + 1.0);
    const double z = s * s;
    const double p = ln_poly(z);
    const double lm = 2.0 * s + 2.0 * s * (z * p);
    const double de = (double)e;
    return fma(de, kLn2Hi, fma(de, kLn2Lo, lm));
}

// atan2(y, x) on (-pi, pi], y = -0 read as +0, (x, y) != (0, 0) (Cody &
// Waite): with mn, mx = min, max of |x|, |y|, t = mn/mx in [0, 1]; above
// tan(pi/12) the addition formula with k = 1/sqrt(3) gives
// atan t = pi/6 + atan((mn - k mx)/(mx + k mn)), so one division serves
// both ranges; atan(t) = t (1 + w Q(w)), w = t^2, for |t| <= tan(pi/12)
// (atan_poly, error below 1.6e-17); then the octant.
__device__ __forceinline__ double atan2_f64(double y, double x)
{
    const double ax = fabs(x), ay = fabs(y);
    const double mn = fmin(ax, ay), mx = fmax(ax, ay);
    const bool red = mn > kTanPi12 * mx;
    const double num = red ? fma(-kInvSqrt3, mx, mn) : mn;
    const double den = red ? fma(kInvSqrt3, mn, mx) : mx;
    const double t = div_f64(num, den);
    const double z = t * t;
    const double p = atan_poly(z);
    double a = fma(t * z, p, t);
    a = red ? kPi6Hi + (kPi6Lo + a) : a;
    a = (ay > ax) ? kPi2Hi + (kPi2Lo - a) : a;
    a = (x < 0.0) ? kPiHi + (kPiLo - a) : a;
    return (y < 0.0) ? -a : a;
}


// ln(r2) and the angle of (|x|, |y|) in [0, pi/2] together, as ln_f64 and
// atan2_f64 but with one reciprocal for both divisions.  The logarithm's
// reduction is shifted so that frexp's mantissa m in [1/2, 1) needs no
// adjustment: with c = sqrt(1/2) (rounded), s = (m - c)/(m + c) covers the
// same interval |s| <= 3 - 2 sqrt2 as (m' - 1)/(m' + 1) for m' in
// [sqrt(1/2), sqrt2), and ln r2 = e ln 2 + ln c + 2 atanh(s).  With
// D = (m + c) den and R = 1/D, s2 = 2s = 2(m - c) den R (2(m - c) exact) and
// t = num (m + c) R; each quotient is within a few ulp, far below what the
// FP64 near field needs.  R refines the hardware reciprocal R0 (relative error
// d = 1 - D R0) as R0 (1 + d + d^2), leaving d^3.  The pi/6 rotation of
// atan2_f64 is applied with a 0/1 factor instead of selects; with the factor
// 0 every step returns its input unchanged.
__device__ __forceinline__ void ln_angle_f64(double r2, double ax, double ay, double &lnr2, double &a)
{
    int e;
    const double m = frexp(r2, &e);   // m in [1/2, 1)
    const double mn = fmin(ax, ay), mx = fmax(ax, ay);
    const double rot = mn > kTanPi12 * mx ? 1.0 : 0.0;
    const double k = rot * kInvSqrt3;
    const double num = fma(-k, mx, mn), den = fma(k, mn, mx);
    const double mpc = m + kSqrtHalf;
    const double D = mpc * den;
    const double R0 = __builtin_amdgcn_rcp(D);
    const double d = fma(-D, R0, 1.0);
    const double R = fma(R0, fma(d, d, d), R0);
    const double s2 = (fma(m, 2.0, -2.0 * kSqrtHalf) * den) * R;
    const double t = (num * mpc) * R;
    const double z4 = s2 * s2;
    const double lm = fma(s2, z4 * ln_poly4(z4), s2);   // 2 atanh(s)
    const double de = (double)e;
    lnr2 = fma(de, kLn2Hi, fma(de, kLn2Lo, lm + kLnC));
    const double w = t * t;
    a = fma(t * w, atan_poly(w), t);
    a = fma(rot, kPi6Hi, fma(rot, kPi6Lo, a));
    a = (ay > ax) ? kPi2Hi + (kPi2Lo - a) : a;
}

// ln(r2) and atan2(y, x) on (-pi, pi] (y = -0 read as +0).
__device__ __forceinline__ void ln_atan2_f64(double r2, double y, double x, double &lnr2, double &at)
{
    double a;
    ln_angle_f64(r2, fabs(x), fabs(y), lnr2, a);
    a = (x < 0.0) ? kPiHi + (kPiLo - a) : a;
    at = (y < 0.0) ? -a : a;
}

// One wave per work item, laid out as the FP32 kernel: g = min(near slots,
// 64/m) groups of m target lanes, group q summing the q-th of g equal slices
// of the item's sources (listed cell after cell) in rounds of LDS-staged
// chunks (64/g sources rounded down to a multiple of
// 8, at least 8, padded with zero-strength sources far away); the groups'
// partial sums are added in group order.  Only slot 0, the leaf itself, can
// hold a source at the target's exact position (equal points share a key),
// so only rounds that include it test for zero separation.  With FIELD the
// kernel also sums u / (y - x) = u (dx - i dy) / r^2 into the field's near
// sums (bm.nfield).
template <bool FIELD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(FIELD ? 3 : 4, 8))) void k_near_fp64(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    constexpr int kStage = kNearSlots * 9;   // g (cl + 1) <= 117 for every g
    __shared__ double shbuf[3 * kStage];
    __shared__ int32_t cbeg[kNearSlots], cend[kNearSlots], cum[kNearSlots + 1];
    double *const shx = shbuf, *const shy = shbuf + kStage, *const shu = shbuf + 2 * kStage;
    double(*red)[64] = reinterpret_cast<double(*)[64]>(shbuf);   // after the rounds
    static_assert(3 * kStage >= 4 * 64, "reduction buffer");
    const int lane = threadIdx.x;
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
        const int stride = cl + 1;
        const int grp = lane / m, tau = lane - grp * m;
        const bool in = grp < g;
        const int32_t t = st + tau;
        const double y0 = in ? J.tx[t] : 0.0, y1 = in ? J.ty[t] : 0.0;

        __syncthreads();   // the previous item is done with the LDS
        if (lane < nw) {
            const int32_t c = J.near[li * nw + lane];
            cbeg[lane] = c >= 0 ? J.sb[c] : 0;
            cend[lane] = c >= 0 ? J.se[c] : 0;
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

        double re = 0.0, im = 0.0, fr = 0.0, fi = 0.0;
        // This lane's group sums the slice [pos, hi) of the item's sources
        // listed cell after cell; k is the cell holding pos, base its index.
        const int32_t total = cum[nw];
        int32_t pos = in ? (int32_t)((int64_t)grp * total / g) : total;
        const int32_t hi = in ? (int32_t)((int64_t)(grp + 1) * total / g) : total;
        int k = 0;
        while (k + 1 < nw && cum[k + 1] <= pos) ++k;
        int32_t base = cbeg[k] + (pos - cum[k]);
        const int goff = (in ? grp : 0) * stride;
        for (;;) {
            const bool busy = pos < hi;
            if (!__any(busy)) break;
            const int n = busy ? min(min(cl, cend[k] - base), hi - pos) : 0;
            const bool self_round = __any(busy && k == 0);
            int maxn = n;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) maxn = max(maxn, __shfl_xor(maxn, o));
            const int padn = (maxn + 7) & ~7;
            if (in) {
                for (int j = tau; j < padn; j += m) {
                    double x = 1e100, y = 1e100, u = 0.0;
                    if (j < n) {
                        const int32_t i = base + j;
                        x = J.sx[i];
                        y = J.sy[i];
                        u = J.su[i];
                    }
                    shx[grp * stride + j] = x;
                    shy[grp * stride + j] = y;
                    shu[grp * stride + j] = u;
                }
            }
            __syncthreads();
            const double *sx = shx + goff, *sy = shy + goff, *su = shu + goff;
            if (self_round) {
                for (int j = 0; j < padn; ++j) {
                    const double dx = y0 - sx[j], dy = y1 - sy[j];
                    const double r2 = dx * dx + dy * dy;
                    const bool live = r2 > 0.0;
                    double lg, at;
                    ln_atan2_f64(live ? r2 : 1.0, dy, live ? dx : 1.0, lg, at);
                    re = fma(live ? su[j] : 0.0, lg, re);   // halved at the end
                    im = fma(live ? su[j] : 0.0, at, im);
                    if (FIELD) {
                        const double w = live ? div_f64(su[j], r2) : 0.0;
                        fr = fma(w, dx, fr);
                        fi = fma(-w, dy, fi);
                    }
                }
            } else {
#pragma unroll 2
                for (int j = 0; j < padn; ++j) {   // padn is a multiple of 8
                    const double dx = y0 - sx[j], dy = y1 - sy[j];
                    const double u = su[j];
                    const double r2 = dx * dx + dy * dy;
                    double lg, at;
                    ln_atan2_f64(r2, dy, dx, lg, at);
                    re = fma(u, lg, re);
                    im = fma(u, at, im);
                    if (FIELD) {
                        const double w = div_f64(u, r2);
                        fr = fma(w, dx, fr);
                        fi = fma(-w, dy, fi);
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
        red[0][lane] = 0.5 * re;   // ln r = ln(r2) / 2; the last round's barrier freed the staging buffers
        red[1][lane] = im;
        if (FIELD) {
            red[2][lane] = fr;
            red[3][lane] = fi;
        }
        __syncthreads();
        if (grp == 0) {
            double sr = 0.0, si = 0.0, sfr = 0.0, sfi = 0.0;
            for (int q = 0; q < g; ++q) {
                sr += red[0][q * m + tau];
                si += red[1][q * m + tau];
                if (FIELD) {
                    sfr += red[2][q * m + tau];
                    sfi += red[3][q * m + tau];
                }
            }
            J.nsum[2 * t] = sr;   // sorted order: L2P adds the far field and un-permutes
            J.nsum[2 * t + 1] = si;
            if (FIELD) {
                bm.nfield[2 * t] = sfr;
                bm.nfield[2 * t + 1] = sfi;
            }
        }
    }
}

// L2P: phi (caller's order) = near sum (sorted order) + the target leaf's
// local expansion, FP64 Horner (same items).  For the base-4 tilings, in a
// tree of two or more levels, the leaf level's L2L is done here too: the leaf's row (written by
// M2L) gets its parent's local expansion shifted to the leaf's centre,
//   b~_m += rho^m sum_{k>=m} C(k, m) w^(k-m) b~par_k,
// w = (c_leaf - c_parent)/ell_(L-1), rho = ell_L/ell_(L-1) (lane m, powers
// of w and the parent row in LDS), which saves that level's launch and a
// pass over the leaves' rows.  With FIELD also the field:
// near field sum + the expansion's derivative (Horner carries both; the
// radius scaling contributes a factor 1/ell).
// The leaf's coefficient row is staged in LDS by the whole wave first, so the
// Horner loop reads broadcast LDS instead of a chain of dependent loads.
template <bool FIELD>
__global__ __launch_bounds__(64) void k_l2p(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    static_assert(kChunk <= 64 && kMaxP + 1 <= 64, "one item per wave, a lane per coefficient");
    __shared__ double row[2 * (kMaxP + 1)];
    __shared__ double bpr[kMaxP + 1], bpi[kMaxP + 1], wpr[kMaxP + 1], wpi[kMaxP + 1];
    __shared__ int8_t bsn[kNearSlots];   // chunks of each lower neighbour that wrote second sides
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
        // The lane's target data is requested before the row is staged, so
        // all of the item's loads are in flight together.
        const int32_t t = st + lane;
        const bool inb = lane < kChunk && t < J.n_tgt;
        const double tx = inb ? J.tx[t] : 0.0, ty = inb ? J.ty[t] : 0.0;
        const double n0 = inb ? J.nsum[2 * t] : 0.0, n1 = inb ? J.nsum[2 * t + 1] : 0.0;
        const int64_t o = inb ? J.tperm[t] : 0;
        double f0 = 0.0, f1 = 0.0;
        if (FIELD && inb) {
            f0 = bm.nfield[2 * t];
            f1 = bm.nfield[2 * t + 1];
        }
        const int32_t te = J.te[gid];
        const double cx = J.cx[gid], cy = J.cy[gid];
        const bool shift = J.L >= 2 && J.base == 4;   // the septree's L2L keeps its lane form
        // With the symmetric near field, each lower neighbour (by cell id)
        // with at most kSymChunks chunks left this leaf's second-side sums,
        // one per chunk of it.
        const bool two = (J.bside != nullptr || J.bside64 != nullptr) && bm.nfield == nullptr;
        __syncthreads();
        if (two && lane < J.nw) {
            int nch = 0;
            const int32_t c = lane ? J.near[li * J.nw + lane] : -1;
            if (c >= 0 && c < gid) {
                nch = sym_chunks(J.se[c] - J.sb[c], J.bside64 ? kWide : kChunk);
                if (nch > kSymChunks) nch = 0;
            }
            bsn[lane] = (int8_t)nch;
        }
        if (lane < 2 * P1) row[lane] = b[lane];
        if (lane + 64 < 2 * P1) row[lane + 64] = b[lane + 64];
        if (shift) {
            // the leaf level's L2L
            const int32_t par = J.parent[gid];
            const double pinv = 1.0 / J.scale[J.L - 1];
            if (lane < P1) {
                bpr[lane] = J.lc[(int64_t)par * 2 * P1 + 2 * lane];
                bpi[lane] = J.lc[(int64_t)par * 2 * P1 + 2 * lane + 1];
            }
            if (lane == 0) {
                const double wr = (cx - J.cx[par]) * pinv, wi = (cy - J.cy[par]) * pinv;
                double qr = 1.0, qi = 0.0;
                for (int k = 0; k <= J.p; ++k) {
                    wpr[k] = qr;
                    wpi[k] = qi;
                    const double nr = fma(qr, wr, -qi * wi), ni = fma(qr, wi, qi * wr);
                    qr = nr;
                    qi = ni;
                }
            }
            __syncthreads();
            if (lane < P1) {
                double sr = 0.0, si = 0.0;
                for (int k = lane; k <= J.p; ++k) {
                    const double c = J.binom[k * kBinomStride + lane];
                    const double ar = bpr[k], ai = bpi[k], xr = wpr[k - lane], xi = wpi[k - lane];
                    sr = fma(c, fma(ar, xr, -ai * xi), sr);
                    si = fma(c, fma(ar, xi, ai * xr), si);
                }
                const double rho = J.scale[J.L] * pinv;
                double rm = 1.0;
                for (int j = 0; j < lane; ++j) rm *= rho;
                row[2 * lane] = fma(sr, rm, row[2 * lane]);
                row[2 * lane + 1] = fma(si, rm, row[2 * lane + 1]);
            }
        }
        __syncthreads();
        if (!inb || t >= te) continue;
        double n0s = n0, n1s = n1;
        if (two)
            for (int k = 1; k < J.nw; ++k)
                for (int ch = 0; ch < bsn[k]; ++ch) {
                    const int64_t at = (int64_t)((k - 1) * kSymChunks + ch) * J.n_tgt + t;
                    if (J.bside64) {
                        const double2 v = J.bside64[at];
                        n0s += v.x;
                        n1s += v.y;
                    } else {
                        const float2 v = J.bside[at];
                        n0s += (double)v.x;
                        n1s += (double)v.y;
                    }
                }
        const double inv = 1.0 / J.scale[J.L];
        const double zr = (tx - cx) * inv, zi = (ty - cy) * inv;
        double fr = row[2 * J.p], fi = row[2 * J.p + 1], dr = 0.0, di = 0.0;
        // Explicit FMAs: the value's arithmetic is the same with and
        // without the derivative beside it.
        for (int m = J.p - 1; m >= 0; --m) {
            if (FIELD) {
                const double ndr = fma(dr, zr, fma(-di, zi, fr));
                const double ndi = fma(dr, zi, fma(di, zr, fi));
                dr = ndr;
                di = ndi;
            }
            const double nr = fma(fr, zr, fma(-fi, zi, row[2 * m]));
            const double ni = fma(fr, zi, fma(fi, zr, row[2 * m + 1]));
            fr = nr;
            fi = ni;
        }
        phi[2 * o] = n0s + fr;
        phi[2 * o + 1] = n1s + fi;
        if (FIELD) {
            bm.field_override[2 * o] = f0 + dr * inv;
            bm.field_override[2 * o + 1] = f1 + di * inv;
        }
    }
}

// Direct sum over a grid of (256-target block, source slice): each thread
// sums one target over its block's slice of the sources, staged through LDS
// 256 at a time in index order, and writes the slice's partial sum (with
// one slice, Phi itself).  Pairs are taken eight at a time: their terms are
// added plainly, then the group is Kahan-added to the running sums.  A
// source at the target's exact coordinates is skipped; the padding sources
// have zero strength and sit far away.
__global__ __launch_bounds__(256) void k_direct(const double *__restrict__ src, int64_t n_src,
                                                const double *__restrict__ tgt, int64_t n_tgt,
                                                const double *__restrict__ u, int64_t slice,
                                                double *__restrict__ out)
{
    __shared__ double sx[256], sy[256], su[256];
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool ok = j < n_tgt;
    const double y0 = ok ? tgt[2 * j] : 0.0, y1 = ok ? tgt[2 * j + 1] : 0.0;
    const int64_t s0 = blockIdx.y * slice;
    const int64_t s1 = min(n_src, s0 + slice);
    double re = 0.0, rc = 0.0, im = 0.0, ic = 0.0;
    for (int64_t base = s0; base < s1; base += 256) {
        __syncthreads();
        const int64_t i = base + threadIdx.x;
        const bool in = i < s1;
        sx[threadIdx.x] = in ? src[2 * i] : 1e100;
        sy[threadIdx.x] = in ? src[2 * i + 1] : 1e100;
        su[threadIdx.x] = in ? u[i] : 0.0;
        __syncthreads();
        const int ns = (int)min((int64_t)256, (s1 - base + 7) & ~(int64_t)7);
        for (int k = 0; k < ns; k += 8) {
            double pr = 0.0, pi = 0.0;
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                const double dx = y0 - sx[k + kk], dy = y1 - sy[k + kk];
                const double r2 = dx * dx + dy * dy;
                const bool live = r2 > 0.0;
                const double w = live ? su[k + kk] : 0.0;
                pr = fma(0.5 * w, ln_f64(live ? r2 : 1.0), pr);
                pi = fma(w, atan2_f64(dy, live ? dx : 1.0), pi);
            }
            const double yr = pr - rc, tr = re + yr;
            rc = (tr - re) - yr;
            re = tr;
            const double yi = pi - ic, ti = im + yi;
            ic = (ti - im) - yi;
            im = ti;
        }
    }
    if (ok) {
        double *o = out + 2 * (blockIdx.y * n_tgt + j);
        o[0] = re - rc;
        o[1] = im - ic;
    }
}

// Phi[j] = the slices' partial sums for target j, added in slice order
// (Neumaier).
__global__ __launch_bounds__(256) void k_direct_reduce(const double *__restrict__ part, int64_t n_tgt,
                                                       int slices, double *__restrict__ phi)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n_tgt) return;
    double s[2] = {0.0, 0.0}, c[2] = {0.0, 0.0};
    for (int q = 0; q < slices; ++q)
        for (int h = 0; h < 2; ++h) {
            const double v = part[2 * (q * n_tgt + j) + h];
            const double t = s[h] + v;
            c[h] += fabs(s[h]) >= fabs(v) ? (s[h] - t) + v : (v - t) + s[h];
            s[h] = t;
        }
    phi[2 * j] = s[0] + c[0];
    phi[2 * j + 1] = s[1] + c[1];
}

int direct_slices(int64_t n_src, int64_t n_tgt)
{
    // Enough (block, slice) pairs for about eight waves per SIMD, slices of
    // at least 32 sources, at most 1024 slices.
    const int64_t lanes = ((n_tgt + 255) / 256) * 256;
    int64_t want = (256 * 4 * 8 * 64 + lanes - 1) / lanes;
    const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(1024, (n_src + 31) / 32));
    return (int)std::max<int64_t>(1, std::min(want, cap));
}

void launch_direct(const double *src, int64_t n_src, const double *tgt, int64_t n_tgt, const double *u,
                   double *phi, double *part, int slices, hipStream_t s)
{
    if (n_tgt <= 0) return;
    const int64_t slice = slices > 1 ? (n_src + slices - 1) / slices : std::max<int64_t>(n_src, 1);
    const unsigned tb = (unsigned)((n_tgt + 255) / 256);
    hipLaunchKernelGGL(k_direct, dim3(tb, (unsigned)slices), dim3(256), 0, s, src, n_src, tgt, n_tgt, u, slice,
                       slices > 1 ? part : phi);
    if (slices > 1)
        hipLaunchKernelGGL(k_direct_reduce, dim3(tb), dim3(256), 0, s, part, n_tgt, slices, phi);
}

// ------------------------------------------------------------ symmetric form
// ln r2 with the arguments of the pair, (x, y), and of the reverse pair,
// (-x, -y), both on the principal branch with a zero y read as +0: the
// octant's last step is taken once for x and once for -x from the same
// angle in [0, pi/2].
__device__ __forceinline__ void ln_atan2_pair_f64(double r2, double y, double x, double &lnr2, double &at,
                                                  double &atr)
{
    double a;
    ln_angle_f64(r2, fabs(x), fabs(y), lnr2, a);
    const double pa = kPiHi + (kPiLo - a);
    const double af = (x < 0.0) ? pa : a, ab = (x > 0.0) ? pa : a;
    at = (y < 0.0) ? -af : af;
    atr = (y > 0.0) ? -ab : ab;
}

// The value v of the lane whose byte address (4 x lane) is addr, by two
// 32-bit permutes.
__device__ __forceinline__ double bperm_f64(int addr, double v)
{
    const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// The FP64 near field for a plan whose targets are its sources: a neighbour
// pair {A, B} (A the lower cell id, with at most kSymChunks chunks) is
// evaluated once, by A's items, for both sides; the leaf itself, and pairs
// whose lower leaf is larger, one-sided.  A lane tile of R target rows by
// 64 / R source columns: A's targets (all of a leaf of up to kWide = 96,
// else a chunk of 64) in LDS in blocks of R rows, 64 / R sources per round in
// the columns (absolute coordinates, loaded a round ahead), so every
// separation, and with it the sign of dy, is exact; R = 8, or R = 4 for
// items of at most kSmall = 48 targets, whose last block then pads at most
// three rows and whose per-round work is spread over twice the sources.  The
// item runs two loops: the leaf's own sources (one side, zero separations
// skipped), then the sources of its other neighbour cells as one
// concatenated sequence, so a round's columns may come from two cells and
// only the sequence's last round is padded.
// Each column keeps a cursor (cell, position) into the sequence.  Sums are
// FP64 throughout: A's in the lanes, reduced over the columns at the end;
// each round's second-side sums reduced over the rows and stored per
// (point, lower neighbour, its chunk) in bside64 for L2P (columns of a cell
// taken one-sided store nothing).
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_near_fp64_sym(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    // The item's other neighbour cells in sequence order, per cell {end in
    // the sequence, first source minus start, second-side offset in bside64
    // minus start, whether it has one (else this item takes the cell
    // one-sided)}.
    __shared__ int4 cinfo[kNearSlots];
    __shared__ double2 sxy[kWide];   // A's targets: coordinates
    __shared__ double sau[kWide];    // and strengths
    // A's sums of the target blocks past the first kRegBlocks, per lane, in
    // LDS (each read and written once per round by its own lane): with few
    // sums in registers the kernel needs 146 VGPRs without spills, three
    // waves per SIMD, and leaves register room for other kernels' waves.
    constexpr int kRegBlocks = 2;
    __shared__ double2 sacc[kWide / 8 - kRegBlocks][64];
    const int lane = threadIdx.x;
    static_assert(kNearSlots <= 16, "neighbour lists scanned within 16 lanes");
    for (int64_t item = blockIdx.x; item < bm.pre[bm.n]; item += gridDim.x) {
        // (the entry and its job are the same in every lane: scalar)
        const int e = uniform(batch_entry(bm, item));
        const EvalJob &J = jobs[uniform(bm.job[e])];
        const int64_t it = item - bm.pre[e];
        if (it >= J.counts[0]) continue;
        const int32_t li = uniform(J.work_near[2 * it]), st = uniform(J.work_near[2 * it + 1]);
        const int64_t gid = J.leaf_off + li;
        const int nw = uniform(J.nw);
        const int32_t tb = uniform(J.tb[gid]), te = uniform(J.te[gid]);
        // A leaf of at most kWide targets is one item (its first); larger
        // leaves go in chunks of kChunk.
        const bool wide = te - tb <= kWide;
        if (wide && st != tb) continue;
        const int m = wide ? te - tb : min(kChunk, te - st);
        const int nblk = (m + 7) >> 3;
        const int chunk = wide ? 0 : (st - tb) / kChunk;
        const bool own_sym = sym_chunks(te - tb, kWide) <= kSymChunks;

        __syncthreads();   // the previous item is done with the LDS
        for (int q = lane; q < kWide; q += 64) {
            // Padding targets: zero strength, far from every source and from
            // the padding source, so no separation in the tile is zero (the
            // neighbour rounds have no zero-separation guard, and a zero
            // there would turn a padding row's 0 x log 0 into a NaN in the
            // second-side sums).
            const bool ok = q < m;
            sxy[q] = make_double2(ok ? J.tx[st + q] : -1e100, ok ? J.ty[st + q] : -1e100);
            sau[q] = ok ? J.su[st + q] : 0.0;
        }
        // Lane k (1 <= k < nw) classifies neighbour slot k: its sources
        // (none if the other leaf's items take the pair for both sides) and,
        // if this item takes both sides, this leaf's slot in the other
        // leaf's list, which names the second-side row.
        int32_t b0 = 0, cnt = 0, slot = -1;
        if (lane > 0 && lane < nw) {
            const int32_t c = J.near[li * nw + lane];
            if (c >= 0) {
                b0 = J.sb[c];
                cnt = J.se[c] - b0;
                if (c > gid && own_sym) {
                    const int32_t *lc = J.near + (c - J.leaf_off) * nw;
                    int k2 = nw;
#pragma unroll
                    for (int k = kNearSlots - 1; k >= 1; --k)   // independent loads
                        if (k < nw && lc[k] == (int32_t)gid) k2 = k;
                    if (k2 < nw) slot = (k2 - 1) * kSymChunks + chunk;
                } else if (c < gid && sym_chunks(cnt, kWide) <= kSymChunks) {
                    cnt = 0;
                }
            }
        }
        int32_t incl = cnt;   // inclusive prefix over lanes 0..15
#pragma unroll
        for (int d = 1; d < 16; d <<= 1) {
            const int32_t v = __shfl_up(incl, d, 16);
            if ((lane & 15) >= d) incl += v;
        }
        const uint64_t taken = __ballot(cnt > 0);
        const int nc = __popcll(taken);
        const int32_t total = uniform(__shfl(incl, 15));
        if (cnt > 0) {
            // second-side offsets fit 32 bits: the plan keeps
            // (near width - 1) kSymChunks n_tgt below 2^31
            const int32_t start = incl - cnt, base = b0 - start;
            const int32_t row = slot >= 0 ? (int32_t)((int64_t)slot * J.n_tgt) + base : 0;
            cinfo[__popcll(taken & ((1ull << lane) - 1))] = make_int4(incl, base, row, slot >= 0);
        }
        const int32_t c0 = uniform(J.near[li * nw]);   // slot 0: the leaf itself
        const int32_t sb0 = c0 >= 0 ? uniform(J.sb[c0]) : 0, se0 = c0 >= 0 ? uniform(J.se[c0]) : 0;
        __syncthreads();

        struct Src {
            double x, y, w;
        };
        auto load = [&](int32_t i) {
            Src r;
            r.x = gload(J.sx, i);
            r.y = gload(J.sy, i);
            r.w = gload((const double *)J.su, i);
            return r;
        };
        // The item's rounds for NB target blocks of R rows (dispatched once
        // per item, so the accumulators stay in place from round to round):
        // lane = row x TC + column, TC = 64 / R sources per round.
        auto item_rounds = [&](auto r_const, auto nb_const) {
            constexpr int R = decltype(r_const)::value, NB = decltype(nb_const)::value;
            constexpr int TC = 64 / R;
            constexpr int NR = NB < kRegBlocks ? NB : kRegBlocks;   // blocks summed in registers
            static_assert(NB - NR <= kWide / 8 - kRegBlocks && R * NB <= kWide, "LDS sums and targets");
            const int row = lane / TC, col = lane % TC;
            double ar[NR], ai[NR];
#pragma unroll
            for (int blk = 0; blk < NR; ++blk) ar[blk] = ai[blk] = 0.0;
#pragma unroll
            for (int blk = NR; blk < NB; ++blk) sacc[blk - NR][lane] = make_double2(0.0, 0.0);
            // A's sum of block blk (a constant after unrolling) += w (lg, at)
            auto add_a = [&](int blk, double w, double lg, double at) {
                if (blk < NR) {
                    const int b = blk < NR ? blk : 0;
                    ar[b] = fma(w, lg, ar[b]);
                    ai[b] = fma(w, at, ai[b]);
                } else {
                    double2 &v = sacc[blk < NR ? 0 : blk - NR][lane];
                    const double2 o = v;
                    v = make_double2(fma(w, lg, o.x), fma(w, at, o.y));
                }
            };
            // The leaf's own sources, one side; a zero separation (the point
            // itself, or an equal point) is skipped.  Padding columns read
            // source 0 with zero strength.
            {
                int32_t b = sb0;
                bool ok = b + col < se0;
                Src nxt = load(ok ? b + col : 0);
                while (b < se0) {
                    const double sx = nxt.x, sy = nxt.y, su = ok ? nxt.w : 0.0;
                    b += TC;
                    ok = b + col < se0;
                    nxt = load(ok ? b + col : 0);
                    // The targets are read from LDS every round (an opaque
                    // copy of the row index keeps the reads in the loop):
                    // holding twelve blocks' coordinates and strengths in
                    // registers would spill.
                    int qrow = row;
                    asm volatile("" : "+v"(qrow));
#pragma unroll
                    for (int blk = 0; blk < NB; ++blk) {
                        const int q = R * blk + qrow;
                        const double2 t = sxy[q];
                        const double dx = t.x - sx, dy = t.y - sy;
                        const double r2 = fma(dx, dx, dy * dy);
                        const bool live = r2 > 0.0;
                        double lg, at;
                        ln_atan2_f64(live ? r2 : 1.0, dy, live ? dx : 1.0, lg, at);
                        add_a(blk, live ? su : 0.0, lg, at);
                    }
                }
            }
            // The other neighbours' sources, both sides where the cell has a
            // second-side slot.  Each column keeps the sequence cell j of its
            // source; the cell's record gives the source index and the
            // second-side offset of a sequence position.
            if (total > 0) {
                int j = 0;
                auto locate = [&](int32_t p) {
                    while (p >= cinfo[j].x && j + 1 < nc) ++j;
                    return cinfo[j];
                };
                int32_t p = col;
                int4 c = locate(p);
                bool ok = p < total;
                int32_t dst = ok && c.w ? c.z + p : -1;   // the column's second-side sum
                Src nxt = load(ok ? c.y + p : 0);
                for (int32_t P = 0; P < total; P += TC) {
                    // padding: zero strength, far away
                    const double sx = ok ? nxt.x : 1e100, sy = ok ? nxt.y : 1e100;
                    const double su = ok ? nxt.w : 0.0;
                    const int32_t out = dst;
                    p = P + TC + col;
                    c = locate(p);
                    ok = p < total;
                    dst = ok && c.w ? c.z + p : -1;
                    nxt = load(ok ? c.y + p : 0);
                    int qrow = row;
                    asm volatile("" : "+v"(qrow));
                    double br = 0.0, bi = 0.0;
#pragma unroll
                    for (int blk = 0; blk < NB; ++blk) {
                        const int q = R * blk + qrow;
                        const double2 t = sxy[q];
                        const double dx = t.x - sx, dy = t.y - sy, u = sau[q];
                        double lg, at, atr;
                        ln_atan2_pair_f64(fma(dx, dx, dy * dy), dy, dx, lg, at, atr);
                        add_a(blk, su, lg, at);
                        br = fma(u, lg, br);
                        bi = fma(u, atr, bi);
                    }
                    // B's sums over the rows (lane ^ TC, ^ 2 TC, ..., ^ 32)
#pragma unroll
                    for (int k = TC; k < 64; k <<= 1) {
                        const int a = (lane ^ k) << 2;
                        br += bperm_f64(a, br);
                        bi += bperm_f64(a, bi);
                    }
                    if (row == 0 && out >= 0) J.bside64[(uint32_t)out] = make_double2(0.5 * br, bi);
                }
            }
            // A's sums over the columns; column 0 writes
#pragma unroll
            for (int blk = 0; blk < NB; ++blk) {
                double vr, vi;
                if (blk < NR) {
                    vr = ar[blk < NR ? blk : 0];
                    vi = ai[blk < NR ? blk : 0];
                } else {
                    const double2 v = sacc[blk < NR ? 0 : blk - NR][lane];
                    vr = v.x;
                    vi = v.y;
                }
#pragma unroll
                for (int k = 1; k < TC; k <<= 1) {
                    const int a = (lane ^ k) << 2;
                    vr += bperm_f64(a, vr);
                    vi += bperm_f64(a, vi);
                }
                const int q = R * blk + row;
                if (col == 0 && q < m) {
                    J.nsum[2 * (st + q)] = 0.5 * vr;
                    J.nsum[2 * (st + q) + 1] = vi;
                }
            }
        };
        // Items of at most kSmall targets take blocks of four rows and sixteen
        // sources per round (less padding and per-round work for small
        // leaves), larger ones blocks of eight rows and eight sources.
        static_assert(kWide == 96 && kSmall == 48, "one case per number of target blocks");
        using I4 = std::integral_constant<int, 4>;
        using I8 = std::integral_constant<int, 8>;
        if (m <= kSmall) {
            // (an item of up to four targets takes two blocks: the one-block
            // loop alone would raise the kernel from 154 to 168 VGPRs, which
            // leaves no registers for other kernels' waves beside its three
            // per SIMD)
            switch (m <= 4 ? 2 : (m + 3) >> 2) {
            case 2: item_rounds(I4{}, std::integral_constant<int, 2>{}); break;
            case 3: item_rounds(I4{}, std::integral_constant<int, 3>{}); break;
            case 4: item_rounds(I4{}, std::integral_constant<int, 4>{}); break;
            case 5: item_rounds(I4{}, std::integral_constant<int, 5>{}); break;
            case 6: item_rounds(I4{}, std::integral_constant<int, 6>{}); break;
            case 7: item_rounds(I4{}, std::integral_constant<int, 7>{}); break;
            case 8: item_rounds(I4{}, std::integral_constant<int, 8>{}); break;
            case 9: item_rounds(I4{}, std::integral_constant<int, 9>{}); break;
            case 10: item_rounds(I4{}, std::integral_constant<int, 10>{}); break;
            case 11: item_rounds(I4{}, std::integral_constant<int, 11>{}); break;
            default: item_rounds(I4{}, std::integral_constant<int, 12>{}); break;
            }
        } else {
            switch (nblk) {
            case 7: item_rounds(I8{}, std::integral_constant<int, 7>{}); break;
            case 8: item_rounds(I8{}, std::integral_constant<int, 8>{}); break;
            case 9: item_rounds(I8{}, std::integral_constant<int, 9>{}); break;
            case 10: item_rounds(I8{}, std::integral_constant<int, 10>{}); break;
            case 11: item_rounds(I8{}, std::integral_constant<int, 11>{}); break;
            default: item_rounds(I8{}, std::integral_constant<int, 12>{}); break;
            }
        }
    }
}

// Issue-rate probe of the FP64 pair evaluation: every lane evaluates
// ln_atan2_pair_f64 for `rounds` rounds of eight independent pairs whose
// separations it steps in registers (no loads, no LDS, no second-side
// reductions), summing the three results, which it stores so that no
// evaluation is dropped.  One-wave blocks at three waves per SIMD, as the
// near field runs: the rate it reaches is the pair-evaluation ceiling of
// this code on the chip as it clocks under the load.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_pair_rate(int rounds, double *out)
{
    const int lane = threadIdx.x;
    double dx[8], dy[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        dx[j] = 0.37 + 0.011 * lane - 0.29 * j;
        dy[j] = -0.21 + 0.005 * (blockIdx.x & 63) + 0.17 * j;
    }
    double sl = 0.0, sa = 0.0, sr = 0.0;
    for (int r = 0; r < rounds; ++r) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            double lg, at, atr;
            ln_atan2_pair_f64(fma(dx[j], dx[j], dy[j] * dy[j]), dy[j], dx[j], lg, at, atr);
            sl += lg;
            sa += at;
            sr += atr;
            dx[j] += 1e-3;
        }
    }
    out[blockIdx.x * 64 + lane] = sl + sa + sr;
}

int probe_pair_rate(int rounds, int blocks, double *evals_per_s)
{
    double *out = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    int err = hipMalloc(&out, sizeof(double) * 64 * (size_t)blocks) != hipSuccess;
    err = err || hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess;
    err = err || hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess;
    if (!err) {
        hipLaunchKernelGGL(k_pair_rate, dim3(blocks), dim3(64), 0, s, 1, out);   // warm-up
        hipEventRecord(a, s);
        hipLaunchKernelGGL(k_pair_rate, dim3(blocks), dim3(64), 0, s, rounds, out);
        hipEventRecord(b, s);
        float ms = 0.0f;
        err = hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess || ms <= 0.0f;
        if (!err) *evals_per_s = 64.0 * blocks * 8.0 * rounds / (ms * 1e-3);
    }
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
    if (s) hipStreamDestroy(s);
    if (out) hipFree(out);
    return err;
}

void batch_near_fp64_sym(const EvalJob *jobs, const BatchMap &m, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    const dim3 grid(persistent_grid(m.pre[m.n], kNearWavesPerCU));
    hipLaunchKernelGGL(k_near_fp64_sym, grid, dim3(64), 0, s, jobs, m);
}

void batch_near_fp64(const EvalJob *jobs, const BatchMap &m, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    const dim3 grid(persistent_grid(m.pre[m.n], kNearWavesPerCU));
    if (m.nfield) hipLaunchKernelGGL(k_near_fp64<true>, grid, dim3(64), 0, s, jobs, m);
    else hipLaunchKernelGGL(k_near_fp64<false>, grid, dim3(64), 0, s, jobs, m);
}

void batch_l2p(const EvalJob *jobs, const BatchMap &m, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    if (m.field_override)
        hipLaunchKernelGGL(k_l2p<true>, dim3(persistent_grid(m.pre[m.n], 64)), dim3(64), 0, s, jobs, m);
    else
        hipLaunchKernelGGL(k_l2p<false>, dim3(persistent_grid(m.pre[m.n], 64)), dim3(64), 0, s, jobs, m);
}

}  // namespace fmm
