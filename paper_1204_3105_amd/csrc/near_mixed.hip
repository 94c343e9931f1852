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
#include <type_traits>

#include "eval.h"

namespace fmm {

// atan(t) = t * sum_k c_k t^(2k) for 0 <= t <= 1: weighted least-squares
// fit on Chebyshev nodes (gen_atan_poly.py); max abs error 1.8e-7 in FP32.
static constexpr float kAtanPoly[8] = {9.999999114e-01f, -3.333209348e-01f, 1.997137453e-01f,
                                       -1.402941598e-01f, 9.942748199e-02f, -5.990455402e-02f,
                                       2.455700589e-02f, -4.780421207e-03f};
// The same fit with seven terms (gen_atan_poly.py 6): max abs error 6.6e-7 in
// FP32, for the symmetric kernel, where it saves an FMA per pair.
static constexpr float kAtanPoly7[7] = {9.999994166e-01f, -3.332701317e-01f, 1.988731901e-01f,
                                        -1.351216669e-01f, 8.435391630e-02f, -3.744282786e-02f,
                                        8.006850172e-03f};
static constexpr float kPi = 3.14159265358979324f, kPi2 = 1.57079632679489662f;

// |atan2(y, x)| in [0, pi]: t = min/max of |x|, |y| (the max floored so
// that t stays finite), then the octant within the upper half plane.
template <int NC = 8>
__device__ __forceinline__ float atan2_abs(float y, float x, float &mn)
{
    const float *c = NC == 8 ? kAtanPoly : kAtanPoly7;
    const float ax = fabsf(x), ay = fabsf(y);
    mn = fminf(ax, ay);
    const float mx = fmaxf(fmaxf(ax, ay), 1e-30f);
    const float t = mn * __builtin_amdgcn_rcpf(mx);
    const float z = t * t;
    float p = c[NC - 1];
#pragma unroll
    for (int k = NC - 2; k >= 0; --k) p = fmaf(p, z, c[k]);
    float a = t * p;
    a = (ay > ax) ? kPi2 - a : a;
    return (x < 0.0f) ? kPi - a : a;
}

// The FP32 offsets carry a separation with an absolute error of at most
// about 9 * 2^-24 of the leaf scale h (two offsets within a leaf, the
// leaf-to-leaf offset and one rounded sum).  Two kinds of pair are hurt by it
// and are evaluated again from the FP64 coordinates:
//  - near the negative real axis a tiny dy can get the wrong sign or become
//    zero, which moves the pair across the logarithm's principal branch cut
//    (its argument jumps by 2 pi): pairs with |dy| below 2^-19 h (about one
//    pair in 10^6 for spread-out points);
//  - a pair at separation d carries about 2^-24 h / d in ln|r| and in its
//    argument, which points on a curve or planted next to each other (d far
//    below h) turn into errors above eps: pairs with r^2 below (h 2^-5)^2, so
//    that every pair kept in FP32 has h / d < 32.
// For those pairs the separation is formed in FP64 from the absolute
// coordinates and rounded to FP32 (relative error 2^-24, whatever d), the
// sign of dy taken from the FP64 difference (+0 when the coordinates are
// equal: the principal branch's arg = pi), and the log and argument terms
// are corrected by the difference to what the hot loop summed.  The hot
// loops only keep each lane's smallest |dy| (or min(|dx|, |dy|), a cheap bound
// for it) and smallest r^2; a round in which some lane saw a value below its
// bound is gone over again for those pairs.  A pair of points with equal FP64
// coordinates contributes nothing, whatever its FP32 offsets.
constexpr float kCloseTau = 0x1p-5f;   // close-pair radius in units of the leaf scale

__device__ __forceinline__ float close_tau2(const EvalJob &J)
{
    const float t = (float)J.scale[J.L] * kCloseTau;
    return t * t;
}

// The pair (target t, source i) from the FP64 coordinates: the separation
// rounded to FP32, the sign of dy (+1, -1, or +0 for equal y) and whether the
// two points differ at all (the FP64 difference of finite values is zero only
// for equal values).
struct Pair64 {
    float ex, ey, sg;
    bool live;
};

__device__ __forceinline__ Pair64 pair_fp64(const EvalJob &J, int32_t t, int32_t i)
{
    const double ddx = J.tx[t] - J.sx[i], ddy = J.ty[t] - J.sy[i];
    Pair64 r;
    r.ex = (float)ddx;
    r.ey = (float)ddy;
    r.sg = ddy > 0.0 ? 1.0f : (ddy < 0.0 ? -1.0f : 0.0f);
    r.live = ddx != 0.0 || ddy != 0.0;
    return r;
}

// atan2 on the principal branch (-pi, pi]; y = -0 is treated as +0 and
// (0, 0) gives 0.
template <int NC = 8>
__device__ __forceinline__ float atan2_abs(float y, float x)
{
    float mn;
    return atan2_abs<NC>(y, x, mn);
}

__device__ __forceinline__ float atan2_f32(float y, float x, float &mn)
{
    const float a = atan2_abs(y, x, mn);
    return (y < 0.0f) ? -a : a;
}

__device__ __forceinline__ float atan2_f32(float y, float x)
{
    float mn;
    return atan2_f32(y, x, mn);
}

// Running minimum of non-negative floats kept as their bit patterns (which
// order as unsigned integers): one integer min, no NaN handling.
__device__ __forceinline__ void keep_min(uint32_t &w, float v) { w = min(w, __float_as_uint(v)); }

// arg with the sign of s taken for the sign of dy (s = -0 as +0); a = |arg|.
__device__ __forceinline__ float signed_arg(float a, float s) { return s < 0.0f ? -a : a; }
// arg of the reverse pair, -(dx, dy): pi - a for s <= 0, a - pi for s > 0.
__device__ __forceinline__ float reverse_arg(float a, float s)
{
    const float pm = kPi - a;
    return s <= 0.0f ? pm : -pm;
}

// The symmetric kernel's hot-loop forms, one bit-field insert each: the sign
// of dy copied onto |arg| and onto pi - |arg| (the reverse argument is minus
// the latter).  They differ from the two above only for dy = +-0, which the
// branch-cut pass always revisits (|dy| is then below its bound) and
// corrects against these same forms.
__device__ __forceinline__ float fast_arg(float a, float dy) { return copysignf(a, dy); }
__device__ __forceinline__ float fast_rev_neg(float a, float dy) { return copysignf(kPi - a, dy); }

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
        const float dtol = (float)(J.scale[J.L] * 0x1p-19), tau2 = close_tau2(J);

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
            float worst = 1e30f, wclose = 1e30f;   // smallest |dy| and r^2 of the round
            if (self_round) {
                for (int j = 0; j < padn; ++j) {
                    const float4 sv = gsh[j];
                    const float dx = ax - sv.x, dy = ay - sv.y;
                    const float r2 = fmaf(dx, dx, dy * dy);
                    const bool live = r2 > 0.0f;
                    const float lg = __log2f(live ? r2 : 1.0f);
                    const float at = atan2_f32(dy, dx);
                    worst = fminf(worst, fabsf(dy));
                    wclose = fminf(wclose, r2);
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
                        worst = fminf(worst, fabsf(dy));
                        wclose = fminf(wclose, r2);
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
            const bool flagged = worst < dtol || wclose < tau2;
            if (__any(flagged)) {
                // pairs near the branch cut or close together: again from
                // the FP64 coordinates, corrected by the difference to the
                // terms the loop above summed
                if (flagged && busy) {
                    for (int j = 0; j < n; ++j) {
                        const float4 sv = gsh[j];
                        const float dx = ax - sv.x, dy = ay - sv.y;
                        const float r2 = self_round ? fmaf(dx, dx, dy * dy) : fmaf(dx, dx, fmaf(dy, dy, 1e-37f));
                        if (!(fabsf(dy) < dtol || r2 < tau2)) continue;
                        const bool live0 = !self_round || r2 > 0.0f;
                        const float lg0 = live0 ? __log2f(r2) : 0.0f;
                        const float at0 = live0 ? atan2_f32(dy, dx) : 0.0f;
                        const Pair64 q = pair_fp64(J, t, base + j);
                        const float lg1 = q.live ? __log2f(fmaf(q.ex, q.ex, fmaf(q.ey, q.ey, 1e-37f))) : 0.0f;
                        const float at1 = q.live ? signed_arg(atan2_abs(q.ey, q.ex), q.sg) : 0.0f;
                        acc(sv.z * (lg1 - lg0), sv.w * (at1 - at0));
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

// ------------------------------------------------------------ symmetric form
// For a plan whose targets are its sources.  The pair of distinct
// neighbouring leaves {A, B}, A the lower cell id, is evaluated once, by A's
// items, when A has at most kSymChunks chunks: one log2 r^2 and one argument
// serve both directions, since on the principal branch
//     arg(x_b - y_a) = arg(y_a - x_b) - pi  (arg > 0),  + pi  (arg <= 0),
// i.e. pi - |arg| for dy <= 0 and |arg| - pi for dy > 0 (dy = -0 taken as
// +0).  A's sums stay in registers; B's are reduced over
// the wave and stored, one FP32 (re, im) per (B point, A chunk), in the plan's
// second-side array, which L2P adds in a fixed order.  The leaf itself, and
// a neighbour pair whose lower leaf has more chunks, are evaluated for one
// side (by both leaves' items).
//
// Lane layout: an 8 x 8 tile, row i = lane / 8, column j = lane % 8.  The
// item's targets (up to 64) sit in registers in eight blocks of eight
// (target 8 blk + i in row i, the same in every column); each round the
// columns take the next eight sources of one cell (source j in column j,
// padded with zero-strength sources far away), and each lane evaluates its
// (target, source) pair for every target block.  The next round's sources
// are loaded during the current one.  A lane adds its terms plainly in
// FP32 (one per round and target block); every kFlush rounds A's partial
// sums are reduced over the columns and added to FP64 sums in LDS, so a
// plain FP32 sum never spans more than kFlush terms, whatever the leaf
// sizes.  B's sums (at most 64 terms) are reduced over the rows in FP32.


constexpr int kFlush = 16;

// v + (v of the lane given by a DPP pattern): quad_perm [1,0,3,2] (lane ^ 1),
// quad_perm [2,3,0,1] (lane ^ 2), row_half_mirror (lane 7 - lane within 8).
template <int CTRL>
__device__ __forceinline__ float add_dpp(float v)
{
    return v + __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_near_mixed_sym(const EvalJob *__restrict__ jobs, BatchMap bm)
{
    __shared__ int32_t cbeg[kNearSlots], cend[kNearSlots], cslot[kNearSlots];
    __shared__ float cdx[kNearSlots], cdy[kNearSlots];
    __shared__ int8_t cmode[kNearSlots];
    __shared__ double sre[64], sim[64];   // A's sums, target 8 blk + row
    __shared__ float4 sA[64];             // A's targets: offset x, y, strength
    const int lane = threadIdx.x, row = lane >> 3, col = lane & 7;
    const int perm16 = (lane ^ 16) << 2, perm32 = (lane ^ 32) << 2;   // ds_bpermute byte addresses
    const float half_ln2 = 0.34657359027997264f;
    for (int64_t item = blockIdx.x; item < bm.pre[bm.n]; item += gridDim.x) {
        const int e = uniform(batch_entry(bm, item));
        const EvalJob &J = jobs[uniform(bm.job[e])];
        const int64_t it = item - bm.pre[e];
        if (it >= J.counts[0]) continue;
        // (item values are the same in every lane: kept in scalar registers
        // so that the loops below branch on the scalar unit)
        const int32_t li = uniform(J.work_near[2 * it]), st = uniform(J.work_near[2 * it + 1]);
        const int64_t gid = J.leaf_off + li;
        const int nw = uniform(J.nw);
        const int32_t tb = uniform(J.tb[gid]), te = uniform(J.te[gid]);
        const int m = min(kChunk, te - st);
        const int nblk = (m + 7) >> 3;
        const int chunk = (st - tb) / kChunk;
        const bool own_sym = (te - tb + kChunk - 1) / kChunk <= kSymChunks;
        const float dtol = (float)(J.scale[J.L] * 0x1p-19), tau2 = close_tau2(J);

        // Cell table: range, offset from this leaf's centre, and how the
        // cell's pairs are taken.  Slot 0 is the leaf itself.
        __syncthreads();   // the previous item is done with the LDS
        sre[lane] = sim[lane] = 0.0;
        {
            const bool ok = lane < m;
            sA[lane] = make_float4(ok ? J.txl[st + lane] : 0.0f, ok ? J.tyl[st + lane] : 0.0f,
                                   ok ? J.suf[st + lane] : 0.0f, 0.0f);
        }
        if (lane < nw) {
            const int32_t c = J.near[li * nw + lane];
            int32_t b0 = 0, e0 = 0, slot = 0;
            int8_t mode = kCellSkip;
            float dx = 0.0f, dy = 0.0f;
            if (c >= 0) {
                b0 = J.sb[c];
                e0 = J.se[c];
                dx = (float)(J.cx[c] - J.cx[gid]);
                dy = (float)(J.cy[c] - J.cy[gid]);
                mode = kCellOne;
                if (lane > 0 && c > gid && own_sym) {
                    // this leaf's slot in the neighbour's list (the
                    // neighbour relation is symmetric; one-sided otherwise)
                    const int64_t lb = c - J.leaf_off;
                    int k2 = 1;
                    while (k2 < nw && J.near[lb * nw + k2] != (int32_t)gid) ++k2;
                    if (k2 < nw) {
                        mode = kCellSym;
                        slot = (k2 - 1) * kSymChunks + chunk;
                    }
                } else if (lane > 0 && c < gid && (e0 - b0 + kChunk - 1) / kChunk <= kSymChunks) {
                    // the neighbour's items evaluate the pair (if this leaf
                    // is in its list, which the symmetric relation ensures)
                    mode = kCellSkip;
                }
            }
            if (mode == kCellSkip) e0 = b0;
            cbeg[lane] = b0;
            cend[lane] = e0;
            cslot[lane] = slot;
            cdx[lane] = dx;
            cdy[lane] = dy;
            cmode[lane] = mode;
        }
        __syncthreads();

        // This lane's source of round (k, b): its loads are issued a round
        // ahead (from a valid index), and the values are formed -- coordinates
        // relative to this leaf's centre, or the padding source where out of
        // range -- only when the round starts.
        struct Src {
            float lx, ly, lw, ox, oy;
            bool ok;
        };
        auto fetch = [&](int k, int32_t b) {
            Src r;
            const int kk = k < nw ? k : 0;
            const int32_t i = b + col;
            r.ok = k < nw && i < cend[kk];
            const int32_t ic = r.ok ? i : 0;
            r.lx = gload(J.sxl, ic);
            r.ly = gload(J.syl, ic);
            r.lw = gload((const float *)J.suf, ic);
            r.ox = cdx[kk];
            r.oy = cdy[kk];
            return r;
        };
        auto next_cell = [&](int k) {
            while (k < nw && uniform(cbeg[k]) >= uniform(cend[k])) ++k;
            return k;
        };
        // The item's rounds for NB target blocks (dispatched once per item,
        // so the accumulators stay in place from round to round).
        auto item_rounds = [&](auto nb_const) {
            constexpr int NB = decltype(nb_const)::value;
            float ar[NB], ai[NB];
#pragma unroll
            for (int blk = 0; blk < NB; ++blk) ar[blk] = ai[blk] = 0.0f;
            // A's partial sums of each target block: over the columns
            // (DPP), then column 0 adds them to the FP64 sums.
            auto flush = [&]() {
#pragma unroll
                for (int blk = 0; blk < NB; ++blk) {
                    float vr = ar[blk], vi = ai[blk];
                    vr = add_dpp<0xB1>(vr);
                    vi = add_dpp<0xB1>(vi);
                    vr = add_dpp<0x4E>(vr);
                    vi = add_dpp<0x4E>(vi);
                    vr = add_dpp<0x141>(vr);
                    vi = add_dpp<0x141>(vi);
                    if (col == 0) {
                        sre[8 * blk + row] += (double)vr;
                        sim[8 * blk + row] += (double)vi;
                    }
                    ar[blk] = ai[blk] = 0.0f;
                }
            };
            int k = next_cell(0);
            int32_t b = k < nw ? uniform(cbeg[k]) : 0;
            Src nxt = fetch(k, b);
            int rounds = 0;
            while (k < nw) {
                const int32_t ce = uniform(cend[k]);
                int k2 = k;
                int32_t b2 = b + 8;
                if (b2 >= ce) {
                    k2 = next_cell(k + 1);
                    b2 = k2 < nw ? uniform(cbeg[k2]) : 0;
                }
                const float sx = nxt.ok ? nxt.lx + nxt.ox : 1e18f;
                const float sy = nxt.ok ? nxt.ly + nxt.oy : 1e18f;
                const float su = nxt.ok ? nxt.lw : 0.0f;
                nxt = fetch(k2, b2);
                // smallest min(|dx|, |dy|) (a cheap bound for the smallest
                // |dy|) and smallest r^2 of the round, as bits
                uint32_t worst = 0x7f800000u, wclose = 0x7f800000u;
                auto flagged = [&]() {
                    return __uint_as_float(worst) < dtol || __uint_as_float(wclose) < tau2;
                };
                // pairs near the branch cut or close together: again from the
                // FP64 coordinates, corrected by the difference to the terms
                // the round summed (the B-side terms only for a symmetric cell)
                auto fix_pairs = [&](bool two, float &br, float &bi) {
                    if (!flagged()) return;
                    const int32_t i = b + col;
#pragma unroll
                    for (int blk = 0; blk < NB; ++blk) {
                        const int q = 8 * blk + row;
                        if (q < m && i < ce) {
                            const float4 A = sA[q];
                            const float dx = A.x - sx, dy = A.y - sy;
                            const float r2 = two ? fmaf(dx, dx, fmaf(dy, dy, 1e-37f)) : fmaf(dx, dx, dy * dy);
                            if (fabsf(dy) < dtol || r2 < tau2) {
                                const bool live0 = two || r2 > 0.0f;
                                const float lg0 = live0 ? __log2f(r2) : 0.0f;
                                const float a0 = atan2_abs<7>(dy, dx);
                                const Pair64 p64 = pair_fp64(J, st + q, i);
                                const float lg1 = p64.live ? __log2f(fmaf(p64.ex, p64.ex, fmaf(p64.ey, p64.ey, 1e-37f))) : 0.0f;
                                const float a1 = atan2_abs(p64.ey, p64.ex);
                                const float th1 = p64.live ? signed_arg(a1, p64.sg) : 0.0f;
                                const float th0 = live0 ? fast_arg(a0, dy) : 0.0f;
                                ar[blk] += su * (lg1 - lg0);
                                ai[blk] += su * (th1 - th0);
                                if (two) {
                                    br += A.z * (lg1 - lg0);
                                    bi += A.z * (reverse_arg(a1, p64.sg) + fast_rev_neg(a0, dy));
                                }
                            }
                        }
                    }
                };
                if (uniform(cmode[k]) == kCellSym) {
                    float br = 0.0f, bi = 0.0f;
#pragma unroll
                    for (int blk = 0; blk < NB; ++blk) {
                        // distinct leaves: the 1e-37 only keeps a pair closer
                        // than FP32 resolution finite
                        const float4 A = sA[8 * blk + row];
                        const float dx = A.x - sx, dy = A.y - sy;
                        const float r2 = fmaf(dx, dx, fmaf(dy, dy, 1e-37f));
                        const float lg = __log2f(r2);
                        float mn;
                        const float a = atan2_abs<7>(dy, dx, mn);
                        keep_min(worst, mn);
                        keep_min(wclose, r2);
                        ar[blk] = fmaf(su, lg, ar[blk]);
                        ai[blk] = fmaf(su, fast_arg(a, dy), ai[blk]);
                        br = fmaf(A.z, lg, br);
                        bi = fmaf(-A.z, fast_rev_neg(a, dy), bi);
                    }
                    if (__any(flagged())) fix_pairs(true, br, bi);
                    // B's sums over the rows: lane ^ 8 by DPP (a rotation by
                    // eight within each 16-lane row), lane ^ 16 and ^ 32 by
                    // permutes with addresses computed once
                    br = add_dpp<0x128>(br);
                    bi = add_dpp<0x128>(bi);
                    br += __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(perm16, __builtin_bit_cast(int, br)));
                    bi += __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(perm16, __builtin_bit_cast(int, bi)));
                    br += __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(perm32, __builtin_bit_cast(int, br)));
                    bi += __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(perm32, __builtin_bit_cast(int, bi)));
                    const int32_t i = b + col;
                    if (row == 0 && i < ce)
                        J.bside[(int64_t)uniform(cslot[k]) * J.n_tgt + i] = make_float2(br * half_ln2, bi);
                } else {
                    // one side; a zero separation (the point itself, or an
                    // equal point) is skipped
#pragma unroll
                    for (int blk = 0; blk < NB; ++blk) {
                        const float4 A = sA[8 * blk + row];
                        const float dx = A.x - sx, dy = A.y - sy;
                        const float r2 = fmaf(dx, dx, dy * dy);
                        const bool live = r2 > 0.0f;
                        const float lg = __log2f(live ? r2 : 1.0f);
                        float mn;
                        const float th = fast_arg(atan2_abs<7>(dy, dx, mn), dy);
                        const float w = live ? su : 0.0f;
                        keep_min(worst, mn);
                        keep_min(wclose, r2);
                        ar[blk] = fmaf(w, lg, ar[blk]);
                        ai[blk] = fmaf(w, th, ai[blk]);
                    }
                    if (__any(flagged())) {
                        float unused_r = 0.0f, unused_i = 0.0f;
                        fix_pairs(false, unused_r, unused_i);
                    }
                }
                k = k2;
                b = b2;
                if (++rounds == kFlush) {
                    flush();
                    rounds = 0;
                }
            }
            flush();
        };
        switch (nblk) {
        case 1: item_rounds(std::integral_constant<int, 1>{}); break;
        case 2: item_rounds(std::integral_constant<int, 2>{}); break;
        case 3: item_rounds(std::integral_constant<int, 3>{}); break;
        case 4: item_rounds(std::integral_constant<int, 4>{}); break;
        case 5: item_rounds(std::integral_constant<int, 5>{}); break;
        case 6: item_rounds(std::integral_constant<int, 6>{}); break;
        case 7: item_rounds(std::integral_constant<int, 7>{}); break;
        default: item_rounds(std::integral_constant<int, 8>{}); break;
        }
        __syncthreads();
        if (lane < m) {
            J.nsum[2 * (st + lane)] = sre[lane] * 0.34657359027997264;   // ln 2 / 2
            J.nsum[2 * (st + lane) + 1] = sim[lane];
        }
    }
}

void batch_near_mixed_sym(const EvalJob *jobs, const BatchMap &m, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    const dim3 grid(persistent_grid(m.pre[m.n], kNearWavesPerCU));
    hipLaunchKernelGGL(k_near_mixed_sym, grid, dim3(64), 0, s, jobs, m);
}

void batch_near_mixed(const EvalJob *jobs, const BatchMap &m, hipStream_t s)
{
    if (m.n <= 0 || m.pre[m.n] <= 0) return;
    const dim3 grid(persistent_grid(m.pre[m.n], kNearWavesPerCU));
    if (m.nfield) hipLaunchKernelGGL(k_near_mixed<true>, grid, dim3(64), 0, s, jobs, m);
    else hipLaunchKernelGGL(k_near_mixed<false>, grid, dim3(64), 0, s, jobs, m);
}

}  // namespace fmm
