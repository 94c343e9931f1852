// keys.hip -- bounding box, leaf-key assignment (CellIndex) and point gather.
//
// CellIndex for the three tilings (paper Sec. 4, Sec. 5 "CellIndex",
// Sec. 6 "CellIndex").  Keys are integers whose base-4 (quadtree,
// triangle-quadtree) or base-7 (septree) digits are the hierarchical
// address, most significant digit = level 1, so the level-l key is a prefix.
//
// The floating-point decisions (floor of the scaled offset; nearest of the
// candidate lattice centres) follow one fixed expression order with no FMA
// contraction (this file is compiled with -ffp-contract=off), so the integer
// keys are reproducible bit for bit on any IEEE FP64 machine.  The integer
// parts are done in exact integer arithmetic: Morton interleave for the
// quadtree, Eisenstein-integer division by beta = 1 + 2w for the septree's
// GBT digits (w = e^{i pi/3}), integer triangle-centre units for the
// triangle-quadtree.
#include "fmm_internal.h"

namespace fmm {

// ------------------------------------------------------------ bounding box
__global__ void k_bbox(const double *__restrict__ pts, int64_t n, double *__restrict__ partial)
{
    double mnx = INFINITY, mxx = -INFINITY, mny = INFINITY, mxy = -INFINITY, bad = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double x = pts[2 * i], y = pts[2 * i + 1];
        if (!isfinite(x) || !isfinite(y)) {
            bad += 1.0;
            continue;
        }
        mnx = fmin(mnx, x);
        mxx = fmax(mxx, x);
        mny = fmin(mny, y);
        mxy = fmax(mxy, y);
    }
    for (int o = 32; o > 0; o >>= 1) {
        mnx = fmin(mnx, __shfl_xor(mnx, o));
        mxx = fmax(mxx, __shfl_xor(mxx, o));
        mny = fmin(mny, __shfl_xor(mny, o));
        mxy = fmax(mxy, __shfl_xor(mxy, o));
        bad += __shfl_xor(bad, o);
    }
    __shared__ double sh[5][16];
    int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        sh[0][w] = mnx;
        sh[1][w] = mxx;
        sh[2][w] = mny;
        sh[3][w] = mxy;
        sh[4][w] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int nw = blockDim.x >> 6;
        for (int k = 1; k < nw; ++k) {
            sh[0][0] = fmin(sh[0][0], sh[0][k]);
            sh[1][0] = fmax(sh[1][0], sh[1][k]);
            sh[2][0] = fmin(sh[2][0], sh[2][k]);
            sh[3][0] = fmax(sh[3][0], sh[3][k]);
            sh[4][0] += sh[4][k];
        }
        for (int k = 0; k < 5; ++k) partial[5 * blockIdx.x + k] = sh[k][0];
    }
}

__global__ void k_bbox_final(const double *__restrict__ partial, int nparts, double *__restrict__ out,
                             int32_t *__restrict__ zero)
{
    // One block of 256 threads reduces the partial boxes; it also clears
    // the out-of-domain counter that the key kernel increments.
    if (zero && threadIdx.x == 0) *zero = 0;
    double mnx = INFINITY, mxx = -INFINITY, mny = INFINITY, mxy = -INFINITY, bad = 0.0;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) {
        mnx = fmin(mnx, partial[5 * k]);
        mxx = fmax(mxx, partial[5 * k + 1]);
        mny = fmin(mny, partial[5 * k + 2]);
        mxy = fmax(mxy, partial[5 * k + 3]);
        bad += partial[5 * k + 4];
    }
    for (int o = 32; o > 0; o >>= 1) {
        mnx = fmin(mnx, __shfl_xor(mnx, o));
        mxx = fmax(mxx, __shfl_xor(mxx, o));
        mny = fmin(mny, __shfl_xor(mny, o));
        mxy = fmax(mxy, __shfl_xor(mxy, o));
        bad += __shfl_xor(bad, o);
    }
    __shared__ double sh[5][4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = mnx;
        sh[1][w] = mxx;
        sh[2][w] = mny;
        sh[3][w] = mxy;
        sh[4][w] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
            sh[0][0] = fmin(sh[0][0], sh[0][k]);
            sh[1][0] = fmax(sh[1][0], sh[1][k]);
            sh[2][0] = fmin(sh[2][0], sh[2][k]);
            sh[3][0] = fmax(sh[3][0], sh[3][k]);
            sh[4][0] += sh[4][k];
        }
        for (int k = 0; k < 5; ++k) out[k] = sh[k][0];
    }
}

void launch_bbox(const double *pts, int64_t n, double *partial, int nblocks, hipStream_t s)
{
    // n = 0 writes empty boxes, so the final reduction can always read them.
    hipLaunchKernelGGL(k_bbox, dim3(nblocks), dim3(256), 0, s, pts, n, partial);
}

void launch_bbox_final(const double *partial, int nparts, double *out4, int32_t *zero, hipStream_t s)
{
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(256), 0, s, partial, nparts, out4, zero);
}

// ------------------------------------------------------------------ keys
__device__ __forceinline__ uint32_t spread16(uint32_t v)
{
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// Quadtree: cell (floor((x-ox)/h), floor((y-oy)/h)) at the leaf level,
// h = side / 2^L; Morton key with x in the even bits.
__device__ int64_t key_quad(const GeoParams &g, double x, double y)
{
    double h = ldexp(g.size, -g.L);
    double fx = floor((x - g.ox) / h);
    double fy = floor((y - g.oy) / h);
    double n = ldexp(1.0, g.L);
    if (!(fx >= 0.0 && fx < n && fy >= 0.0 && fy < n)) return -1;
    return (int64_t)(spread16((uint32_t)fx) | (spread16((uint32_t)fy) << 1));
}

// Eisenstein value z = a + b w -> GBT digits (least significant first) by
// repeated division by beta.  The residue of z modulo beta is (a + 3b) mod 7
// (w = 3 mod beta); residue -> digit k whose value w^(k-1) has that residue.
// After the digit is removed, z conj(beta) = z (3 - 2w) is divisible by
// 7 = beta conj(beta).  Small values (|a|, |b| < 2^27, every point inside a
// root of up to 11 levels) divide exactly in 32-bit arithmetic by the inverse
// of 7 mod 2^32; larger ones (far outside the root) take the 64-bit path.
__device__ __forceinline__ int64_t gbt_encode(int64_t a, int64_t b, int ndig)
{
    // residue r -> digit, and the digit's (a, b) value
    const int rdig[7] = {0, 1, 3, 2, 5, 6, 4};
    const int da[7] = {0, 1, 0, -1, -1, 0, 1};
    const int db[7] = {0, 0, 1, 1, 0, -1, -1};
    const int64_t lim = (int64_t)1 << 27;
    if (a > -lim && a < lim && b > -lim && b < lim) {
        constexpr uint32_t kInv7 = 0xB6DB6DB7u;
        int32_t x = (int32_t)a, y = (int32_t)b;
        uint32_t key = 0, pw = 1;
        for (int i = 0; i < ndig; ++i) {
            int32_t r = (x + 3 * y) % 7;
            if (r < 0) r += 7;
            const int d = rdig[r];
            x -= da[d];
            y -= db[d];
            const uint32_t nx = (uint32_t)(3 * x + 2 * y), ny = (uint32_t)(y - 2 * x);
            x = (int32_t)(nx * kInv7);
            y = (int32_t)(ny * kInv7);
            key += (uint32_t)d * pw;
            pw *= 7u;
        }
        if (x != 0 || y != 0) return -1;   // needs more than ndig digits
        return key;
    }
    int64_t key = 0, pw = 1;
    for (int i = 0; i < ndig; ++i) {
        int64_t r = (a + 3 * b) % 7;
        if (r < 0) r += 7;
        int d = rdig[r];
        a -= da[d];
        b -= db[d];
        int64_t na = 3 * a + 2 * b;   // z * conj(beta), conj(beta) = 3 - 2w
        int64_t nb = b - 2 * a;
        a = na / 7;
        b = nb / 7;
        key += d * pw;
        pw *= 7;
    }
    if (a != 0 || b != 0) return -1;   // needs more than ndig digits
    return key;
}

// Septree: change of basis (b, c) = (2X/(3r), (sqrt3 Y - X)/(3r)), the four
// floor/ceil candidates, nearest lattice centre (3 r b/2, r sqrt3 (2c+b)/2)
// by squared distance with strict '<' in the listed order, then GBT digits.
__device__ int64_t key_sept(const GeoParams &g, double x, double y)
{
    const double r = g.size, s3 = g.s3;
    double X = x - g.ox, Y = y - g.oy;
    double b = (2.0 * X) / (3.0 * r);
    double c = (s3 * Y - X) / (3.0 * r);
    if (!isfinite(b) || !isfinite(c) || fabs(b) > 1e12 || fabs(c) > 1e12) return -1;
    double bf = floor(b), bc = ceil(b), cf = floor(c), cc = ceil(c);
    double cb[4] = {bf, bc, bf, bc};
    double ccc[4] = {cf, cf, cc, cc};
    int best = 0;
    double bestd = INFINITY;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double px = (3.0 * r * cb[i]) / 2.0;
        double py = (r * s3 * (2.0 * ccc[i] + cb[i])) / 2.0;
        double dx = X - px, dy = Y - py;
        double d2 = dx * dx + dy * dy;
        if (d2 < bestd) {
            bestd = d2;
            best = i;
        }
    }
    return gbt_encode((int64_t)cb[best], (int64_t)ccc[best], g.L);
}

// Triangle-quadtree: root triangle check, then descend L levels choosing
// the nearest of the four child centroids (strict '<', types 0..3).
// Centres are integer units (U, V): x = U (sqrt3/2) r, y = V r/2.
__device__ int64_t key_tri(const GeoParams &g, double x, double y)
{
    const double r = g.size, s3 = g.s3;
    double X = x - g.ox, Y = y - g.oy;
    double rho0 = ldexp(r, g.L - 1);
    double hs3 = s3 / 2.0;
    if (!isfinite(X) || !isfinite(Y)) return -1;
    if (Y < -rho0 || hs3 * X + 0.5 * Y > rho0 || -hs3 * X + 0.5 * Y > rho0) return -1;
    double ax = (s3 * r) / 2.0, ay = r / 2.0;
    int64_t U = 0, V = 0, key = 0;
    int up = 1;
    for (int i = 1; i <= g.L; ++i) {
        int64_t R = (int64_t)1 << (g.L - i);
        int64_t cu[4] = {U, U, U - R, U + R};
        int64_t cv[4] = {V, V + 2 * up * R, V - up * R, V - up * R};
        int best = 0;
        double bestd = INFINITY;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            double px = (double)cu[t] * ax, py = (double)cv[t] * ay;
            double dx = X - px, dy = Y - py;
            double d2 = dx * dx + dy * dy;
            if (d2 < bestd) {
                bestd = d2;
                best = t;
            }
        }
        U = cu[best];
        V = cv[best];
        if (best == 0) up = -up;
        key = key * 4 + best;
    }
    return key;
}

__device__ __forceinline__ int64_t key_of(const GeoParams &g, double x, double y)
{
    if (g.tiling == kQuad) return key_quad(g, x, y);
    if (g.tiling == kSept) return key_sept(g, x, y);
    return key_tri(g, x, y);
}

// ------------------------------------------------------------------ depth statistics
// Occupancy histogram at a trial leaf level (one counter per key) of every
// stride-th point.
__global__ void k_depth_hist(GeoParams g, const double *__restrict__ pts, int64_t n, int64_t stride,
                             uint32_t *__restrict__ hist)
{
    const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * stride;
    if (i >= n) return;
    const int64_t k = key_of(g, pts[2 * i], pts[2 * i + 1]);
    if (k >= 0) atomicAdd(&hist[k], 1u);
}

// All candidate levels in one pass over the trial-level histogram: thread
// per cell of the coarsest candidate level L0, which covers base^(nl-1)
// trial-level keys (keys are digit prefixes); candidate level L0 + k groups
// them base^(nl-1-k) at a time.  Accumulates per level sum_c s_c t_c and the
// source- and target-occupied cell counts (64-bit integer sums: exact in any
// order) over a bounded grid, three atomics per level and block.
constexpr int kDepthLevels = 3;
__global__ __launch_bounds__(256) void k_depth_stats(const uint32_t *__restrict__ hs, const uint32_t *__restrict__ ht,
                                                      int64_t ncells0, int base, int nl,
                                                      unsigned long long *__restrict__ out)
{
    __shared__ unsigned long long part[3 * kDepthLevels][4];
    int64_t span = 1;
    int gsz[kDepthLevels];
    for (int k = nl - 1; k >= 0; --k) {
        gsz[k] = (int)span;
        span *= base;
    }
    span /= base;   // base^(nl-1)
    unsigned long long v[3 * kDepthLevels] = {};
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncells0;
         c += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long gs[kDepthLevels] = {}, gt[kDepthLevels] = {};
        for (int64_t j = 0; j < span; ++j) {
            const unsigned long long s = hs[c * span + j], t = ht[c * span + j];
            for (int k = 0; k < nl; ++k) {
                gs[k] += s;
                gt[k] += t;
                if ((j + 1) % gsz[k] == 0) {
                    v[3 * k] += gs[k] * gt[k];
                    v[3 * k + 1] += gs[k] ? 1 : 0;
                    v[3 * k + 2] += gt[k] ? 1 : 0;
                    gs[k] = gt[k] = 0;
                }
            }
        }
    }
    // block sums first: three atomics per level and block
    for (int q = 0; q < 3 * nl; ++q) {
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o);
        if ((threadIdx.x & 63) == 0) part[q][threadIdx.x >> 6] = v[q];
    }
    __syncthreads();
    if (threadIdx.x < 3 * nl) {
        unsigned long long a = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) a += part[threadIdx.x][w];
        if (a) atomicAdd(&out[threadIdx.x], a);
    }
}

__global__ void k_copy_u64(const unsigned long long *__restrict__ a, int n, unsigned long long *__restrict__ b)
{
    if ((int)threadIdx.x < n) b[threadIdx.x] = a[threadIdx.x];
}

void launch_depth_hist(const GeoParams &g, const double *pts, int64_t n, int64_t stride, uint32_t *hist,
                       hipStream_t s)
{
    if (n <= 0) return;
    const int64_t m = (n + stride - 1) / stride;
    hipLaunchKernelGGL(k_depth_hist, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, g, pts, n, stride, hist);
}

void launch_depth_stats(const uint32_t *hs, const uint32_t *ht, int64_t ncells0, int base, int nl,
                        unsigned long long *out, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>((ncells0 + 255) / 256, 1024);
    hipLaunchKernelGGL(k_depth_stats, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s, hs, ht, ncells0,
                       base, nl, out);
}

void launch_copy_u64(const unsigned long long *a, int n, unsigned long long *b, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_u64, dim3(1), dim3(256), 0, s, a, n, b);
}

__global__ void k_keys(GeoParams g, const double *__restrict__ pts, int64_t n,
                       uint32_t *__restrict__ key, int32_t *__restrict__ idx,
                       int32_t *__restrict__ bad, int32_t *__restrict__ zero, int64_t n_zero)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n_zero) zero[i] = 0;   // the cell-flag map, cleared on the way
    if (i >= n) return;
    int64_t k = key_of(g, pts[2 * i], pts[2 * i + 1]);
    if (k < 0) {
        atomicAdd(bad, 1);
        k = 0;
    }
    key[i] = (uint32_t)k;
    idx[i] = (int32_t)i;
}

void launch_keys(const GeoParams &g, const double *pts, int64_t n, uint32_t *key, int32_t *idx,
                 int32_t *bad_count, int32_t *zero, int64_t n_zero, hipStream_t s)
{
    const int64_t m = n > n_zero ? n : n_zero;
    if (m <= 0) return;
    int64_t nb = (m + 255) / 256;
    hipLaunchKernelGGL(k_keys, dim3((unsigned)nb), dim3(256), 0, s, g, pts, n, key, idx,
                       bad_count, zero, n_zero);
}

__global__ void k_gather_points(const double *__restrict__ pts, const int32_t *__restrict__ perm,
                                int64_t n, double *__restrict__ x, double *__restrict__ y)
{
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    int64_t i = perm[j];
    x[j] = pts[2 * i];
    y[j] = pts[2 * i + 1];
}

void launch_gather_points(const double *pts, const int32_t *perm, int64_t n, double *x, double *y,
                          hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pts,
                       perm, n, x, y);
}

}  // namespace fmm
