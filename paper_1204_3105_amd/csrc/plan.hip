// plan.hip -- host side of the C ABI: planner, plan/eval drivers, exports,
// error reporting and the device-memory pool.
//
// Planner (paper Sec. 8 for p; the leaf-level rule targets a mean number of
// points per occupied leaf, the S_opt idea of Sec. 8 with the density given
// by the caller):
//   quadtree          root square = bounding square of the points, side
//                     w (1 + 2^-20) from the lower-left corner;
//                     L = smallest with max(N, M) / 4^L <= leaf_size.
//   septree           leaf hexagon 0 at the bounding-box centre; for each L
//                     the leaf radius r that makes the root aggregate's
//                     inscribed disk (c_L sqrt7^L r sqrt3) cover the box's
//                     circumscribed disk; L = smallest whose mean occupancy
//                     (box area / leaf area) is <= leaf_size.
//   triangle-quadtree upright root triangle at the box centre whose inscribed
//                     disk covers the box's circumscribed disk; L as above.
//   p = ceil(ln eps / ln q) - 1, q = max(r/R, 1/(1 + rho/r)) of the tiling.
#include <math.h>
#include <cmath>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "eval.h"
#include "fmm_tables.h"

namespace fmm {

// ------------------------------------------------------------ errors
static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

static fmm_status fail(fmm_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

// ------------------------------------------------------------ pool
// Device memory is taken in 2 MiB granules and cached on release, keyed by
// size, so repeated plans of similar size reuse their buffers.  A plan that
// runs on a caller's stream is released without waiting: its blocks carry a
// fence (an event recorded behind the plan's last work), and whoever takes
// such a block makes its stream wait for the fence (or the host, with no
// stream) before touching it.
struct Fence {
    hipEvent_t ev = nullptr;
    uint64_t id = 0;
    hipStream_t stream = nullptr;   // the stream the event was recorded on
    bool passed = false;            // the event was seen complete (it is never recorded again)
    ~Fence()
    {
        if (ev) hipEventDestroy(ev);
    }
};
struct PoolBlock {
    void *p;
    size_t bytes;
    int device;
    std::shared_ptr<Fence> fence;
};
static std::mutex g_pool_mu;
static std::vector<PoolBlock> g_pool;
static size_t g_pool_cached = 0;
static uint64_t g_fence_id = 0;
static const size_t kPoolCap = (size_t)16 << 30;

// hipEventQuery reports "not ready" as an error code, which the runtime keeps
// as the thread's last error; clear exactly that, so that a later
// hipGetLastError check sees only real failures.
static hipError_t event_query(hipEvent_t ev)
{
    const hipError_t e = hipEventQuery(ev);
    if (e == hipErrorNotReady && hipPeekAtLastError() == hipErrorNotReady) (void)hipGetLastError();
    return e;
}

static size_t round_granule(size_t b) { return (b + ((size_t)2 << 20) - 1) & ~(((size_t)2 << 20) - 1); }

static void drop_pool_locked()
{
    for (auto &b : g_pool) {
        if (b.fence) hipEventSynchronize(b.fence->ev);
        hipFree(b.p);
    }
    g_pool.clear();
    g_pool_cached = 0;
}

void *dev_alloc(size_t bytes, int *err, std::vector<uint64_t> *waited, hipStream_t stream)
{
    bytes = round_granule(bytes ? bytes : 1);
    int dev = 0;
    hipGetDevice(&dev);
    void *p = nullptr;
    std::shared_ptr<Fence> fence;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        // Among blocks of a fitting size, prefer one that needs no wait (no
        // fence, a fence on this stream, or one already passed), so plans on
        // different streams do not wait for each other's work; then the
        // smallest.
        // (A fence seen complete is remembered, so each event is queried
        // until it passes and not after; an exact fit that needs no wait ends
        // the search.)
        int best = -1, best_rank = 3;
        for (int i = 0; i < (int)g_pool.size(); ++i) {
            const PoolBlock &b = g_pool[i];
            if (b.device != dev || b.bytes < bytes || b.bytes > 2 * bytes) continue;
            int rank = 0;
            if (b.fence && !(waited && b.fence->stream == stream)) {
                if (!b.fence->passed && event_query(b.fence->ev) == hipSuccess) b.fence->passed = true;
                rank = b.fence->passed ? 1 : 2;
            }
            if (best < 0 || rank < best_rank || (rank == best_rank && b.bytes < g_pool[best].bytes)) {
                best = i;
                best_rank = rank;
            }
            if (best_rank == 0 && g_pool[best].bytes == bytes) break;
        }
        if (best >= 0) {
            p = g_pool[best].p;
            fence = std::move(g_pool[best].fence);
            if (fence && fence->passed) fence.reset();   // nothing to wait for
            g_pool_cached -= g_pool[best].bytes;
            g_pool.erase(g_pool.begin() + best);
        }
    }
    if (p) {
        if (fence) {
            // With `waited`, the block is used in the order of `stream`
            // (which may be the null stream); without, by the host.
            bool done = false;
            if (waited)
                for (uint64_t id : *waited) done = done || id == fence->id;
            if (!done) {
                if (waited) {
                    hipStreamWaitEvent(stream, fence->ev, 0);
                    waited->push_back(fence->id);
                } else {
                    hipEventSynchronize(fence->ev);
                }
            }
        }
        return p;
    }
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        // release the cache and retry once
        {
            std::lock_guard<std::mutex> lk(g_pool_mu);
            drop_pool_locked();
        }
        (void)hipGetLastError();
        e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            if (err) *err = 1;
            return nullptr;
        }
    }
    return p;
}

static void pool_put(void *p, size_t bytes, std::shared_ptr<Fence> fence)
{
    if (!p) return;
    bytes = round_granule(bytes ? bytes : 1);
    int dev = 0;
    hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (g_pool_cached + bytes > kPoolCap) {
        if (fence) hipEventSynchronize(fence->ev);
        hipFree(p);
        return;
    }
    g_pool.push_back({p, bytes, dev, std::move(fence)});
    g_pool_cached += bytes;
}

void dev_free(void *p, size_t bytes) { pool_put(p, bytes, nullptr); }

// ------------------------------------------------------------ uploads
// Host tables go to the device through a pinned ring so the copies stay on
// the plan's stream; a region is reused once the copy that read it is done.
namespace {
struct Staging {
    std::mutex mu;
    char *buf = nullptr;
    size_t cap = 0, head = 0;
    struct Use {
        size_t off, bytes;
        hipEvent_t ev;
    };
    std::vector<Use> busy;
};
Staging g_stage;
constexpr size_t kStageCap = (size_t)32 << 20;
}  // namespace

static hipError_t upload(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_stage.mu);
    if (!g_stage.buf && hipHostMalloc((void **)&g_stage.buf, kStageCap, hipHostMallocDefault) == hipSuccess)
        g_stage.cap = kStageCap;
    if (!g_stage.buf || bytes > g_stage.cap) {
        // No ring: order the synchronous copy behind the stream's work.
        (void)hipGetLastError();
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    }
    const size_t sz = (bytes + 255) & ~(size_t)255;
    if (g_stage.head + sz > g_stage.cap) g_stage.head = 0;
    const size_t off = g_stage.head;
    for (size_t i = 0; i < g_stage.busy.size();) {
        const Staging::Use &u = g_stage.busy[i];
        if (u.off < off + sz && off < u.off + u.bytes) {
            hipEventSynchronize(u.ev);
            hipEventDestroy(u.ev);
            g_stage.busy.erase(g_stage.busy.begin() + i);
        } else {
            ++i;
        }
    }
    memcpy(g_stage.buf + off, src, bytes);
    hipError_t e = hipMemcpyAsync(dst, g_stage.buf + off, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    hipEvent_t ev;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    hipEventRecord(ev, s);
    g_stage.busy.push_back({off, sz, ev});
    g_stage.head = off + sz;
    return hipSuccess;
}

// ------------------------------------------------------------ readbacks
// The planner needs two small results on the host (the bounding box, the
// level boundaries).  Kernels write them straight into coherent pinned host
// memory (one buffer per host thread, kept for the thread's life); the host
// spins on an event recorded behind the writer instead of sleeping in a
// stream synchronisation.
struct Readback {
    char *host = nullptr;
    char *dev = nullptr;
};
static constexpr size_t kReadbackBytes = 4096;

static Readback *readback()
{
    static thread_local Readback rb;
    if (!rb.host) {
        void *h = nullptr, *d = nullptr;
        if (hipHostMalloc(&h, kReadbackBytes, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
            (void)hipGetLastError();
            hipHostFree(h);
            return nullptr;
        }
        rb.host = (char *)h;
        rb.dev = (char *)d;
    }
    return &rb;
}

static hipError_t spin_wait(hipEvent_t ev, hipStream_t s)
{
    hipError_t e = hipEventRecord(ev, s);
    if (e != hipSuccess) return e;
    while ((e = event_query(ev)) == hipErrorNotReady) {
    }
    return e;
}

// ------------------------------------------------------------ plan storage
struct PlanImpl : Plan {
    std::vector<std::pair<void *, size_t>> allocs;
    std::vector<uint64_t> waited;   // fences this plan's stream already waits for
    int64_t device_bytes = 0;
    int64_t n_items_cap = 0;
    void *scratch = nullptr;
    size_t scratch_sz = 0;
    double *nfield = nullptr;     // near-field sums of the field (first field evaluation)
    double *io_field = nullptr;   // host mode: field staging
};

template <typename T>
static T *take(PlanImpl *P, int64_t count, int *err)
{
    size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    void *p = dev_alloc(bytes, err, &P->waited, P->stream);
    if (p) {
        P->allocs.push_back({p, bytes});
        P->device_bytes += (int64_t)round_granule(bytes);
    }
    return (T *)p;
}

static void release(PlanImpl *P)
{
    std::shared_ptr<Fence> fence;
    if (!P->own_stream && !P->allocs.empty()) {
        fence = std::make_shared<Fence>();
        fence->stream = P->stream;
        if (hipEventCreateWithFlags(&fence->ev, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(fence->ev, P->stream) != hipSuccess) {
            (void)hipGetLastError();
            fence.reset();
        } else {
            std::lock_guard<std::mutex> lk(g_pool_mu);
            fence->id = ++g_fence_id;
        }
    }
    if (!fence) hipStreamSynchronize(P->stream);
    for (auto &a : P->allocs) pool_put(a.first, a.second, fence);
    P->allocs.clear();
    for (auto &e : P->ev)
        if (e) hipEventDestroy(e);
    if (P->own_stream && P->stream) hipStreamDestroy(P->stream);
}

// Hand a block used on stream s back to the pool behind a fence recorded on
// s (or after waiting for s if no event can be made).
static void put_fenced(void *p, size_t bytes, hipStream_t s)
{
    auto fence = std::make_shared<Fence>();
    fence->stream = s;
    if (hipEventCreateWithFlags(&fence->ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(fence->ev, s) != hipSuccess) {
        (void)hipGetLastError();
        fence.reset();
        hipStreamSynchronize(s);
    } else {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        fence->id = ++g_fence_id;
    }
    pool_put(p, bytes, fence);
}

int64_t plan_device_bytes(const Plan *P) { return ((const PlanImpl *)P)->device_bytes; }

static int order_for(int tiling, double eps);

// Device bytes a plan of these sizes takes, from the buffers build_plan
// allocates (a bound for admission: the depth rule and the point layout
// decide the exact cell counts).  Per point: inputs, sorted coordinates,
// keys, permutation, strengths, the sort's scratch, near sums, output, the
// mixed form's FP32 copies and the symmetric near field's second-side sums;
// per cell (at most 3 n / leaf over all levels, more for clustered inputs
// at deeper levels): multipole and local rows, E4 and near lists, the dense
// key maps, the M2L tiles; plus 2 MiB granules per buffer.
int64_t plan_bytes_estimate(int tiling, int64_t n_src, int64_t n_tgt, bool same, double eps, int precision,
                            int leaf_size)
{
    int prec = precision;
    if (prec == FMM_PREC_AUTO || (prec == FMM_PREC_MIXED && !(eps >= kMixedMinEps)))
        prec = eps >= kMixedMinEps ? FMM_PREC_MIXED : FMM_PREC_FP64;
    const int p = std::max(order_for(tiling, eps), 1);
    const int ew = tiling == kQuad ? 27 : tiling == kSept ? 42 : 39;
    const int nw = tiling == kQuad ? 9 : tiling == kSept ? 7 : 13;
    const int64_t pts = std::max(n_src, n_tgt);
    const int64_t sides = same ? 1 : 2;
    int64_t per_pt = 24 + sides * 40 + 24 + 32;   // inputs, sorted arrays, sort scratch, sums and output
    if (prec == FMM_PREC_MIXED) per_pt += sides * 12 + (same ? (nw - 1) * kSymChunks * 8 : 0);
    else if (same) per_pt += (nw - 1) * kSymChunks * 16;
    const int64_t cells = 3 * pts / std::max(leaf_size, 1) + 64;
    int64_t per_cell = 2 * 16 * (p + 1) + 4 * (ew + nw) + 64 + 48;
    per_cell += 24;   // M2L tiles: cell list, sort keys and the sort scratch
    return per_pt * pts + per_cell * cells + ((int64_t)48 << 20);
}

// ------------------------------------------------------------ fixed scratch
// Device scratch of fmm_direct_noalloc: the slices' partial sums (complex128
// per slice and target).  The slicing rule (direct_slices) keeps them under
// 12 MiB for every size, so 16 MiB covers all calls; each GPU the library
// runs on holds its own copy until the process ends.
static constexpr size_t kDirectScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) double direct_scratch[kDirectScratchBytes / sizeof(double)];

// The device address of this device's direct_scratch, looked up once per
// device with that device current (the host-side name of the array is not
// a device address).
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64] = {};

static fmm_status direct_scratch_ptr(void **out)
{
    int dev = 0;
    FMM_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(FMM_E_DEVICE, "device ordinal out of range for the fixed scratch");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(direct_scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(FMM_E_DEVICE, std::string("hipGetSymbolAddress(direct_scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FMM_OK;
}

// ------------------------------------------------------------ rules
static const double kQ[3] = {
    0.54691816067802259,   // quadtree 1/(1 + 2(sqrt2 - 1))
    0.52443357281057,      // septree, GBT aggregates: 1/(1 + rho/r) with rho/r = 0.906819,
                           // the smallest over 0..10 levels above the leaves (reached at 8)
    0.60762521851393328    // triangle-quadtree 1/(sqrt7 - 1)
};

static int order_for(int tiling, double eps)
{
    if (!(eps > 0.0 && eps < 0.5) || tiling < 0 || tiling > 2) return -1;
    int p = (int)ceil(log(eps) / log(kQ[tiling])) - 1;
    return std::max(1, std::min(p, kMaxP));
}

struct BBox {
    double x0, x1, y0, y1;
};

static void choose_geometry(int tiling, const BBox &bb, int64_t nmax, int leaf, int lmax_opt,
                            GeoParams &g)
{
    double cx = 0.5 * (bb.x0 + bb.x1), cy = 0.5 * (bb.y0 + bb.y1);
    double wx = bb.x1 - bb.x0, wy = bb.y1 - bb.y0;
    double rho = 0.5 * hypot(wx, wy);
    if (!(rho > 0.0)) rho = 1.0;
    double area = std::max(wx * wy, 0.01 * M_PI * rho * rho);
    double dens = (double)std::max<int64_t>(nmax, 1);
    g.tiling = tiling;
    g.s3 = sqrt(3.0);
    if (tiling == kQuad) {
        double w = std::max(wx, wy);
        if (!(w > 0.0)) w = 1.0;
        g.ox = bb.x0;
        g.oy = bb.y0;
        g.size = w * (1.0 + ldexp(1.0, -20));
        int L = 0;
        while (L < 15 && dens / ldexp(1.0, 2 * L) > leaf) ++L;
        g.L = lmax_opt >= 0 ? lmax_opt : L;
    } else if (tiling == kSept) {
        g.ox = cx;
        g.oy = cy;
        double rr = rho * (1.0 + 1e-9);
        int Lmax = (int)(sizeof(kSeptInscribed) / sizeof(double)) - 1;
        int L = 0;
        double r = 0;
        for (L = 0; L <= Lmax; ++L) {
            r = rr / (kSeptInscribed[L] * (1.0 - 1e-9) * pow(sqrt(7.0), L) * sqrt(3.0));
            double leaf_area = 1.5 * sqrt(3.0) * r * r;
            if (dens / std::max(1.0, area / leaf_area) <= leaf || L == Lmax) break;
        }
        if (lmax_opt >= 0) {
            L = std::min(lmax_opt, Lmax);
            r = rr / (kSeptInscribed[L] * (1.0 - 1e-9) * pow(sqrt(7.0), L) * sqrt(3.0));
        }
        g.L = L;
        g.size = r;
    } else {
        g.ox = cx;
        g.oy = cy;
        double rr = rho * (1.0 + 1e-9);
        int L = 0;
        double r = 0;
        for (L = 0; L <= 15; ++L) {
            r = 2.0 * rr / ldexp(1.0, L);
            double leaf_area = 0.75 * sqrt(3.0) * r * r;
            if (dens / std::max(1.0, area / leaf_area) <= leaf || L == 15) break;
        }
        if (lmax_opt >= 0) {
            L = lmax_opt;
            r = 2.0 * rr / ldexp(1.0, L);
        }
        g.L = L;
        g.size = r;
    }
}

static double level_scale(const GeoParams &g, int l)
{
    if (g.tiling == kQuad) return ldexp(g.size, -l);
    if (g.tiling == kSept) return g.size * sqrt(3.0) * pow(sqrt(7.0), g.L - l);
    return ldexp(g.size, g.L - l);
}

static int key_bits(const GeoParams &g)
{
    if (g.tiling == kSept) {
        double k = 1;
        for (int i = 0; i < g.L; ++i) k *= 7.0;
        int b = 0;
        while ((double)((uint64_t)1 << b) < k) ++b;
        return b;
    }
    return 2 * g.L;
}

static float elapsed(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();
        return 0.f;
    }
    return ms;
}

// ------------------------------------------------------------ plan
// Depth by a cost model (fmm_options.depth_rule = FMM_DEPTH_COST).  From the
// points' occupancy histogram at a trial level Lc = L0 + 2 (L0 from the mean
// rule; base^Lc <= 2^24), each candidate leaf level l in [L0, Lc] is priced
// as a uniform-depth tree: near-field pairs ~ (near slots) sum_c s_c t_c over
// the level's cells (from every m-th point, m making at most 2^20 samples,
// scaled back), a cost per occupied leaf (near-field item, L2P, shifts),
// and M2L pairs ~ (E4 slots) min(source cells, target cells) per level added
// below L0; the cheapest level wins (ties: the shallower).  The weights are
// per-unit times measured on this GPU for the mixed and the FP64 forms.
static int depth_trial_level(int tiling, int L0)
{
    const int cap = tiling == kSept ? std::min(8, (int)(sizeof(kSeptInscribed) / sizeof(double)) - 1) : 12;
    return std::max(L0, std::min(L0 + 2, cap));
}

// Scratch bytes of the depth statistics (the histogram, then 3 counters per
// level); the plan lends its sort scratch, which the sort uses later.
static size_t depth_scratch_bytes(int tiling, int L0, bool same)
{
    const int Lc = depth_trial_level(tiling, L0);
    int64_t K = 1;
    for (int i = 0; i < Lc; ++i) K *= base_of(tiling);
    return sizeof(uint32_t) * (size_t)K * (same ? 1 : 2) + 256 + sizeof(unsigned long long) * 3 * (Lc - L0 + 1);
}

static fmm_status depth_by_cost(PlanImpl *P, int tiling, const BBox &bb, int64_t N, int64_t M, const double *dsrc,
                                const double *dtgt, bool same, const fmm_options &o, int p, int L0, Readback *rb,
                                char *scratch, int *out_L)
{
    *out_L = L0;
    hipStream_t s = P->stream;
    const int base = base_of(tiling);
    const int Lc = depth_trial_level(tiling, L0);
    if (Lc <= L0) return FMM_OK;
    GeoParams gc;
    choose_geometry(tiling, bb, std::max(N, M), o.leaf_size, Lc, gc);
    int64_t K = 1;
    for (int i = 0; i < Lc; ++i) K *= base;
    const int nl = Lc - L0 + 1;
    const size_t hb = sizeof(uint32_t) * (size_t)K * (same ? 1 : 2), ab = sizeof(unsigned long long) * 3 * nl;
    uint32_t *hist = (uint32_t *)scratch;
    unsigned long long *acc = (unsigned long long *)(scratch + ((hb + 255) & ~(size_t)255));
    uint32_t *hs = hist, *ht = same ? hist : hist + K;
    // At most 2^20 sampled points per side (every m-th): counts are scaled
    // back by m; occupied cells are those with a sampled point.
    const int64_t ms = std::max<int64_t>(1, (N + (1 << 20) - 1) >> 20);
    const int64_t mt = same ? ms : std::max<int64_t>(1, (M + (1 << 20) - 1) >> 20);
    hipError_t e = hipMemsetAsync(hist, 0, hb, s);
    if (e == hipSuccess) e = hipMemsetAsync(acc, 0, ab, s);
    if (e == hipSuccess) {
        launch_depth_hist(gc, dsrc, N, ms, hs, s);
        if (!same) launch_depth_hist(gc, dtgt, M, mt, ht, s);
        int64_t cells0 = 1;
        for (int l = 0; l < L0; ++l) cells0 *= base;
        launch_depth_stats(hs, ht, cells0, base, nl, acc, s);
        launch_copy_u64(acc, 3 * nl, (unsigned long long *)rb->dev, s);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = spin_wait(P->ev[11], s);
    if (e != hipSuccess) return fail(FMM_E_DEVICE, std::string("depth statistics failed: ") + hipGetErrorString(e));
    unsigned long long st[3 * (kMaxL + 1)];
    memcpy(st, (const void *)rb->host, sizeof(unsigned long long) * 3 * nl);
    const ListTables t = build_tables(tiling);
    const bool mixed = P->precision == FMM_PREC_MIXED;
    const double q = (p + 1) / 23.0;
    const double w_pair = mixed ? 1.1e-12 : 4.5e-12;
    const double w_leaf = mixed ? 2.0e-9 : 2.5e-9;
    const double w_m2l = (mixed ? 1.5e-10 : 1.0e-9) * q * q;
    double best = 0.0, m2l = 0.0;
    for (int l = L0; l <= Lc; ++l) {
        const double pairs = (double)t.near_width * (double)st[3 * (l - L0)] * (double)ms * (double)mt;
        const double cs = (double)st[3 * (l - L0) + 1], ct = (double)st[3 * (l - L0) + 2];
        if (l > L0) m2l += (double)t.e4_width * std::min(cs, ct);
        const double c = w_pair * pairs + w_leaf * (cs + ct) + w_m2l * m2l;
        if (l == L0 || c < best) {
            best = c;
            *out_L = l;
        }
    }
    return FMM_OK;
}

// The symmetric near field addresses its second-side sums by 32-bit offsets
// ((slot) n + point); above that many points the plan takes the one-sided
// kernels.
static bool sym_offsets_fit(int nw, int64_t n) { return (int64_t)(nw - 1) * kSymChunks * n < ((int64_t)1 << 31); }

static fmm_status build_plan(PlanImpl *P, int tiling, const double *src, int64_t n_src,
                             const double *tgt, int64_t n_tgt, double eps, const fmm_options &o)
{
    int err = 0;
    hipStream_t s = P->stream;
    const bool same = P->same;
    // Device copies of the inputs.
    const double *dsrc = src, *dtgt = tgt;
    if (!o.device_pointers) {
        double *a = take<double>(P, 2 * std::max<int64_t>(n_src, 1), &err);
        double *b = same ? a : take<double>(P, 2 * std::max<int64_t>(n_tgt, 1), &err);
        if (err) return fail(FMM_E_NOMEM, "device allocation failed (inputs)");
        if (n_src) FMM_HIP_CHECK(hipMemcpyAsync(a, src, 16 * n_src, hipMemcpyHostToDevice, s));
        if (!same && n_tgt)
            FMM_HIP_CHECK(hipMemcpyAsync(b, tgt, 16 * n_tgt, hipMemcpyHostToDevice, s));
        dsrc = a;
        dtgt = b;
    }
    FMM_HIP_CHECK(hipEventRecord(P->ev[0], s));

    // Bounding box (sources and targets), also flags non-finite input.
    const int nbb = 1024;   // partial boxes: four points per thread
    double *bbp = take<double>(P, 5 * 2 * nbb, &err);
    if (err) return fail(FMM_E_NOMEM, "device allocation failed (bbox)");
    // The source and target partial boxes are reduced together.
    int32_t *bad = take<int32_t>(P, 4, &err);   // out-of-domain count, cleared by the bbox pass
    if (err) return fail(FMM_E_NOMEM, "device allocation failed (bbox)");
    launch_bbox(dsrc, n_src, bbp, nbb, s);
    if (!same) launch_bbox(dtgt, n_tgt, bbp + 5 * nbb, nbb, s);
    Readback *rb = readback();
    if (!rb) return fail(FMM_E_DEVICE, "pinned readback buffer unavailable");
    launch_bbox_final(bbp, same ? nbb : 2 * nbb, (double *)rb->dev, bad, s);
    FMM_HIP_CHECK(spin_wait(P->ev[10], s));
    double hb[5];
    memcpy(hb, (const void *)rb->host, sizeof(hb));
    if (hb[4] > 0) return fail(FMM_E_INVALID, "non-finite coordinate in the input");
    if (n_src + n_tgt == 0) hb[0] = hb[2] = 0.0, hb[1] = hb[3] = 1.0;

    GeoParams &g = P->geo;
    char *sort_tmp = nullptr;   // sort scratch (lent to the depth statistics first)
    if (o.has_geometry) {
        if (o.lmax < 0 || o.lmax > kMaxL) return fail(FMM_E_INVALID, "explicit geometry needs 0 <= lmax <= 16");
        if (!(o.geometry[2] > 0.0) || !isfinite(o.geometry[0]) || !isfinite(o.geometry[1]))
            return fail(FMM_E_INVALID, "bad explicit geometry");
        g.tiling = tiling;
        g.L = o.lmax;
        g.ox = o.geometry[0];
        g.oy = o.geometry[1];
        g.size = o.geometry[2];
        g.s3 = sqrt(3.0);
    } else {
        BBox bb{hb[0], hb[1], hb[2], hb[3]};
        choose_geometry(tiling, bb, std::max(n_src, n_tgt), o.leaf_size, o.lmax, g);
        if (o.depth_rule == FMM_DEPTH_COST && o.lmax < 0 && n_src > 0 && n_tgt > 0) {
            const int pp = o.p > 0 ? std::min(o.p, kMaxP) : order_for(tiling, eps);
            const size_t need = std::max(radix_tmp_bytes(std::max(n_src, n_tgt)), depth_scratch_bytes(tiling, g.L, same));
            sort_tmp = take<char>(P, (int64_t)need, &err);
            if (err) return fail(FMM_E_NOMEM, "device allocation failed (depth statistics)");
            int L = g.L;
            const fmm_status st =
                depth_by_cost(P, tiling, bb, n_src, n_tgt, dsrc, dtgt, same, o, pp, g.L, rb, sort_tmp, &L);
            if (st != FMM_OK) return st;
            if (L != g.L) choose_geometry(tiling, bb, std::max(n_src, n_tgt), o.leaf_size, L, g);
        }
    }
    if (g.L > kMaxL || (tiling == kSept && g.L > 11))
        return fail(FMM_E_INVALID, "tree too deep for 32-bit keys");
    P->p = o.p > 0 ? std::min(o.p, kMaxP) : order_for(tiling, eps);
    for (int l = 0; l <= g.L; ++l) P->scale[l] = level_scale(g, l);

    // Keys and sort.
    const int64_t N = n_src, M = n_tgt;
    P->skey = take<uint32_t>(P, N, &err);
    P->sperm = take<int32_t>(P, N, &err);
    P->sx = take<double>(P, N, &err);
    P->sy = take<double>(P, N, &err);
    if (same) {
        P->tkey = P->skey;
        P->tperm = P->sperm;
        P->tx = P->sx;
        P->ty = P->sy;
    } else {
        P->tkey = take<uint32_t>(P, M, &err);
        P->tperm = take<int32_t>(P, M, &err);
        P->tx = take<double>(P, M, &err);
        P->ty = take<double>(P, M, &err);
    }
    if (!sort_tmp) sort_tmp = take<char>(P, (int64_t)std::max(radix_tmp_bytes(N), radix_tmp_bytes(M)), &err);
    if (err) return fail(FMM_E_NOMEM, "device allocation failed (keys)");
    // Levels: dense key spaces; the key pass clears their occupancy flags.
    int64_t dense_total = 0;
    for (int l = 0; l <= g.L; ++l) {
        int64_t K = 1;
        for (int k = 0; k < l; ++k) K *= base_of(tiling);
        P->lev[l].K = K;
        P->lev[l].dense_off = dense_total;
        dense_total += K;
    }
    P->dense_total = dense_total;
    int32_t *flags = take<int32_t>(P, 2 * dense_total + 1, &err);
    if (err) return fail(FMM_E_NOMEM, "device allocation failed (levels)");
    launch_keys(g, dsrc, N, P->skey, P->sperm, bad, flags, dense_total, s);
    if (!same) launch_keys(g, dtgt, M, P->tkey, P->tperm, bad, nullptr, 0, s);
    int bits = key_bits(g);
    radix_sort(P->skey, P->sperm, N, bits, sort_tmp, s);
    if (!same) radix_sort(P->tkey, P->tperm, M, bits, sort_tmp, s);
    launch_gather_points(dsrc, P->sperm, N, P->sx, P->sy, s);
    if (!same) launch_gather_points(dtgt, P->tperm, M, P->tx, P->ty, s);

    P->dense = take<int32_t>(P, dense_total, &err);
    char *scan_tmp = take<char>(P, (int64_t)scan_tmp_bytes(std::max<int64_t>(dense_total, 256 * 1024)) + 4096, &err);
    int32_t *total = take<int32_t>(P, 4, &err);
    if (err) return fail(FMM_E_NOMEM, "device allocation failed (levels)");
    if (same) {
        launch_mark_cells(g, P->lev, P->skey, N, 3, flags, s);   // both occupancy bits at once
    } else {
        launch_mark_cells(g, P->lev, P->skey, N, 1, flags, s);
        launch_mark_cells(g, P->lev, P->tkey, M, 2, flags, s);
    }
    launch_flags_to_ids(flags, dense_total, s);
    int32_t *ids = flags + dense_total;
    scan_exclusive(ids, ids, dense_total, total, scan_tmp, s);
    // Level boundaries and the out-of-domain count -> host, in one copy.
    std::vector<int32_t> bnd(g.L + 3);
    launch_gather_bounds(P->lev, g.L, ids, total, bad, (int32_t *)rb->dev, s);
    FMM_HIP_CHECK(spin_wait(P->ev[11], s));
    memcpy(bnd.data(), (const void *)rb->host, sizeof(int32_t) * (g.L + 3));
    const int32_t hbad = bnd[g.L + 2];
    if (hbad) return fail(FMM_E_DOMAIN, "points outside the root of the given geometry");
    for (int l = 0; l <= g.L; ++l) {
        P->lev[l].cell_off = bnd[l];
        P->lev[l].n = bnd[l + 1] - bnd[l];
    }
    P->n_cells = bnd[g.L + 1];
    const int64_t C = std::max<int64_t>(P->n_cells, 1);
    const int64_t NL = std::max<int64_t>(P->lev[g.L].n, 1);

    // Per-cell arrays.
    P->tables = build_tables(tiling);
    const int ew = P->tables.e4_width, nw = P->tables.near_width;
    P->cell_key = take<uint32_t>(P, C, &err);
    P->cell_occ = take<uint8_t>(P, C, &err);
    P->sb = take<int32_t>(P, C, &err);
    P->se = take<int32_t>(P, C, &err);
    if (same) {
        P->tb = P->sb;
        P->te = P->se;
    } else {
        P->tb = take<int32_t>(P, C, &err);
        P->te = take<int32_t>(P, C, &err);
    }
    P->cx = take<double>(P, C, &err);
    P->cy = take<double>(P, C, &err);
    P->parent = take<int32_t>(P, C, &err);
    P->group = take<uint8_t>(P, C, &err);
    P->e4 = take<int32_t>(P, C * ew, &err);
    P->near = take<int32_t>(P, NL * nw, &err);
    P->mp = take<double>(P, C * 2 * (P->p + 1), &err);
    P->lc = take<double>(P, C * 2 * (P->p + 1), &err);
    P->binom = device_binom(&err);
    P->su = take<double>(P, N, &err);
    int32_t *ncount = take<int32_t>(P, NL + 1, &err);
    int64_t items_cap = (M + kChunk - 1) / kChunk + NL + 1;
    P->work_near = take<int32_t>(P, 2 * items_cap, &err);
    P->counts = take<int32_t>(P, 8, &err);
    if (err) return fail(FMM_E_NOMEM, "device allocation failed (cells)");

    // Compaction also clears the root's local expansion: only a one-level
    // tree reads a local expansion that no M2L writes.
    launch_compact(g, P->lev, dense_total, flags, ids, P->dense, P->cell_key, P->cell_occ, P->sb,
                   P->se, same ? nullptr : P->tb, same ? nullptr : P->te, P->lc, 2 * (P->p + 1), s);
    launch_cell_ranges(g, P->lev, P->skey, N, P->dense, P->sb, P->se, s);
    if (!same) launch_cell_ranges(g, P->lev, P->tkey, M, P->dense, P->tb, P->te, s);
    launch_cell_geometry(g, P->lev, P->n_cells, P->cell_key, P->dense, P->sb, P->se, P->tb, P->te,
                         P->cx, P->cy, P->parent, P->group, P->cell_occ, s);
    launch_lists(g, P->lev, P->tables, P->n_cells, P->cell_key, P->group, P->cell_occ, P->dense,
                 P->e4, P->near, s);
    launch_near_items(P->lev, g.L, P->tb, P->te, ncount, s);
    scan_exclusive(ncount, ncount, P->lev[g.L].n, P->counts + 0, scan_tmp, s);
    launch_near_items_fill(P->lev, g.L, P->tb, P->te, ncount, P->work_near, s);
    if (P->lev[g.L].n > 0 && M > 0) {
        // the items in decreasing order of estimated cost
        uint32_t *ikeys = take<uint32_t>(P, items_cap, &err);
        int32_t *ivals = take<int32_t>(P, items_cap, &err);
        int32_t *sorted = take<int32_t>(P, 2 * items_cap, &err);
        char *itmp = take<char>(P, (int64_t)radix_tmp_bytes(items_cap), &err);
        if (err) return fail(FMM_E_NOMEM, "device allocation failed (near items)");
        // (the FP64 symmetric kernel takes leaves of up to kWide targets as
        // one item and small items in its four-row tile)
        const bool sym64 = P->precision != FMM_PREC_MIXED && same && N > 0 && sym_offsets_fit(nw, N);
        launch_near_items_order(P->lev[g.L].cell_off, nw, sym64 ? kWide : kChunk, sym64 ? kSmall : 0,
                                (int32_t)items_cap, P->counts + 0, P->work_near, P->tb, P->te, P->near, P->sb, P->se,
                                ikeys, ivals, itmp, sorted, s);
        P->work_near = sorted;
    }
    P->m2l_pm = m2l_pm_for(P->p);
    if (P->m2l_pm > 0 && g.L >= 1) {
        double *tab = take<double>(P, (int64_t)m2l_table_doubles(*P, P->m2l_pm), &err);
        if (err) return fail(FMM_E_NOMEM, "device allocation failed (M2L tables)");
        launch_m2l_tables(*P, P->m2l_pm, tab, s);
    }
    if (P->precision == FMM_PREC_MIXED) {
        P->sxl = take<float>(P, N, &err);
        P->syl = take<float>(P, N, &err);
        P->suf = take<float>(P, N, &err);
        if (same) {
            P->txl = P->sxl;
            P->tyl = P->syl;
        } else {
            P->txl = take<float>(P, M, &err);
            P->tyl = take<float>(P, M, &err);
        }
        if (same && N > 0 && sym_offsets_fit(nw, N))
            P->bside = take<float2>(P, (int64_t)(nw - 1) * kSymChunks * N, &err);
        if (err) return fail(FMM_E_NOMEM, "device allocation failed (mixed)");
        launch_local_coords(P->sx, P->sy, P->skey, N, g, P->lev, P->dense, P->cx, P->cy, P->sxl,
                            P->syl, s);
        if (!same)
            launch_local_coords(P->tx, P->ty, P->tkey, M, g, P->lev, P->dense, P->cx, P->cy,
                                P->txl, P->tyl, s);
        size_t mb = mixed_bytes(*P);
        P->mixed = take<char>(P, (int64_t)mb, &err);
        if (err) return fail(FMM_E_NOMEM, "device allocation failed (mixed M2L)");
        if (mixed_setup(*P)) return fail(FMM_E_DEVICE, "mixed-precision setup failed");
    } else if (P->m2l_pm > 0 && g.L >= 1 && m2l_f64_mfma_class(P->p) > 0) {
        // FP64 M2L on MFMA: target tiles grouped by (level, group)
        P->mixed = take<char>(P, (int64_t)mixed_bytes(*P), &err);
        if (err) return fail(FMM_E_NOMEM, "device allocation failed (M2L tiles)");
        if (mixed_setup(*P)) return fail(FMM_E_DEVICE, "M2L tile setup failed");
    }
    FMM_HIP_CHECK(hipEventRecord(P->ev[1], s));
    // Item counts stay on the device; launches use these upper bounds and
    // kernels stop at the counts.
    P->n_work_near = P->lev[g.L].n > 0 && M > 0 ? items_cap : 0;
    P->n_m2l_pairs = P->n_near_pairs = -1;   // counted on first request
    if (!o.device_pointers) {
        P->io_u = take<double>(P, std::max<int64_t>(N, 1), &err);
        P->io_phi = take<double>(P, 2 * std::max<int64_t>(M, 1), &err);
        if (err) return fail(FMM_E_NOMEM, "device allocation failed (io)");
    }
    P->phi_int = take<double>(P, 2 * std::max<int64_t>(M, 1), &err);
    P->nsum = take<double>(P, 2 * std::max<int64_t>(M, 1), &err);
    if (P->precision != FMM_PREC_MIXED && same && N > 0 && sym_offsets_fit(nw, N))
        P->bside64 = take<double2>(P, (int64_t)(nw - 1) * kSymChunks * N, &err);
    if (P->lev[g.L].n == 0 || M == 0) FMM_HIP_CHECK(hipMemsetAsync(P->counts, 0, sizeof(int32_t), s));
    P->job_dev = take<EvalJob>(P, 1, &err);
    if (err) return fail(FMM_E_NOMEM, "device allocation failed (descriptor)");
    EvalJob J = make_job(*P);
    FMM_HIP_CHECK(upload(P->job_dev, &J, sizeof(J), s));
    return FMM_OK;
}

}  // namespace fmm

using namespace fmm;

extern "C" {

fmm_status fmm_options_default(fmm_options *opt)
{
    if (!opt) return fail(FMM_E_INVALID, "null options");
    memset(opt, 0, sizeof(*opt));
    opt->struct_size = sizeof(fmm_options);
    opt->leaf_size = 64;
    opt->lmax = -1;
    opt->p = -1;
    opt->precision = FMM_PREC_AUTO;
    return FMM_OK;
}

int32_t fmm_order_for_eps(fmm_tiling tiling, double eps) { return order_for((int)tiling, eps); }

fmm_status fmm_direct(const double *src, int64_t n_src, const double *tgt, int64_t n_tgt,
                      const double *u, double *phi, const fmm_options *opt)
{
    g_err.clear();
    if (n_src < 0 || n_tgt < 0) return fail(FMM_E_INVALID, "negative size");
    if ((n_src > 0 && (!src || !u)) || (n_tgt > 0 && (!tgt || !phi)))
        return fail(FMM_E_INVALID, "null array");
    if (opt && opt->struct_size != sizeof(fmm_options)) return fail(FMM_E_INVALID, "bad options struct size");
    if (n_tgt == 0) return FMM_OK;
    const bool dev = opt && opt->device_pointers;
    const int slices = direct_slices(n_src, n_tgt);
    const size_t bpart = slices > 1 ? 16 * (size_t)slices * (size_t)n_tgt : 0;
    if (dev) {
        // The partial sums live in a pool block used in stream order and
        // handed back behind a fence, so the call does not wait.
        hipStream_t s = (hipStream_t)opt->stream;
        int err = 0;
        std::vector<uint64_t> waited;
        double *part = bpart ? (double *)dev_alloc(bpart, &err, &waited, s) : nullptr;
        if (err) return fail(FMM_E_NOMEM, "device allocation failed (direct)");
        launch_direct(src, n_src, tgt, n_tgt, u, phi, part, slices, s);
        const hipError_t e = hipGetLastError();
        if (part) put_fenced(part, bpart, s);
        FMM_HIP_CHECK(e);
        return FMM_OK;
    }
    for (int64_t i = 0; i < 2 * n_src; ++i)
        if (!std::isfinite(src[i])) return fail(FMM_E_INVALID, "non-finite coordinate in the input");
    for (int64_t i = 0; i < 2 * n_tgt; ++i)
        if (!std::isfinite(tgt[i])) return fail(FMM_E_INVALID, "non-finite coordinate in the input");
    hipStream_t s;
    FMM_HIP_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    int err = 0;
    const size_t bs = 16 * (size_t)std::max<int64_t>(n_src, 1), bt = 16 * (size_t)n_tgt;
    const size_t bu = 8 * (size_t)std::max<int64_t>(n_src, 1);
    double *ds = (double *)dev_alloc(bs, &err), *dt = (double *)dev_alloc(bt, &err);
    double *du = (double *)dev_alloc(bu, &err), *dp = (double *)dev_alloc(bt, &err);
    double *part = bpart ? (double *)dev_alloc(bpart, &err) : nullptr;
    fmm_status st = FMM_OK;
    if (err) {
        st = fail(FMM_E_NOMEM, "device allocation failed (direct)");
    } else if (hipMemcpyAsync(ds, src, 16 * n_src, hipMemcpyHostToDevice, s) != hipSuccess ||
               hipMemcpyAsync(dt, tgt, bt, hipMemcpyHostToDevice, s) != hipSuccess ||
               hipMemcpyAsync(du, u, 8 * n_src, hipMemcpyHostToDevice, s) != hipSuccess) {
        st = fail(FMM_E_DEVICE, "host to device copy failed (direct)");
    } else {
        launch_direct(ds, n_src, dt, n_tgt, du, dp, part, slices, s);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(phi, dp, bt, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = fail(FMM_E_DEVICE, "direct sum failed");
    }
    hipStreamSynchronize(s);
    dev_free(ds, bs);
    dev_free(dt, bt);
    dev_free(du, bu);
    dev_free(dp, bt);
    dev_free(part, bpart);
    hipStreamDestroy(s);
    return st;
}

fmm_status fmm_direct_noalloc(const double *src, int64_t n_src, const double *tgt, int64_t n_tgt,
                              const double *u, double *phi, void *stream)
{
    g_err.clear();
    if (n_src < 0 || n_tgt < 0) return fail(FMM_E_INVALID, "negative size");
    if ((n_src > 0 && (!src || !u)) || (n_tgt > 0 && (!tgt || !phi)))
        return fail(FMM_E_INVALID, "null array");
    if (n_tgt == 0) return FMM_OK;
    const int slices = direct_slices(n_src, n_tgt);
    const size_t bpart = slices > 1 ? 16 * (size_t)slices * (size_t)n_tgt : 0;
    if (bpart > kDirectScratchBytes)
        return fail(FMM_E_INVALID, "direct sum: partial sums need " + std::to_string(bpart) +
                                       " bytes, the fixed scratch holds " + std::to_string(kDirectScratchBytes));
    double *part = nullptr;
    if (bpart) {
        void *ptr = nullptr;
        const fmm_status st = direct_scratch_ptr(&ptr);
        if (st != FMM_OK) return st;
        part = (double *)ptr;
    }
    launch_direct(src, n_src, tgt, n_tgt, u, phi, part, slices, (hipStream_t)stream);
    FMM_HIP_CHECK(hipGetLastError());
    return FMM_OK;
}

fmm_status fmm_probe_pair_rate(int32_t rounds, int32_t blocks, double *evals_per_s)
{
    g_err.clear();
    if (rounds < 1 || blocks < 0 || !evals_per_s) return fail(FMM_E_INVALID, "bad probe arguments");
    if (probe_pair_rate(rounds, blocks ? blocks : 3072, evals_per_s))
        return fail(FMM_E_DEVICE, "pair-rate probe failed");
    return FMM_OK;
}

fmm_status fmm_plan(fmm_tiling tiling, const double *src, int64_t n_src, const double *tgt,
                    int64_t n_tgt, double eps, const fmm_options *opt, fmm_plan_t *out)
{
    g_err.clear();
    if (!out) return fail(FMM_E_INVALID, "null output plan pointer");
    *out = nullptr;
    fmm_options o;
    fmm_options_default(&o);
    if (opt) {
        if (opt->struct_size != sizeof(fmm_options)) return fail(FMM_E_INVALID, "fmm_options.struct_size mismatch");
        o = *opt;
    }
    if ((int)tiling < 0 || (int)tiling > 2) return fail(FMM_E_INVALID, "bad tiling");
    if (n_src < 0 || n_tgt < 0) return fail(FMM_E_INVALID, "negative point count");
    if (n_src > INT32_MAX / 2 || n_tgt > INT32_MAX / 2) return fail(FMM_E_INVALID, "too many points");
    if ((n_src > 0 && !src) || (n_tgt > 0 && !tgt && tgt != src))
        return fail(FMM_E_INVALID, "null point array");
    if (!(eps > 0.0 && eps < 0.5)) return fail(FMM_E_INVALID, "eps must lie in (0, 0.5)");
    if (o.leaf_size < 1) return fail(FMM_E_INVALID, "leaf_size must be >= 1");
    if (o.p > kMaxP) return fail(FMM_E_INVALID, "p above the supported maximum (60)");
    if (o.lmax > kMaxL) return fail(FMM_E_INVALID, "lmax above the supported maximum (16)");
    if (o.precision < 0 || o.precision > 2) return fail(FMM_E_INVALID, "bad precision");
    if (o.depth_rule != FMM_DEPTH_MEAN && o.depth_rule != FMM_DEPTH_COST) return fail(FMM_E_INVALID, "bad depth_rule");
    if (o.near_stream != 0 && o.near_stream != 1) return fail(FMM_E_INVALID, "bad near_stream");
    PlanImpl *P = new PlanImpl();
    P->device_pointers = o.device_pointers != 0;
    P->n_src = n_src;
    P->n_tgt = n_tgt;
    P->same = (tgt == src) && (n_tgt == n_src);
    P->near_own_stream = o.near_stream == 1;
    P->leaf_size = o.leaf_size;
    // The mixed form holds eps down to 1e-6 (its arithmetic floor is about
    // 2e-8 in relative L2: FP32 pair terms, FP32 accumulation of the split
    // M2L products); a smaller eps takes the FP64 form, also when the mixed
    // form was asked for.
    int prec = o.precision;
    if (prec == FMM_PREC_AUTO || (prec == FMM_PREC_MIXED && !(eps >= kMixedMinEps)))
        prec = eps >= kMixedMinEps ? FMM_PREC_MIXED : FMM_PREC_FP64;
    P->precision = prec;
    hipGetDevice(&P->device);
    if (o.device_pointers) {
        P->stream = (hipStream_t)o.stream;   // NULL: the null stream
    } else {
        const hipError_t e = hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete P;
            return fail(FMM_E_DEVICE, std::string("hipStreamCreate failed: ") + hipGetErrorString(e));
        }
        P->own_stream = true;
    }
    for (auto &ev : P->ev) {
        const hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            release(P);
            delete P;
            return fail(FMM_E_DEVICE, std::string("hipEventCreate failed: ") + hipGetErrorString(e));
        }
    }
    fmm_status st = build_plan(P, (int)tiling, src, n_src, tgt, n_tgt, eps, o);
    if (st != FMM_OK) {
        std::string msg = g_err;
        release(P);
        delete P;
        g_err = msg;
        return st;
    }
    *out = (fmm_plan_t)(Plan *)P;
    return FMM_OK;
}

static fmm_status eval_impl(fmm_plan_t plan, const double *u, double *phi, double *field, bool want_field)
{
    g_err.clear();
    if (!plan) return fail(FMM_E_INVALID, "null plan");
    PlanImpl *P = (PlanImpl *)(Plan *)plan;
    if ((P->n_src > 0 && !u) || (P->n_tgt > 0 && (!phi || (want_field && !field))))
        return fail(FMM_E_INVALID, "null array");
    hipStream_t s = P->stream;
    if (P->n_tgt == 0) return FMM_OK;
    if (want_field && (!P->nfield || (!P->device_pointers && !P->io_field))) {
        int err = 0;
        if (!P->nfield) P->nfield = take<double>(P, 2 * P->n_tgt, &err);
        if (!P->device_pointers && !P->io_field) P->io_field = take<double>(P, 2 * P->n_tgt, &err);
        if (err) return fail(FMM_E_NOMEM, "device allocation failed (field buffers)");
    }
    double *dphi = P->device_pointers ? phi : P->io_phi;
    double *dfield = want_field ? (P->device_pointers ? field : P->io_field) : nullptr;
    const double *du = P->device_pointers ? u : P->io_u;
    if (!P->device_pointers && P->n_src)
        FMM_HIP_CHECK(hipMemcpyAsync(P->io_u, u, sizeof(double) * P->n_src, hipMemcpyHostToDevice, s));
    FMM_HIP_CHECK(hipEventRecord(P->ev[2], s));
    if (P->n_src == 0) {
        FMM_HIP_CHECK(hipMemsetAsync(dphi, 0, sizeof(double) * 2 * P->n_tgt, s));
        if (dfield) FMM_HIP_CHECK(hipMemsetAsync(dfield, 0, sizeof(double) * 2 * P->n_tgt, s));
        FMM_HIP_CHECK(hipEventRecord(P->ev[3], s));
        FMM_HIP_CHECK(hipEventRecord(P->ev[4], s));
        FMM_HIP_CHECK(hipEventRecord(P->ev[5], s));
        FMM_HIP_CHECK(hipEventRecord(P->ev[6], s));
        FMM_HIP_CHECK(hipEventRecord(P->ev[8], s));
        FMM_HIP_CHECK(hipEventRecord(P->ev[9], s));
    } else {
        Plan *one = P;
        run_batch(&one, 1, (const EvalJob *)P->job_dev, dphi, s, P->near_own_stream ? s : side_stream(), &P->ev[3], dfield,
                  dfield ? P->nfield : nullptr, du);
    }
    FMM_HIP_CHECK(hipGetLastError());
    P->evaluated = true;
    if (!P->device_pointers) {
        FMM_HIP_CHECK(hipMemcpyAsync(phi, P->io_phi, sizeof(double) * 2 * P->n_tgt,
                                     hipMemcpyDeviceToHost, s));
        if (dfield)
            FMM_HIP_CHECK(hipMemcpyAsync(field, P->io_field, sizeof(double) * 2 * P->n_tgt,
                                         hipMemcpyDeviceToHost, s));
        FMM_HIP_CHECK(hipStreamSynchronize(s));
    }
    return FMM_OK;
}

fmm_status fmm_eval(fmm_plan_t plan, const double *u, double *phi)
{
    return eval_impl(plan, u, phi, nullptr, false);
}

fmm_status fmm_eval_field(fmm_plan_t plan, const double *u, double *phi, double *field)
{
    return eval_impl(plan, u, phi, field, true);
}

fmm_status fmm_plan_info_get(fmm_plan_t plan, fmm_plan_info *info)
{
    if (!plan || !info) return fail(FMM_E_INVALID, "null argument");
    PlanImpl *P = (PlanImpl *)(Plan *)plan;
    memset(info, 0, sizeof(*info));
    info->tiling = P->geo.tiling;
    info->lmax = P->geo.L;
    info->p = P->p;
    info->precision = P->precision;
    info->geometry[0] = P->geo.ox;
    info->geometry[1] = P->geo.oy;
    info->geometry[2] = P->geo.size;
    info->n_src = P->n_src;
    info->n_tgt = P->n_tgt;
    info->targets_are_sources = P->same;
    info->e4_width = P->tables.e4_width;
    for (int l = 0; l <= P->geo.L && l < 32; ++l) info->n_cells[l] = P->lev[l].n;
    if (P->n_m2l_pairs < 0) {
        int err = 0;
        unsigned long long *pairs = (unsigned long long *)dev_alloc(16, &err);
        unsigned long long hp[2] = {0, 0};
        if (!err) {
            hipMemsetAsync(pairs, 0, 16, P->stream);
            launch_count_pairs(P->lev, P->geo.L, P->tables.e4_width, P->tables.near_width, P->e4,
                               P->near, P->cell_occ, P->sb, P->se, P->tb, P->te, pairs, P->stream);
            hipMemcpyAsync(hp, pairs, 16, hipMemcpyDeviceToHost, P->stream);
            hipStreamSynchronize(P->stream);
            dev_free(pairs, 16);
        }
        P->n_m2l_pairs = (int64_t)hp[0];
        P->n_near_pairs = (int64_t)hp[1];
    }
    if (P->plan_ms == 0 && hipEventSynchronize(P->ev[1]) == hipSuccess) P->plan_ms = elapsed(P->ev[0], P->ev[1]);
    info->n_m2l_pairs = P->n_m2l_pairs;
    info->n_near_pairs = P->n_near_pairs;
    info->device_bytes = P->device_bytes;
    info->plan_ms = P->plan_ms;
    if (P->evaluated && hipEventSynchronize(P->ev[6]) == hipSuccess && P->n_tgt > 0) {
        info->eval_ms = elapsed(P->ev[2], P->ev[6]);
        info->stage_ms[0] = elapsed(P->ev[2], P->ev[3]);
        info->stage_ms[1] = elapsed(P->ev[3], P->ev[4]);
        info->stage_ms[2] = elapsed(P->ev[4], P->ev[5]);
        info->stage_ms[3] = elapsed(P->ev[8], P->ev[9]);
        info->stage_ms[4] = elapsed(P->ev[5], P->ev[6]);
    }
    (void)hipGetLastError();
    return FMM_OK;
}

fmm_status fmm_plan_export_points(fmm_plan_t plan, int64_t *src_keys, int64_t *tgt_keys,
                                  int64_t *src_perm, int64_t *tgt_perm)
{
    if (!plan) return fail(FMM_E_INVALID, "null plan");
    PlanImpl *P = (PlanImpl *)(Plan *)plan;
    FMM_HIP_CHECK(hipStreamSynchronize(P->stream));
    auto one = [&](const uint32_t *dk, const int32_t *dp, int64_t n, int64_t *keys,
                   int64_t *perm) -> fmm_status {
        if (n <= 0) return FMM_OK;
        std::vector<uint32_t> k(n);
        std::vector<int32_t> p(n);
        FMM_HIP_CHECK(hipMemcpy(k.data(), dk, 4 * n, hipMemcpyDeviceToHost));
        FMM_HIP_CHECK(hipMemcpy(p.data(), dp, 4 * n, hipMemcpyDeviceToHost));
        for (int64_t j = 0; j < n; ++j) {
            if (keys) keys[p[j]] = k[j];
            if (perm) perm[j] = p[j];
        }
        return FMM_OK;
    };
    fmm_status st = one(P->skey, P->sperm, P->n_src, src_keys, src_perm);
    if (st) return st;
    return one(P->tkey, P->tperm, P->n_tgt, tgt_keys, tgt_perm);
}

fmm_status fmm_plan_export_level(fmm_plan_t plan, int32_t level, int64_t *keys, int32_t *occupancy,
                                 int64_t *src_range, int64_t *tgt_range, int64_t *e4, int64_t *near)
{
    if (!plan) return fail(FMM_E_INVALID, "null plan");
    PlanImpl *P = (PlanImpl *)(Plan *)plan;
    if (level < 0 || level > P->geo.L) return fail(FMM_E_INVALID, "level out of range");
    FMM_HIP_CHECK(hipStreamSynchronize(P->stream));
    const int64_t n = P->lev[level].n, off = P->lev[level].cell_off, C = P->n_cells;
    if (n == 0) return FMM_OK;
    std::vector<uint32_t> ck(C);
    FMM_HIP_CHECK(hipMemcpy(ck.data(), P->cell_key, 4 * C, hipMemcpyDeviceToHost));
    if (keys)
        for (int64_t i = 0; i < n; ++i) keys[i] = ck[off + i];
    if (occupancy) {
        std::vector<uint8_t> oc(n);
        FMM_HIP_CHECK(hipMemcpy(oc.data(), P->cell_occ + off, n, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i) occupancy[i] = oc[i];
    }
    auto ranges = [&](const int32_t *b, const int32_t *e, int64_t *out) -> fmm_status {
        std::vector<int32_t> hb(n), he(n);
        FMM_HIP_CHECK(hipMemcpy(hb.data(), b + off, 4 * n, hipMemcpyDeviceToHost));
        FMM_HIP_CHECK(hipMemcpy(he.data(), e + off, 4 * n, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i) {
            out[2 * i] = hb[i];
            out[2 * i + 1] = he[i];
        }
        return FMM_OK;
    };
    if (src_range && ranges(P->sb, P->se, src_range)) return FMM_E_DEVICE;
    if (tgt_range && ranges(P->tb, P->te, tgt_range)) return FMM_E_DEVICE;
    auto lists = [&](const int32_t *d, int64_t row0, int w, int64_t *out) -> fmm_status {
        std::vector<int32_t> h(n * w);
        FMM_HIP_CHECK(hipMemcpy(h.data(), d + row0 * w, 4 * n * w, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i) {
            std::vector<int64_t> v;
            for (int k = 0; k < w; ++k)
                if (h[i * w + k] >= 0) v.push_back(ck[h[i * w + k]]);
            std::sort(v.begin(), v.end());
            for (int k = 0; k < w; ++k) out[i * w + k] = k < (int)v.size() ? v[k] : -1;
        }
        return FMM_OK;
    };
    if (e4 && lists(P->e4, off, P->tables.e4_width, e4)) return FMM_E_DEVICE;
    if (near && level == P->geo.L) {
        std::vector<int64_t> tmp(n * P->tables.near_width);
        if (lists(P->near, 0, P->tables.near_width, tmp.data())) return FMM_E_DEVICE;
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < kNearSlots; ++k)
                near[i * kNearSlots + k] = k < P->tables.near_width ? tmp[i * P->tables.near_width + k] : -1;
    }
    return FMM_OK;
}

void fmm_plan_destroy(fmm_plan_t plan)
{
    if (!plan) return;
    PlanImpl *P = (PlanImpl *)(Plan *)plan;
    release(P);
    delete P;
}

const char *fmm_last_error(void) { return g_err.c_str(); }

}  // extern "C"
