// eval.h -- per-plan evaluation descriptors and batched launches.
//
// Every evaluation kernel takes a device array of EvalJob descriptors (one
// per plan) and a BatchMap passed by value that lists, for the phase being
// launched, which jobs take part and where each job's work items start in
// the global item range.  A kernel's workgroups walk that range with a
// fixed-size, grid-stride (persistent) loop, so one launch serves any mix of
// requests; a single fmm_eval is a batch of one.  An item's arithmetic
// depends only on its own job's data, so a result is bitwise the same alone
// and in a batch.
#pragma once

#include "fmm_internal.h"

namespace fmm {

constexpr int kMaxBatch = 64;
constexpr int kBinomStride = 2 * kMaxP + 2;

struct EvalJob {
    int p, L, tiling, base, prec;
    int nw, ew, G, pm, sept;
    int64_t n_src, n_tgt, n_cells, leaf_off, n_leaf, m2l_first;
    double scale[kMaxL + 1];
    int64_t cell_off[kMaxL + 2];
    int64_t dense_off[kMaxL + 1];
    const double *sx, *sy;
    double *su;
    float *suf;
    const float *sxl, *syl, *txl, *tyl;
    const double *tx, *ty;
    const int32_t *sperm, *tperm;
    const int32_t *sb, *se, *tb, *te, *dense, *parent, *e4, *near, *work_near;
    const uint32_t *cell_key;
    const uint8_t *occ, *group;
    const double *cx, *cy;
    double *mp, *lc;
    const double *m2l_pw, *m2l_lg, *m2l_a0, *binom;
    // M2L tiles of up to 16 target cells of one (level, group) {key, first
    // list position, count, 0}, their launch order, and the list of the cells
    const int32_t *mix_tiles, *mix_order, *mix_list;
    // Device counts written at plan time: [0] near-field items, [1] M2L
    // tiles.  Launches are sized by host upper bounds; kernels stop here.
    const int32_t *counts;
    double *phi;    // output, caller's target order, 2 n_tgt doubles
    double *nsum;   // near-field sums, sorted target order, 2 n_tgt doubles
    // Second-side near sums of the symmetric near field (targets = sources,
    // mixed): one FP32 (re, im) per (point, lower neighbour, its chunk), at
    // [((near slot - 1) * kSymChunks + chunk) * n_tgt + point]; null when
    // the plan cannot take that path.
    float2 *bside;
    double2 *bside64;   // the same for the FP64 symmetric near field
};

struct BatchMap {
    int n;                        // participating entries
    int64_t pre[kMaxBatch + 1];   // item prefix per entry
    int16_t job[kMaxBatch];       // job index of each entry
    int8_t aux[kMaxBatch];        // phase argument (level) of each entry
    double *phi_override;         // single-job output redirect (or null)
    double *field_override;       // single-job field output, caller's order (or null: no field)
    double *nfield;               // single-job near-field sums of the field, sorted order
    const double *u_in;           // single-job strengths in the caller's order: P2M gathers them
};

__device__ __forceinline__ int batch_entry(const BatchMap &m, int64_t item)
{
    int e = 0;
    while (e + 1 < m.n && item >= m.pre[e + 1]) ++e;
    return e;
}

__device__ __forceinline__ int level_of(const EvalJob &J, int64_t gid)
{
    int l = 0;
    while (l < J.L && gid >= J.cell_off[l + 1]) ++l;
    return l;
}

// The near field runs beside the far-field passes as a persistent grid of
// one-wave blocks (up to 32 per SIMD, so effectively one per work item).
constexpr int kNearWavesPerCU = 128;

// Persistent-grid size for a phase with `items` work items.
// The far-field passes (M2M, M2L, L2L) form a chain of small, latency-bound
// launches that share the SIMDs with the long-running near-field waves on
// the side stream.  Their waves raise their issue priority so the chain is
// not slowed to the near field's share of each SIMD; the near field fills
// the remaining issue slots.
__device__ __forceinline__ void far_field_priority() { __builtin_amdgcn_s_setprio(2); }

// A value that is the same in every lane, moved to a scalar register.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// A load through a pointer known to address global memory: the compiler
// then waits for it by count (flat loads are waited for all at once).
template <typename T>
__device__ __forceinline__ T gload(const T *p, int64_t i)
{
    return ((const __attribute__((address_space(1))) T *)p)[i];
}

// How a neighbour cell's pairs are taken by the symmetric near field.
enum : int8_t { kCellSkip = 0, kCellOne = 1, kCellSym = 2 };

inline unsigned persistent_grid(int64_t items, int per_cu)
{
    int64_t cap = (int64_t)256 * per_cu;
    return (unsigned)(items < cap ? (items > 0 ? items : 1) : cap);
}

// Launchers (items are counted on the host from plan sizes, or bounded
// there when only the device knows the count).
void batch_gather_u(const EvalJob *jobs_d, const EvalJob &J, const double *u, hipStream_t s);
void batch_p2m(const EvalJob *jobs, const BatchMap &m, int pmax, hipStream_t s);
void batch_m2m(const EvalJob *jobs, const BatchMap &m, hipStream_t s);
void batch_l2l(const EvalJob *jobs, const BatchMap &m, hipStream_t s);
void batch_m2m_lanes(const EvalJob *jobs, const BatchMap &m, int pm, int gs, hipStream_t s);
void batch_l2l_lanes(const EvalJob *jobs, const BatchMap &m, int pm, hipStream_t s);
void batch_m2l_block(const EvalJob *jobs, const BatchMap &m, hipStream_t s);
void batch_m2l_lanes(const EvalJob *jobs, const BatchMap &m, int pm, hipStream_t s);
// FP64 M2L on MFMA; every job of the batch has kernel class m2l_f64_mfma_class(p).
void batch_m2l_f64_mfma(const EvalJob *jobs, const BatchMap &m, int p, hipStream_t s);
// Mixed M2L, factored BF16x3 on MFMA; every job has class m2l_bf16x3f_class(p).
void batch_m2l_bf16x3f(const EvalJob *jobs, const BatchMap &m, int p, hipStream_t s);
int m2l_bf16x3f_class(int p);
void batch_near_fp64(const EvalJob *jobs, const BatchMap &m, hipStream_t s);
void batch_l2p(const EvalJob *jobs, const BatchMap &m, hipStream_t s);
void batch_near_mixed(const EvalJob *jobs, const BatchMap &m, hipStream_t s);
void batch_near_mixed_sym(const EvalJob *jobs, const BatchMap &m, hipStream_t s);
void batch_near_fp64_sym(const EvalJob *jobs, const BatchMap &m, hipStream_t s);

// Host view of one plan for batching: its descriptor (host copy) and the
// device copy.
EvalJob make_job(const Plan &P);

// Run the evaluation phases for a batch of plans on stream s.  jobs_dev
// holds the descriptors in device memory (jobs_dev[i] describes plans[i]).
// phi_single, when not null and the batch has one plan, receives the output
// instead of the plan's own buffer.
// Evaluates a batch of plans on stream s.  ev[0..3]: ends of the upward
// pass, M2L, L2L and the whole evaluation (recorded on s); ev[4]: fork to
// the side stream, ev[5..6]: start and end of the P2P near field there.
hipStream_t side_stream();   // per-device stream for the near field
// field_single / nfield_single (a batch of one only): also evaluate the
// field Phi' into field_single, with nfield_single (2 n_tgt doubles) for the
// near-field part.
// u_single (a batch of one only): the strengths in the caller's order,
// gathered by P2M; otherwise the jobs' sorted strengths are already filled.
void run_batch(Plan *const *plans, int n, const EvalJob *jobs_dev, double *phi_single, hipStream_t s,
               hipStream_t side, hipEvent_t *ev, double *field_single = nullptr,
               double *nfield_single = nullptr, const double *u_single = nullptr);

}  // namespace fmm
