// fmm_internal.h -- shared declarations of the gfx950 FMM library.
//
// Data layout in device memory (one plan):
//   sorted points   SoA: x[], y[] (FP64), key[] (u32 leaf key), perm[] (i32
//                   original index), plus FP32 leaf-local copies for the
//                   mixed-precision near field;
//   cells           one global id space over all levels (level offsets),
//                   each level's occupied cells in ascending key order;
//                   per cell: key, source range, target range, centre,
//                   M2L slots (source cell ids, -1 = empty) and, at the
//                   leaf level, near-field slots;
//   dense maps      per level, key -> global cell id (or -1), concatenated;
//   expansions      multipole / local coefficients, one row of 2(p+1)
//                   doubles (re, im interleaved) per cell, radius-scaled.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fmm2d.h"

namespace fmm {

constexpr int kMaxL = 16;         // deepest leaf level supported (u32 keys)
constexpr int kMaxP = 60;         // highest expansion order
constexpr int kMaxSlots = 42;     // largest E4 list (septree)
constexpr int kNearSlots = 13;    // largest closed neighbourhood (triangles)
constexpr int kMaxGroups = 8;     // M2L target groups (triangle: 4 types x 2)
constexpr double kMixedMinEps = 1e-6;   // smallest eps the mixed form is used for
constexpr int kChunk = 64;        // targets per near-field work item (at most)
// A leaf with at most this many chunks of kChunk targets evaluates the pairs
// with its higher-indexed neighbours for both sides (mixed, targets = sources).
constexpr int kSymChunks = 2;
// The FP64 symmetric near-field kernel takes a leaf of at most kWide targets
// as one item (up to kWide / 8 blocks of eight rows), so a leaf just above
// kChunk points is not split into a full and a nearly empty item; the mixed
// one splits every leaf into chunks of kChunk.
constexpr int kWide = 96;
// Items of the FP64 symmetric kernel with at most this many targets use
// target blocks of four rows and sixteen sources per round (else eight and
// eight).
constexpr int kSmall = 48;
// Chunks of a leaf with n targets in a symmetric kernel whose single items
// hold up to `wide` targets (kWide for FP64, kChunk for mixed): one up to
// `wide`, else ceil(n / kChunk).  Its second-side sums take one slot per chunk.
__host__ __device__ inline int sym_chunks(int n, int wide)
{
    return n <= wide ? 1 : (n + kChunk - 1) / kChunk;
}

enum Tiling { kQuad = 0, kSept = 1, kTri = 2 };

// Geometry and key-assignment constants, passed by value to kernels.
struct GeoParams {
    int tiling;
    int L;
    double ox, oy;
    double size;   // quad: root side; sept/tri: leaf circumradius r
    double s3;     // sqrt(3) as computed on the host
};

// Per-tiling interaction tables (built on the host, read by the list
// kernels).  Offsets are in integer units of the level:
//   quad  (dx, dy) cells;  sept (a, b) Eisenstein a + b w;
//   tri   (dU, dV) in units of the level circumradius (x = U sqrt3/2, y = V/2).
struct ListTables {
    int n_groups;
    int e4_width;                       // 27 / 42 / 39
    int near_width;                     // 9 / 7 / 13 (cell included, slot 0)
    int e4[kMaxGroups][kMaxSlots][2];
    int e4_count[kMaxGroups];
    int near[2][kNearSlots][2];         // [orientation index][slot]
    int near_count[2];
};

struct LevelInfo {
    int64_t K;          // dense key space base^l
    int64_t dense_off;  // offset of this level in the dense map
    int64_t cell_off;   // first global cell id of this level
    int64_t n;          // occupied cells
};

// Arena of device memory with a caching pool behind it.
void *dev_alloc(size_t bytes, int *err, std::vector<uint64_t> *waited = nullptr,
                hipStream_t stream = nullptr);
void dev_free(void *p, size_t bytes);

struct Plan {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool device_pointers = false;
    GeoParams geo{};
    int p = 0;
    int precision = FMM_PREC_FP64;
    int leaf_size = 64;
    int64_t n_src = 0, n_tgt = 0;
    bool same = false;   // targets are the sources
    bool near_own_stream = false;   // evaluation: near field on the plan's stream
    double scale[kMaxL + 1]{};   // radius scale of each level

    // arena
    char *arena = nullptr;
    size_t arena_bytes = 0;

    // sorted points
    double *sx = nullptr, *sy = nullptr;
    uint32_t *skey = nullptr;
    int32_t *sperm = nullptr;
    double *tx = nullptr, *ty = nullptr;
    uint32_t *tkey = nullptr;
    int32_t *tperm = nullptr;
    float *sxl = nullptr, *syl = nullptr;   // leaf-local FP32 coordinates
    float *txl = nullptr, *tyl = nullptr;
    double *su = nullptr;                   // strengths in sorted order
    float *suf = nullptr;
    // mixed precision with targets = sources: the symmetric near field's
    // second-side sums, [(near slot - 1) * kSymChunks + chunk][point]
    float2 *bside = nullptr;
    double2 *bside64 = nullptr;   // FP64 plans with targets = sources: the same in FP64

    // cells
    LevelInfo lev[kMaxL + 1]{};
    int64_t n_cells = 0;
    int64_t dense_total = 0;
    int32_t *dense = nullptr;      // dense key -> global id
    uint32_t *cell_key = nullptr;
    uint8_t *cell_occ = nullptr;   // bit0 sources, bit1 targets
    int32_t *sb = nullptr, *se = nullptr, *tb = nullptr, *te = nullptr;
    double *cx = nullptr, *cy = nullptr;
    int32_t *parent = nullptr;     // global id of the parent cell (-1 at root)
    uint8_t *group = nullptr;      // M2L group of each cell
    ListTables tables{};
    int32_t *e4 = nullptr;         // [n_cells][e4_width]
    int32_t *near = nullptr;       // [n_leaf][near_width]
    int32_t *work_near = nullptr;  // near-field items: (leaf id, start)
    int64_t n_work_near = 0;        // upper bound of near-field items
    int32_t *counts = nullptr;      // device: [0] near items, [1] mixed M2L tiles
    int64_t n_m2l_pairs = 0, n_near_pairs = 0;

    // expansions
    double *mp = nullptr, *lc = nullptr;
    const double *binom = nullptr; // C(n, k), n, k <= 2 kMaxP + 1 (per device)

    // M2L offset tables (lane kernel): (-1/delta)^k and Log(c_T - c_S)
    double *m2l_pw = nullptr, *m2l_lg = nullptr, *m2l_a0 = nullptr;
    int m2l_pm = 0;

    // mixed precision M2L operands
    void *mixed = nullptr;
    int mixed_tiles = 0;

    // timing
    hipEvent_t ev[12]{};
    double plan_ms = 0, eval_ms = 0, stage_ms[8]{};
    bool evaluated = false;

    // evaluation descriptor (device copy) and the output buffer used by
    // batched evaluation (caller's target order)
    void *job_dev = nullptr;
    double *phi_int = nullptr;
    double *nsum = nullptr;         // near-field sums in sorted target order

    // scratch for staging host inputs / outputs
    double *io_u = nullptr;
    double *io_phi = nullptr;
    int32_t *scratch_i32 = nullptr;
    size_t scratch_bytes = 0;
};

// ------------------------------------------------------------------ kernels
// keys.hip
void launch_bbox(const double *pts, int64_t n, double *partial, int nblocks, hipStream_t s);
// Also sets *zero (if not null) to 0.
void launch_bbox_final(const double *partial, int nparts, double *out4, int32_t *zero, hipStream_t s);
// Depth statistics: occupancy histogram of every stride-th point's key at a
// trial leaf level; per coarser level, sum over cells of sources x targets
// and the occupied-cell counts (out[0..2], accumulated); a short device copy.
void launch_depth_hist(const GeoParams &g, const double *pts, int64_t n, int64_t stride, uint32_t *hist,
                       hipStream_t s);
void launch_depth_stats(const uint32_t *hs, const uint32_t *ht, int64_t ncells0, int base, int nl,
                        unsigned long long *out, hipStream_t s);
void launch_copy_u64(const unsigned long long *a, int n, unsigned long long *b, hipStream_t s);
// Also clears zero[0 .. n_zero).
void launch_keys(const GeoParams &g, const double *pts, int64_t n, uint32_t *key, int32_t *idx,
                 int32_t *bad_count, int32_t *zero, int64_t n_zero, hipStream_t s);
void launch_gather_points(const double *pts, const int32_t *perm, int64_t n, double *x, double *y,
                          hipStream_t s);

// sort.hip
size_t scan_tmp_bytes(int64_t n);
void scan_exclusive(const int32_t *in, int32_t *out, int64_t n, int32_t *total, void *tmp,
                    hipStream_t s);
size_t radix_tmp_bytes(int64_t n);
void radix_sort(uint32_t *keys, int32_t *vals, int64_t n, int bits, void *tmp, hipStream_t s);

// tree.hip
void launch_mark_cells(const GeoParams &g, const LevelInfo *lev, const uint32_t *key, int64_t n,
                       uint8_t bit, int32_t *flags, hipStream_t s);
void launch_flags_to_ids(int32_t *flags, int64_t n, hipStream_t s);
void launch_compact(const GeoParams &g, const LevelInfo *lev, int64_t dense_total,
                    const int32_t *flags, const int32_t *ids, int32_t *dense, uint32_t *cell_key,
                    uint8_t *occ, int32_t *sb, int32_t *se, int32_t *tb, int32_t *te, double *zero,
                    int n_zero, hipStream_t s);   // also clears zero[0 .. n_zero)
void launch_gather_bounds(const LevelInfo *lev, int L, const int32_t *ids, const int32_t *total,
                          const int32_t *bad, int32_t *out, hipStream_t s);
void launch_cell_ranges(const GeoParams &g, const LevelInfo *lev, const uint32_t *key, int64_t n,
                        const int32_t *dense, int32_t *b, int32_t *e, hipStream_t s);
void launch_cell_geometry(const GeoParams &g, const LevelInfo *lev, int64_t n_cells,
                          const uint32_t *cell_key, const int32_t *dense, const int32_t *sb,
                          const int32_t *se, const int32_t *tb, const int32_t *te, double *cx,
                          double *cy, int32_t *parent, uint8_t *group, uint8_t *occ,
                          hipStream_t s);
void launch_lists(const GeoParams &g, const LevelInfo *lev, const ListTables &tab, int64_t n_cells,
                  const uint32_t *cell_key, const uint8_t *group, const uint8_t *occ,
                  const int32_t *dense, int32_t *e4, int32_t *near, hipStream_t s);
void launch_local_coords(const double *x, const double *y, const uint32_t *key, int64_t n,
                         const GeoParams &g, const LevelInfo *lev, const int32_t *dense,
                         const double *cx, const double *cy, float *xl, float *yl, hipStream_t s);
void launch_near_items(const LevelInfo *lev, int L, const int32_t *tb, const int32_t *te,
                       int32_t *counts, hipStream_t s);
// Items reordered by decreasing estimated cost into out (2 cap ints); keys,
// vals (cap each) and tmp (radix_tmp_bytes(cap)) are scratch.  `wide`: a
// leaf of at most that many targets is one item; `small`: items of at most
// that many targets use the four-row tile (0 = none).
void launch_near_items_order(int64_t leaf_off, int nw, int wide, int small, int32_t cap, const int32_t *count,
                             const int32_t *items, const int32_t *tb, const int32_t *te, const int32_t *near,
                             const int32_t *sb, const int32_t *se, uint32_t *keys, int32_t *vals, void *tmp,
                             int32_t *out, hipStream_t s);
void launch_near_items_fill(const LevelInfo *lev, int L, const int32_t *tb, const int32_t *te,
                            const int32_t *offs, int32_t *items, hipStream_t s);
void launch_count_pairs(const LevelInfo *lev, int L, int e4w, int nw, const int32_t *e4,
                        const int32_t *near, const uint8_t *occ, const int32_t *sb,
                        const int32_t *se, const int32_t *tb, const int32_t *te,
                        unsigned long long *out2, hipStream_t s);
ListTables build_tables(int tiling);

// expand.hip
const double *device_binom(int *err);

// m2l.hip
int m2l_pm_for(int p);
// FP64 M2L on MFMA: kernel class of order p (0 = not supported).
int m2l_f64_mfma_class(int p);
// The mixed form's M2L runs as BF16x3 products on MFMA when the order needs
// more than one 16-row output tile (16 <= p <= 47); at lower orders the FP64
// MFMA kernel (2 ceil(p/4) FP64 MFMAs per pair and row tile) finishes before
// the BF16x3 kernel has split its operands, so the mixed form uses it too.
inline bool m2l_bf16x3_form(const Plan &P) { return P.precision == FMM_PREC_MIXED && P.p >= 16 && P.p <= 47; }
size_t m2l_table_doubles(const Plan &P, int pm);
void launch_m2l_tables(Plan &P, int pm, double *base, hipStream_t s);

// m2l_mixed.hip
size_t mixed_bytes(const Plan &P);
int64_t plan_device_bytes(const Plan *P);
// Device bytes a plan of these sizes may take (admission estimate).
int64_t plan_bytes_estimate(int tiling, int64_t n_src, int64_t n_tgt, bool same, double eps, int precision,
                            int leaf_size);
// Direct sum: slices of the sources per target block (direct_slices), with
// partial sums in part (slices * n_tgt complex128; unused for one slice).
int direct_slices(int64_t n_src, int64_t n_tgt);
// FP64 pair-evaluation rate of k_pair_rate (evaluations per second); nonzero on failure.
int probe_pair_rate(int rounds, int blocks, double *evals_per_s);
void launch_direct(const double *src, int64_t n_src, const double *tgt, int64_t n_tgt, const double *u,
                   double *phi, double *part, int slices, hipStream_t s);
int mixed_setup(Plan &P);

// errors
void set_error(const std::string &msg);

#define FMM_HIP_CHECK(expr)                                                             \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess) {                                                         \
            ::fmm::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));      \
            return FMM_E_DEVICE;                                                        \
        }                                                                               \
    } while (0)

__host__ __device__ inline int base_of(int tiling) { return tiling == kSept ? 7 : 4; }

}  // namespace fmm
