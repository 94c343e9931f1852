// eval.hip -- evaluation phases over a batch of plans.
//
// Phase order (Greengard-Rokhlin sweep; paper Sec. 2 cites it):
//   P2M at the leaves, M2M from level L-1 up to 1, M2L on every level >= 1
//   (the E4 lists), L2L from level 2 down to L, then L2P per target leaf.
//   The P2P near field depends on none of these and runs on a side stream
//   once P2M is done; L2P waits for it and adds the far field to its sums.
//   Strengths are gathered into sorted order by P2M (a single plan) or by
//   the caller (a batch).
// Each phase is one launch (per kernel variant) covering every plan of the
// batch that has work in it; level-wise phases pair plans by their distance
// from the leaves (M2M) or from the top (L2L), so plans of different depth
// share launches.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "eval.h"

namespace fmm {

void tile_pointers(const Plan &P, const int32_t **tiles, const int32_t **order, const int32_t **list);

EvalJob make_job(const Plan &P)
{
    EvalJob J;
    memset(&J, 0, sizeof(J));
    J.p = P.p;
    J.L = P.geo.L;
    J.tiling = P.geo.tiling;
    J.base = base_of(P.geo.tiling);
    J.prec = P.precision;
    J.nw = P.tables.near_width;
    J.ew = P.tables.e4_width;
    J.G = P.tables.n_groups;
    J.pm = P.m2l_pm;
    J.sept = P.geo.tiling == kSept;
    J.n_src = P.n_src;
    J.n_tgt = P.n_tgt;
    J.n_cells = P.n_cells;
    J.leaf_off = P.lev[P.geo.L].cell_off;
    J.n_leaf = P.lev[P.geo.L].n;
    J.m2l_first = P.geo.L >= 1 ? P.lev[1].cell_off : P.n_cells;
    for (int l = 0; l <= kMaxL; ++l) {
        J.scale[l] = l <= P.geo.L ? P.scale[l] : 0.0;
        J.dense_off[l] = l <= P.geo.L ? P.lev[l].dense_off : 0;
    }
    for (int l = 0; l < kMaxL + 2; ++l) J.cell_off[l] = P.n_cells;
    for (int l = 0; l <= P.geo.L; ++l) J.cell_off[l] = P.lev[l].cell_off;
    J.sx = P.sx;
    J.sy = P.sy;
    J.su = P.su;
    J.suf = P.suf;
    J.sxl = P.sxl;
    J.syl = P.syl;
    J.txl = P.txl;
    J.tyl = P.tyl;
    J.tx = P.tx;
    J.ty = P.ty;
    J.sperm = P.sperm;
    J.tperm = P.tperm;
    J.sb = P.sb;
    J.se = P.se;
    J.tb = P.tb;
    J.te = P.te;
    J.dense = P.dense;
    J.parent = P.parent;
    J.e4 = P.e4;
    J.near = P.near;
    J.work_near = P.work_near;
    J.cell_key = P.cell_key;
    J.occ = P.cell_occ;
    J.group = P.group;
    J.cx = P.cx;
    J.cy = P.cy;
    J.mp = P.mp;
    J.lc = P.lc;
    J.counts = P.counts;
    J.m2l_pw = P.m2l_pw;
    J.m2l_lg = P.m2l_lg;
    J.m2l_a0 = P.m2l_a0;
    J.binom = P.binom;
    J.phi = P.phi_int;
    J.nsum = P.nsum;
    J.bside = P.bside;
    J.bside64 = P.bside64;
    if (P.mixed) tile_pointers(P, &J.mix_tiles, &J.mix_order, &J.mix_list);
    return J;
}

namespace {

// Collects (job, aux, items) entries and launches when 64 are pending.
struct Launcher {
    const EvalJob *jobs;
    hipStream_t s;
    double *phi_single;
    double *field_single, *nfield_single;
    BatchMap m;
    template <typename F>
    void add(int job, int aux, int64_t items, F &&flush)
    {
        if (items <= 0) return;
        if (m.n == kMaxBatch) {
            flush(m);
            reset();
        }
        m.job[m.n] = (int16_t)job;
        m.aux[m.n] = (int8_t)aux;
        m.pre[m.n + 1] = m.pre[m.n] + items;
        m.n++;
    }
    void reset()
    {
        m.n = 0;
        m.pre[0] = 0;
        m.phi_override = phi_single;
        m.field_override = field_single;
        m.nfield = nfield_single;
        m.u_in = nullptr;
    }
};

}  // namespace

hipStream_t side_stream()
{
    static std::mutex mu;
    static hipStream_t ss[64] = {};
    int dev = 0;
    hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    if (dev < 0 || dev >= 64) return nullptr;
    if (!ss[dev] && hipStreamCreateWithFlags(&ss[dev], hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        ss[dev] = nullptr;
    }
    return ss[dev];
}

void run_batch(Plan *const *plans, int n, const EvalJob *jobs_dev, double *phi_single, hipStream_t s,
               hipStream_t side, hipEvent_t *ev, double *field_single, double *nfield_single,
               const double *u_single)
{
    if (n != 1 || !nfield_single) field_single = nfield_single = nullptr;
    if (!field_single) nfield_single = nullptr;
    Launcher Lc{jobs_dev, s, n == 1 ? phi_single : nullptr, field_single, nfield_single, {}};
    Lc.reset();
    auto go = [&](auto &&launch) {
        if (Lc.m.n > 0) launch(Lc.m);
        Lc.reset();
    };
    int maxL = 0;
    for (int i = 0; i < n; ++i) maxL = std::max(maxL, plans[i]->geo.L);

    int pmax = 1;
    for (int i = 0; i < n; ++i) pmax = std::max(pmax, plans[i]->p);
    // P2M (gathers the strengths of a single plan on the way)
    {
        auto f = [&](const BatchMap &m) {
            BatchMap mu = m;
            mu.u_in = n == 1 ? u_single : nullptr;
            batch_p2m(jobs_dev, mu, pmax, s);
        };
        for (int i = 0; i < n; ++i) Lc.add(i, 0, plans[i]->lev[plans[i]->geo.L].n, f);
        go(f);
    }
    // The P2P near field needs only the sorted sources and the lists: it runs
    // on the side stream beside the far-field passes after P2M (which runs
    // alone, at full occupancy); L2P joins them.
    {
        hipEventRecord(ev[4], s);
        hipStreamWaitEvent(side, ev[4], 0);
        hipEventRecord(ev[5], side);
        {
            Launcher Ls{jobs_dev, side, n == 1 ? phi_single : nullptr, field_single, nfield_single, {}};
            Ls.reset();
            // FP64: the symmetric form where the targets are the sources
            // (not for the field)
            auto sym64 = [&](const Plan &P) { return P.bside64 != nullptr && nfield_single == nullptr; };
            auto fs = [&](const BatchMap &m) { batch_near_fp64_sym(jobs_dev, m, side); };
            for (int i = 0; i < n; ++i)
                if (plans[i]->precision != FMM_PREC_MIXED && sym64(*plans[i])) Ls.add(i, 0, plans[i]->n_work_near, fs);
            if (Ls.m.n > 0) fs(Ls.m);
            Ls.reset();
            auto f = [&](const BatchMap &m) { batch_near_fp64(jobs_dev, m, side); };
            for (int i = 0; i < n; ++i)
                if (plans[i]->precision != FMM_PREC_MIXED && !sym64(*plans[i])) Ls.add(i, 0, plans[i]->n_work_near, f);
            if (Ls.m.n > 0) f(Ls.m);
            Ls.reset();
            // mixed: the symmetric form where the targets are the sources
            // (not for the field, which L2P then reads without second sides)
            auto sym = [&](const Plan &P) { return P.bside != nullptr && nfield_single == nullptr; };
            auto gs = [&](const BatchMap &m) { batch_near_mixed_sym(jobs_dev, m, side); };
            for (int i = 0; i < n; ++i)
                if (plans[i]->precision == FMM_PREC_MIXED && sym(*plans[i])) Ls.add(i, 0, plans[i]->n_work_near, gs);
            if (Ls.m.n > 0) gs(Ls.m);
            Ls.reset();
            auto g = [&](const BatchMap &m) { batch_near_mixed(jobs_dev, m, side); };
            for (int i = 0; i < n; ++i)
                if (plans[i]->precision == FMM_PREC_MIXED && !sym(*plans[i])) Ls.add(i, 0, plans[i]->n_work_near, g);
            if (Ls.m.n > 0) g(Ls.m);
        }
        hipEventRecord(ev[6], side);
    }

    // Translation kernel variants: M2M and L2L take the block form (a wave
    // per cell, a lane per coefficient: few registers, so its waves find
    // room beside the near field's) for the base-4 tilings and for orders
    // above 48; the septree's seven children per parent take the lane form
    // (a lane per parent-child pair, coefficients in registers).
    const int pms[] = {0, 8, 16, 24, 32, 40, 48};
    auto shift_pm = [](const Plan &P) { return base_of(P.geo.tiling) == 4 ? 0 : P.m2l_pm; };
    // M2M, step k: level L_i - 1 - k; lane groups of 4 (base 4) or 8 (base 7).
    for (int k = 0; k < maxL; ++k)
        for (int pm : pms)
            for (int gs : {4, 8}) {
                if (pm == 0 && gs == 8) continue;
                auto f = [&](const BatchMap &m) {
                    if (pm == 0) batch_m2m(jobs_dev, m, s);
                    else batch_m2m_lanes(jobs_dev, m, pm, gs, s);
                };
                for (int i = 0; i < n; ++i) {
                    const Plan &P = *plans[i];
                    const int l = P.geo.L - 1 - k;
                    if (l < 1 || shift_pm(P) != pm || (pm && (base_of(P.geo.tiling) > 4 ? 8 : 4) != gs)) continue;
                    Lc.add(i, l, P.lev[l].n, f);
                }
                go(f);
            }
    hipEventRecord(ev[0], s);

    // M2L, one launch per kernel variant present in the batch.
    {
        for (int pm : pms) {
            if (pm == 0) continue;
            auto f = [&](const BatchMap &m) { batch_m2l_lanes(jobs_dev, m, pm, s); };
            for (int i = 0; i < n; ++i) {
                const Plan &P = *plans[i];
                const bool tiled = P.mixed_tiles > 0;   // mixed or FP64 MFMA form
                if (P.geo.L < 1 || P.m2l_pm != pm || tiled) continue;
                const int64_t cells = P.n_cells - P.lev[1].cell_off;
                Lc.add(i, 0, (cells + 63) / 64, f);
            }
            go(f);
        }
        // FP64 on MFMA, then BF16x3 on MFMA; one launch per kernel class
        // present
        for (int bf = 0; bf < 2; ++bf) {
            auto cls_of = [&](const Plan &P) {
                if (P.mixed_tiles == 0) return 0;
                if (m2l_bf16x3_form(P) != (bf == 1)) return 0;
                return bf ? m2l_bf16x3f_class(P.p) : m2l_f64_mfma_class(P.p);
            };
            std::vector<int> done;
            for (int i = 0; i < n; ++i) {
                const Plan &Pi = *plans[i];
                const int cls = cls_of(Pi);
                if (cls == 0 || std::find(done.begin(), done.end(), cls) != done.end()) continue;
                done.push_back(cls);
                auto f = [&](const BatchMap &m) {
                    if (bf) batch_m2l_bf16x3f(jobs_dev, m, Pi.p, s);
                    else batch_m2l_f64_mfma(jobs_dev, m, Pi.p, s);
                };
                for (int k = i; k < n; ++k)
                    if (cls_of(*plans[k]) == cls) Lc.add(k, 0, plans[k]->mixed_tiles, f);
                go(f);
            }
        }
        auto fb = [&](const BatchMap &m) { batch_m2l_block(jobs_dev, m, s); };
        for (int i = 0; i < n; ++i) {
            const Plan &P = *plans[i];
            if (P.geo.L < 1 || P.m2l_pm != 0) continue;
            Lc.add(i, 0, P.n_cells - P.lev[1].cell_off, fb);
        }
        go(fb);
    }
    hipEventRecord(ev[1], s);

    // L2L, step k: level 2 + k; for the base-4 tilings up to the level above
    // the leaves (L2P shifts the leaves' parents' expansions itself).
    for (int l = 2; l <= maxL; ++l)
        for (int pm : pms) {
            auto f = [&](const BatchMap &m) {
                if (pm == 0) batch_l2l(jobs_dev, m, s);
                else batch_l2l_lanes(jobs_dev, m, pm, s);
            };
            for (int i = 0; i < n; ++i)
                if ((plans[i]->geo.L > l || (plans[i]->geo.L == l && base_of(plans[i]->geo.tiling) != 4)) &&
                    shift_pm(*plans[i]) == pm)
                    Lc.add(i, l, plans[i]->lev[l].n, f);
            go(f);
        }
    hipEventRecord(ev[2], s);

    // L2P, after the near field.
    hipStreamWaitEvent(s, ev[6], 0);
    {
        auto f = [&](const BatchMap &m) { batch_l2p(jobs_dev, m, s); };
        for (int i = 0; i < n; ++i) Lc.add(i, 0, plans[i]->n_work_near, f);
        go(f);
    }
    hipEventRecord(ev[3], s);
}

}  // namespace fmm
