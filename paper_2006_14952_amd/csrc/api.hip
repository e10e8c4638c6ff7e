// C ABI of the solver: argument checks, stage orchestration, statistics.
#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "mlp.h"
#include "state.h"

namespace hfmm {
const char *last_error();
void clear_error();
int pm_forces(const fmm_params *P, int mesh, int64_t n, const double *pos, const double *mass, double *acc,
              hipStream_t st);
int add_into(double *acc, const double *other, int64_t n3, hipStream_t st);
int pm_forces_tree(const fmm_params *P, int mesh, fmm_tree *t, double *acc, hipStream_t st);
const MacModel *current_model(MacModel *host_copy);
uint64_t model_serial();
int run_labels(fmm_tree *t, const fmm_params *P, const double *aref_sorted, double eps, int stride, float *feats,
               int *labels, float *errs, uint64_t *pairs, int cap, int *dcounter, hipStream_t st);
int sort_soa(fmm_tree *t, const double *acc, double *out, hipStream_t st);
int p2p_setup(const fmm_params *P, P2PConst &k);
}  // namespace hfmm

using namespace hfmm;

static int check_params(const fmm_params *P)
{
    if (!P) return set_error(FMM_ERR_ARG, "params is NULL");
    if (!(P->box > 0) || !isfinite(P->box)) return set_error(FMM_ERR_ARG, "box must be > 0");
    if (!(P->r_s > 0) || !isfinite(P->r_s)) return set_error(FMM_ERR_ARG, "r_s must be > 0");
    if (!(P->r_cut > 0) || !(P->r_cut < 0.5 * P->box)) return set_error(FMM_ERR_ARG, "need 0 < r_cut < box/2");
    if (!(P->theta > 0) || !isfinite(P->theta)) return set_error(FMM_ERR_ARG, "theta must be > 0");
    if (!isfinite(P->G)) return set_error(FMM_ERR_ARG, "G must be finite");
    if (P->p < 0 || P->p > FMM_PMAX) return set_error(FMM_ERR_ARG, "p must be in [0, %d]", FMM_PMAX);
    if (P->n_crit < 1) return set_error(FMM_ERR_ARG, "n_crit must be >= 1");
    if (P->mac_mode < 0 || P->mac_mode > 7) return set_error(FMM_ERR_ARG, "mac_mode must be in [0, 7]");
    if (P->precision != 0 && P->precision != 1) return set_error(FMM_ERR_ARG, "precision must be 0 or 1");
    if (P->learned != 0 && P->learned != 1) return set_error(FMM_ERR_ARG, "learned must be 0 or 1");
    if (P->split != 0 && P->split != 1) return set_error(FMM_ERR_ARG, "split must be 0 or 1");
    if (P->learned && P->split) return set_error(FMM_ERR_ARG, "the learned selector requires split 0");
    if (P->pm_assign != 0 && (P->pm_assign < 2 || P->pm_assign > 4))
        return set_error(FMM_ERR_ARG, "pm_assign must be 0, 2 (CIC), 3 (TSC) or 4 (PCS)");
    if (P->m2l_mfma < 0 || P->m2l_mfma > 2) return set_error(FMM_ERR_ARG, "m2l_mfma must be 0, 1 or 2");
    if (P->schedule < 0 || P->schedule > 3) return set_error(FMM_ERR_ARG, "schedule must be 0, 1, 2 or 3");
    if (P->deterministic != 0 && P->deterministic != 1) return set_error(FMM_ERR_ARG, "deterministic must be 0 or 1");
    if (P->deterministic && P->schedule == 2)
        return set_error(FMM_ERR_ARG, "deterministic mode has no persistent P2P + M2L kernel (schedule 2)");
    if (P->deterministic && P->m2l_mfma == 2)
        return set_error(FMM_ERR_ARG, "deterministic mode has no matrix-core M2L (m2l_mfma 2)");
    if (P->p2p_chunk != 0 && P->p2p_chunk != 16 && P->p2p_chunk != 32 && P->p2p_chunk != 64)
        return set_error(FMM_ERR_ARG, "p2p_chunk must be 0, 16, 32 or 64 (got %d)", P->p2p_chunk);
    if (P->schedule == 2 && P->p2p_chunk != 0 && P->p2p_chunk != 32)
        return set_error(FMM_ERR_ARG, "the persistent P2P + M2L kernel (schedule 2) has the sink tile 32 only");
    if (P->precision == 1) {  // the FP32 force law must meet its tolerance at this r_cut / r_s
        P2PConst k;
        if (int rc = p2p_setup(P, k)) return rc;
    }
    if (P->schedule == 2 && !fused_applies(P))
        return set_error(FMM_ERR_ARG, "schedule 2 (one persistent P2P + M2L kernel) requires precision 1, learned 0, "
                                      "3 <= p <= 8, m2l_mfma != 2 and a force law of degree 9 or 10");
    return 0;
}

static void free_buf(DevBuf &b) { release(b); }

static float ev_ms(fmm_tree *t, int a, int b)
{
    float ms = 0;
    (void)hipEventElapsedTime(&ms, t->ev[a], t->ev[b]);  // timing only: 0 if unavailable
    return ms;
}

static void mark(fmm_tree *t, int k, hipStream_t st)
{
    if (t->timing) (void)hipEventRecord(t->ev[k], st);  // a failure shows in the stage's error check
}

// P2P of the leaves of each level as soon as the traversal has listed them: the launch for
// level l waits (on the second stream) for the traversal kernel of level l only, so the
// P2P work of coarse leaves runs beside the traversal of the finer levels.
struct LevelP2P {
    fmm_tree *t;
    const fmm_params *P;
    hipStream_t ax;
};

static int p2p_level_hook(void *ctx, int l, hipStream_t st)
{
    const LevelP2P &c = *static_cast<const LevelP2P *>(ctx);
    fmm_tree *t = c.t;
    if (l + 1 >= (int)t->leaf_lvl.size()) return 0;
    const int first = t->leaf_lvl[l], count = t->leaf_lvl[l + 1] - first;
    if (count <= 0) return 0;
    int rc;
    if ((rc = hip_check(hipEventRecord(t->lev[l], st), "event")) ||
        (rc = hip_check(hipStreamWaitEvent(c.ax, t->lev[l], 0), "event wait")))
        return rc;
    if (t->timing) (void)hipEventRecord(t->p2p_t0[l], c.ax);  // timing only
    // the traversal's overflow flag (counter byte 96): void lists are not read
    if ((rc = p2p_range(t, c.P, first, count, ptr<int>(t->counters) + 24, c.ax))) return rc;
    if (t->timing) (void)hipEventRecord(t->p2p_t1[l], c.ax);
    return 0;
}

// The stages of one short-range evaluation on a built tree (or forest of boxes).
// accumulate: add the short-range accelerations to acc instead of overwriting it.
static int run_forces(fmm_tree *t, const fmm_params *P, double *acc, hipStream_t st, int accumulate = 0)
{
    MacModel hm;
    const MacModel *dm = nullptr;
    if (P->learned) {
        dm = current_model(&hm);
        if (!dm) return set_error(FMM_ERR_STATE, "learned selector requested but no model is loaded");
    }
    if (t->n == 0) return 0;
    // the learned selector chooses orders up to 8: expansions are kept at order 8
    fmm_params P8 = *P;
    if (P->learned) P8.p = 8;
    int rc;
    if (!t->aux) {
        if (hipStreamCreateWithFlags(&t->aux, hipStreamNonBlocking) != hipSuccess)
            return set_error(FMM_ERR_HIP, "hipStreamCreateWithFlags");
        for (auto &e : t->dep)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
                return set_error(FMM_ERR_HIP, "hipEventCreateWithFlags");
    }
    if (!t->lev_ready) {
        for (auto &e : t->lev)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
                return set_error(FMM_ERR_HIP, "hipEventCreateWithFlags");
        for (int l = 0; l <= kMaxLevel; ++l)
            if (hipEventCreate(&t->p2p_t0[l]) != hipSuccess || hipEventCreate(&t->p2p_t1[l]) != hipSuccess)
                return set_error(FMM_ERR_HIP, "hipEventCreate");
        t->lev_ready = true;
    }
    hipStream_t ax = t->aux;
    // Dependencies: upward -> M2L; traversal of level l -> P2P of level l's leaves;
    // traversal -> M2L; M2L -> L2L; {L2L, P2P} -> L2P.
    // The plain traversal does not read multipoles, so the upward pass runs beside it on
    // the second stream; P2P runs there, level by level beside the traversal, then beside
    // M2L and L2L.  The FP32 P2P's leaf boxes depend on the tree only: they are computed
    // on the second stream ahead of P2P.
    if ((rc = hip_check(hipEventRecord(t->dep[0], st), "event")) || (rc = hip_check(hipStreamWaitEvent(ax, t->dep[0], 0), "event wait")))
        return rc;
    mark(t, 0, st);
    const bool fused = P->schedule == 2;
    // P2P level by level beside the traversal, measured on one box each: 134M box 718 ->
    // 697 ms (19M leaves), 16.7M box 75.5 -> 75.0 ms (2.3M leaves), slower on small trees
    // (2M box 9.2 -> 11.4 ms, 64-box forest 12.4 -> 16.6 ms): most P2P work sits in the
    // finest levels, listed last, and each level's launch ends in its own tail
    const bool per_level = P->schedule == 3 || (P->schedule == 0 && t->nleaf >= (1 << 22));
    LevelP2P lp{t, P, ax};
    const TravHook hook{p2p_level_hook, &lp, ax};
    const TravHook *hk = per_level ? &hook : nullptr;
    if (P->learned) {  // the selector's features read the multipoles
        mark(t, 9, st);
        if ((rc = upward(t, &P8, st))) return rc;
        mark(t, 1, st);
        if ((rc = hip_check(hipEventRecord(t->dep[1], st), "event"))) return rc;
        if ((rc = p2p_bbox(t, P, ax))) return rc;
        rc = traverse_mode(t, P, 2, hm.theta_max, t->Mc.p, ncoef(8), P->precision, dm, st, hk);
    } else {
        mark(t, 9, ax);
        if ((rc = upward(t, &P8, ax))) return rc;
        mark(t, 1, ax);
        if ((rc = hip_check(hipEventRecord(t->dep[1], ax), "event"))) return rc;
        if ((rc = p2p_bbox(t, P, ax))) return rc;
        rc = traverse(t, P, st, hk);
    }
    if (rc) return rc;
    mark(t, 2, st);
    if (fused) {  // P2P and M2L in one persistent launch on st, after the second stream's work
        if ((rc = hip_check(hipEventRecord(t->dep[3], ax), "event")) || (rc = hip_check(hipStreamWaitEvent(st, t->dep[3], 0), "event wait")))
            return rc;
        if ((rc = p2p_m2l_fused_prepare(t, P, st))) return rc;
        mark(t, 5, st);
        if ((rc = p2p_m2l_fused_launch(t, P, st))) return rc;
        mark(t, 6, st);
        mark(t, 3, st);
    }
    if (!fused && !per_level) {  // P2P after the whole traversal
        if ((rc = hip_check(hipEventRecord(t->dep[2], st), "event")) ||
            (rc = hip_check(hipStreamWaitEvent(ax, t->dep[2], 0), "event wait")))
            return rc;
        mark(t, 5, ax);
        if ((rc = p2p(t, P, ax))) return rc;
        mark(t, 6, ax);
    }
    if (!fused) {  // (per level: P2P was launched during the traversal)
        if ((rc = hip_check(hipEventRecord(t->dep[3], ax), "event")) || (rc = hip_check(hipStreamWaitEvent(st, t->dep[1], 0), "event wait")))
            return rc;
        if ((rc = P->learned ? m2l_learned(t, P, st) : m2l(t, P, st))) return rc;
        mark(t, 3, st);
    }
    if ((rc = downward_l2l(t, &P8, st))) return rc;
    mark(t, 4, st);
    if (!fused && (rc = hip_check(hipStreamWaitEvent(st, t->dep[3], 0), "event wait"))) return rc;
    mark(t, 10, st);
    if ((rc = l2p_combine(t, &P8, acc, accumulate, st))) return rc;
    mark(t, 11, st);
    t->last_p = P->p;
    t->last_prec = P->precision;
    fmm_stats &S = t->stats;
    S.n_m2l = t->n_m2l;
    S.n_p2p = t->n_p2p;
    S.n_visit = t->n_visit;
    S.levels_traversed = t->nlevel;
    if (t->timing) {  // stages overlap across the two streams; each time is its own span
        if ((rc = hip_check(hipEventSynchronize(t->ev[11]), "timing event"))) return rc;
        S.t_upward_ms = ev_ms(t, 9, 1);
        S.t_traverse_ms = P->learned ? ev_ms(t, 1, 2) : ev_ms(t, 0, 2);
        S.t_m2l_ms = fused ? ev_ms(t, 5, 6) : ev_ms(t, 2, 3);  // schedule 2: both stages are one launch
        S.t_downward_ms = ev_ms(t, 3, 4) + ev_ms(t, 10, 11);
        if (!per_level) {
            S.t_p2p_ms = ev_ms(t, 5, 6);
        } else {  // the sum of the per-level P2P launches
            S.t_p2p_ms = 0.0;
            for (int l = 0; l + 1 < (int)t->leaf_lvl.size() && l <= kMaxLevel; ++l) {
                if (t->leaf_lvl[l + 1] == t->leaf_lvl[l]) continue;
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, t->p2p_t0[l], t->p2p_t1[l]);  // timing only
                S.t_p2p_ms += ms;
            }
        }
        S.t_total_ms = ev_ms(t, 0, 11);
    }
    return hip_check(hipGetLastError(), "short range forces");
}

static int copy_kind(fmm_tree *t, int kind, uint64_t *out, int64_t cap, int64_t *count);

static bool same_params(const fmm_params &a, const fmm_params &b)
{
    return a.box == b.box && a.r_s == b.r_s && a.r_cut == b.r_cut && a.theta == b.theta && a.G == b.G && a.p == b.p &&
           a.n_crit == b.n_crit && a.mac_mode == b.mac_mode && a.precision == b.precision && a.learned == b.learned &&
           a.split == b.split && a.pm_assign == b.pm_assign && a.m2l_mfma == b.m2l_mfma && a.schedule == b.schedule &&
           a.deterministic == b.deterministic && a.p2p_chunk == b.p2p_chunk;
}

static int build_common(const fmm_params *P, int64_t n, const double *pos, const double *mass, int nbox,
                        const int64_t *offsets, void *stream, fmm_tree **out)
{
    hipStream_t st = (hipStream_t)stream;
    fmm_tree *t = *out;
    bool fresh = false;
    if (!t) {
        t = new (std::nothrow) fmm_tree();
        if (!t) return set_error(FMM_ERR_NOMEM, "tree allocation");
        fresh = true;
    }
    if (t->timing) (void)hipEventRecord(t->ev[14], st);  // timing only
    ++t->build_serial;  // buffers may move: a recorded evaluation of the old tree is void
    int rc = tree_build(t, P, n, pos, mass, nbox, offsets, st);
    if (rc) {
        if (fresh) {
            fmm_free_tree(t);
        } else {  // a reused tree that failed part way (e.g. out of memory) is left empty
            t->n = 0;
            t->ncell = t->nleaf = t->nlevel = 0;
            t->lvl_beg.assign(1, 0);
            t->leaf_lvl.assign(1, 0);
            t->stats.n = t->stats.n_cells = t->stats.n_leaves = t->stats.max_level = 0;
        }
        return rc;
    }
    if (t->timing) {
        (void)hipEventRecord(t->ev[15], st);  // timing only
        (void)hipEventSynchronize(t->ev[15]);
        t->stats.t_build_ms = ev_ms(t, 14, 15);
    }
    t->stats.n = n;
    t->stats.n_cells = t->ncell;
    t->stats.n_leaves = t->nleaf;
    t->stats.max_level = t->nlevel - 1;
    *out = t;
    return 0;
}

extern "C" {

const char *fmm_last_error(void) { return last_error(); }

const char *fmm_version(void) { return "hfmm 0.1 gfx950"; }

int fmm_set_timing(fmm_tree *t, int on)
{
    if (!t) return set_error(FMM_ERR_ARG, "tree is NULL");
    if (on && !t->events_ready) {
        for (auto &e : t->ev)
            if (hipEventCreate(&e) != hipSuccess) return set_error(FMM_ERR_HIP, "hipEventCreate");
        t->events_ready = true;
    }
    t->timing = on ? 1 : 0;
    return 0;
}

int fmm_build_tree(const fmm_params *P, int64_t n, const double *pos, const double *mass, void *stream,
                   fmm_tree **out)
{
    clear_error();
    if (int rc = check_params(P)) return rc;
    if (!out) return set_error(FMM_ERR_ARG, "out is NULL");
    if (n < 0) return set_error(FMM_ERR_ARG, "n < 0");
    if (n > 0 && (!pos || !mass)) return set_error(FMM_ERR_ARG, "pos/mass is NULL");
    return build_common(P, n, pos, mass, 1, nullptr, stream, out);
}

int fmm_build_tree_batched(const fmm_params *per_box, int nbox, const int64_t *offsets, const double *pos,
                           const double *mass, void *stream, fmm_tree **out)
{
    clear_error();
    if (!per_box || !offsets || !out) return set_error(FMM_ERR_ARG, "NULL argument");
    if (nbox < 1 || nbox > 65536) return set_error(FMM_ERR_ARG, "nbox must be in [1, 65536]");
    if (int rc = check_params(&per_box[0])) return rc;
    for (int b = 1; b < nbox; ++b)
        if (!same_params(per_box[b], per_box[0]))
            return set_error(FMM_ERR_ARG, "all boxes of a batch must share their parameters (box %d differs)", b);
    if (offsets[0] != 0) return set_error(FMM_ERR_ARG, "offsets[0] must be 0");
    for (int b = 0; b < nbox; ++b)
        if (offsets[b + 1] < offsets[b]) return set_error(FMM_ERR_ARG, "offsets must be non-decreasing");
    int64_t n = offsets[nbox];
    if (n > 0 && (!pos || !mass)) return set_error(FMM_ERR_ARG, "pos/mass is NULL");
    return build_common(&per_box[0], n, pos, mass, nbox, offsets, stream, out);
}

int fmm_short_range_forces(fmm_tree *t, const fmm_params *P, double *acc, void *stream)
{
    clear_error();
    if (!t) return set_error(FMM_ERR_ARG, "tree is NULL");
    if (int rc = check_params(P)) return rc;
    if (P->box != t->box || P->n_crit != t->ncrit)
        return set_error(FMM_ERR_STATE, "box / n_crit differ from the values the tree was built with");
    if (t->n > 0 && !acc) return set_error(FMM_ERR_ARG, "acc is NULL");
    return run_forces(t, P, acc, (hipStream_t)stream);
}

int fmm_short_range_forces_graph(fmm_tree *t, const fmm_params *P, double *acc, void *stream)
{
    clear_error();
    if (!t) return set_error(FMM_ERR_ARG, "tree is NULL");
    if (int rc = check_params(P)) return rc;
    if (P->box != t->box || P->n_crit != t->ncrit)
        return set_error(FMM_ERR_STATE, "box / n_crit differ from the values the tree was built with");
    if (t->n > 0 && !acc) return set_error(FMM_ERR_ARG, "acc is NULL");
    hipStream_t st = (hipStream_t)stream;
    if (!st) return set_error(FMM_ERR_ARG, "the recorded form needs a created stream, not the null stream");
    if (t->n == 0) return 0;
    // replay only while every buffer the graph uses is where it was recorded: no rebuild,
    // and no reallocation since (an eager call with other parameters may grow a buffer)
    if (t->gexec && t->gserial == t->build_serial && t->gmoves == buffer_moves() && same_params(t->gparams, *P) &&
        t->gacc == acc && t->gstream == st && (!P->learned || t->gmodel == model_serial())) {
        for (int o = 0; o < kOrders; ++o) t->stats.n_m2l_by_order[o] = t->g_by_order[o];
        t->n_m2l = t->g_n_m2l;  // the counts of the recorded evaluation, which the replay repeats
        t->n_p2p = t->g_n_p2p;
        t->n_visit = t->g_n_visit;
        t->stats.n_m2l = t->n_m2l;
        t->stats.n_p2p = t->n_p2p;
        t->stats.n_visit = t->n_visit;
        return hip_check(hipGraphLaunch(t->gexec, st), "graph launch");
    }
    if (t->gexec) {
        (void)hipGraphExecDestroy(t->gexec);
        t->gexec = nullptr;
    }
    // one eager evaluation (it sizes every buffer and gives this call's result), then the
    // same stages are recorded; a buffer that would still have to grow fails the recording
    if (int rc = run_forces(t, P, acc, st)) return rc;
    const int timing = t->timing;
    t->timing = 0;
    t->capturing = true;
    int rc = hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture");
    int rc_run = rc ? rc : run_forces(t, P, acc, st);
    hipGraph_t g = nullptr;
    if (!rc) rc = hip_check(hipStreamEndCapture(st, &g), "end capture");
    t->capturing = false;
    t->timing = timing;
    if (!rc) rc = rc_run;
    if (!rc) rc = hip_check(hipGraphInstantiate(&t->gexec, g, nullptr, nullptr, 0), "graph instantiate");
    if (g) (void)hipGraphDestroy(g);
    if (rc) {
        if (t->gexec) (void)hipGraphExecDestroy(t->gexec);
        t->gexec = nullptr;
        (void)hipGetLastError();
        return rc;
    }
    t->gparams = *P;
    t->gacc = acc;
    t->gstream = st;
    t->gserial = t->build_serial;
    t->gmoves = buffer_moves();
    t->gmodel = model_serial();  // the selector's weights and theta_max are part of the recording
    for (int o = 0; o < kOrders; ++o) t->g_by_order[o] = t->stats.n_m2l_by_order[o];
    t->g_n_m2l = t->n_m2l;
    t->g_n_p2p = t->n_p2p;
    t->g_n_visit = t->n_visit;
    return 0;
}

// Times each parameter set of cands (reps timed steps after one untimed one that sizes the
// tree's buffers) and returns the index of the fastest in *best.
static int autotune_sets(const fmm_params *cands, int ncand, int nbox, const int64_t *offsets, int64_t n,
                         const double *pos, const double *mass, double *acc, int reps, void *stream, int *best,
                         double *ms_out)
{
    if (!cands || ncand <= 0) return set_error(FMM_ERR_ARG, "no parameter sets");
    for (int c = 0; c < ncand; ++c)
        if (int rc = check_params(&cands[c])) return rc;
    if (n <= 0 || !pos || !mass || !acc || !best || nbox < 1 || (nbox > 1 && !offsets))
        return set_error(FMM_ERR_ARG, "bad arguments");
    if (nbox > 1 && offsets[nbox] != n) return set_error(FMM_ERR_ARG, "offsets[nbox] != n");
    std::vector<fmm_params> per_box((size_t)nbox);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return set_error(FMM_ERR_HIP, "hipEventCreate");
    fmm_tree *t = nullptr;
    int rc = 0;
    double fastest = 1e300;
    *best = 0;
    const int nrep = reps > 0 ? reps : 1;
    for (int c = 0; c < ncand && !rc; ++c) {
        const fmm_params &Q = cands[c];
        for (auto &b : per_box) b = Q;
        auto build = [&]() {
            return nbox > 1 ? fmm_build_tree_batched(per_box.data(), nbox, offsets, pos, mass, stream, &t)
                            : fmm_build_tree(&Q, n, pos, mass, stream, &t);
        };
        rc = build();
        if (!rc) rc = run_forces(t, &Q, acc, st);
        float total = 0.0f;
        for (int r = 0; r < nrep && !rc; ++r) {
            (void)hipEventRecord(e0, st);  // timing events; failures surface in the step's own checks
            rc = build();
            if (!rc) rc = run_forces(t, &Q, acc, st);
            (void)hipEventRecord(e1, st);
            if (!rc) rc = hip_check(hipEventSynchronize(e1), "autotune");
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            total += ms;
        }
        const double ms = total / nrep;
        if (ms_out) ms_out[c] = ms;
        if (!rc && ms < fastest) {
            fastest = ms;
            *best = c;
        }
    }
    if (t) fmm_free_tree(t);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int fmm_autotune(const fmm_params *P, int nbox, const int64_t *offsets, int64_t n, const double *pos,
                 const double *mass, double *acc, const int *candidates, int ncand, int reps, void *stream,
                 int *best_n_crit, double *ms_out)
{
    clear_error();
    if (int rc = check_params(P)) return rc;
    if (!candidates || ncand <= 0 || !best_n_crit) return set_error(FMM_ERR_ARG, "bad arguments");
    std::vector<fmm_params> cands((size_t)ncand, *P);
    for (int c = 0; c < ncand; ++c) {
        if (candidates[c] < 1) return set_error(FMM_ERR_ARG, "n_crit candidate %d < 1", candidates[c]);
        cands[c].n_crit = candidates[c];
    }
    int bi = 0;
    int rc = autotune_sets(cands.data(), ncand, nbox, offsets, n, pos, mass, acc, reps, stream, &bi, ms_out);
    *best_n_crit = candidates[bi];
    return rc;
}

int fmm_autotune_params(const fmm_params *cands, int ncand, int nbox, const int64_t *offsets, int64_t n,
                        const double *pos, const double *mass, double *acc, int reps, void *stream, int *best,
                        double *ms_out)
{
    clear_error();
    return autotune_sets(cands, ncand, nbox, offsets, n, pos, mass, acc, reps, stream, best, ms_out);
}

int fmm_get_stats(const fmm_tree *tc, fmm_stats *out)
{
    if (!tc || !out) return set_error(FMM_ERR_ARG, "NULL argument");
    fmm_tree *t = const_cast<fmm_tree *>(tc);
    if (t->counters.p && t->n > 0) {  // the P2P kernel counts listed pairs on the device
        unsigned long long v = 0, e = 0;
        if (hipMemcpy(&v, ptr<unsigned long long>(t->counters) + 1, 8, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(&e, ptr<unsigned long long>(t->counters) + 24, 8, hipMemcpyDeviceToHost) != hipSuccess)
            return set_error(FMM_ERR_HIP, "reading counters");
        t->stats.p2p_pairs = (int64_t)v;
        t->stats.p2p_evaluated = (int64_t)e;
    }
    *out = t->stats;
    return 0;
}

int fmm_copy_interactions(const fmm_tree *tc, int kind, uint64_t *out, int64_t cap, int64_t *count)
{
    fmm_tree *t = const_cast<fmm_tree *>(tc);
    if (!t || !count || (kind != 0 && kind != 1)) return set_error(FMM_ERR_ARG, "bad arguments");
    int64_t total = kind ? t->n_p2p : t->n_m2l;
    if (!out) {
        *count = total;
        return 0;
    }
    if (kind == 0 && t->trav_mode == 2)  // learned selector: M2L pairs of every order
        return copy_kind(t, kKindOrd, out, cap, count);
    return copy_kind(t, kind, out, cap, count);
}

static int copy_kind(fmm_tree *t, int kind, uint64_t *out, int64_t cap, int64_t *count)
{
    int nc = t->ncell;
    std::vector<Cell> cells(nc);
    std::vector<int> head(nc), cnt(nc);
    int nchunk = t->lcap[kind] + 1;
    std::vector<uint32_t> items((size_t)nchunk * kChunk);
    std::vector<int> next(nchunk);
    if (hipDeviceSynchronize() != hipSuccess) return set_error(FMM_ERR_HIP, "sync");
    if (hipMemcpy(cells.data(), t->cells.p, (size_t)nc * sizeof(Cell), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(head.data(), ptr<int>(t->lhead) + (size_t)kind * nc, (size_t)nc * 4, hipMemcpyDeviceToHost) !=
            hipSuccess ||
        hipMemcpy(cnt.data(), ptr<int>(t->lcnt) + (size_t)kind * nc, (size_t)nc * 4, hipMemcpyDeviceToHost) !=
            hipSuccess ||
        hipMemcpy(items.data(), t->litems[kind].p, items.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(next.data(), t->lnext[kind].p, next.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return set_error(FMM_ERR_HIP, "copying interaction lists");
    std::vector<uint64_t> key(nc);
    for (int c = 0; c < nc; ++c)
        key[c] = cell_key_host(cell_level(cells[c]), cell_ix(cells[c]), cells[c].iy, cells[c].iz);
    int64_t w = 0;
    for (int c = 0; c < nc && w < cap; ++c) {
        int chunk = head[c];
        for (int e = 0; e < cnt[c] && w < cap; ++e) {
            if (e > 0 && e % kChunk == 0) chunk = next[chunk];
            uint32_t it = items[(size_t)chunk * kChunk + e % kChunk];
            out[3 * w] = key[c];
            out[3 * w + 1] = key[it >> 5];
            out[3 * w + 2] = it & 31;
            ++w;
        }
    }
    *count = w;
    return 0;
}

int fmm_mac_training_data(fmm_tree *t, const fmm_params *P, double theta_max, const double *acc_ref, double eps,
                          int stride, float *feats, int *labels, float *errs, uint64_t *pairs, int64_t cap,
                          int64_t *count, void *stream)
{
    clear_error();
    if (!t || !count || !acc_ref) return set_error(FMM_ERR_ARG, "NULL argument");
    if (int rc = check_params(P)) return rc;
    if (P->box != t->box || P->n_crit != t->ncrit) return set_error(FMM_ERR_STATE, "tree / params mismatch");
    if (!(theta_max > 0) || !(theta_max < 0.75)) return set_error(FMM_ERR_ARG, "theta_max must be in (0, 0.75)");
    if (cap > 0 && (!feats || !labels)) return set_error(FMM_ERR_ARG, "output buffers are NULL");
    if (cap > INT32_MAX) cap = INT32_MAX;
    hipStream_t st = (hipStream_t)stream;
    *count = 0;
    if (t->n == 0) return 0;
    fmm_params P8 = *P;
    P8.p = 8;
    P8.precision = 0;
    P8.learned = 0;
    int rc = upward(t, &P8, st);  // FP64 multipoles of order 8
    if (!rc) rc = traverse_mode(t, P, 1, theta_max, t->Mc.p, ncoef(8), 0, nullptr, st);
    if (rc) return rc;
    DevBuf aref, ctr;
    rc = grow(aref, (size_t)t->n * 24) | grow(ctr, 16);
    if (!rc) rc = sort_soa(t, acc_ref, ptr<double>(aref), st);
    if (!rc) {
        rc = hip_check(hipMemsetAsync(ctr.p, 0, 4, st), "training data");
        if (!rc) rc = run_labels(t, P, ptr<double>(aref), eps, stride, feats, labels, errs, pairs, (int)cap, ptr<int>(ctr), st);
    }
    int n = 0;
    if (!rc) {
        rc = hip_check(hipMemcpyAsync(&n, ctr.p, 4, hipMemcpyDeviceToHost, st), "training data");
        if (!rc) rc = hip_check(hipStreamSynchronize(st), "training data");
    }
    release(aref);
    release(ctr);
    *count = n < cap ? n : cap;
    return rc;
}

int pm_long_range_forces(const fmm_params *P, int mesh, int64_t n, const double *pos, const double *mass,
                         double *acc, void *stream)
{
    clear_error();
    if (int rc = check_params(P)) return rc;
    if (n < 0) return set_error(FMM_ERR_ARG, "n < 0");
    if (n > 0 && (!pos || !mass || !acc)) return set_error(FMM_ERR_ARG, "NULL pointer");
    return pm_forces(P, mesh, n, pos, mass, acc, (hipStream_t)stream);
}

int fmm_hybrid_forces_tree(fmm_tree **tree, const fmm_params *P, int mesh, int64_t n, const double *pos,
                           const double *mass, double *acc, void *stream)
{
    clear_error();
    if (!tree) return set_error(FMM_ERR_ARG, "tree is NULL");
    if (int rc = check_params(P)) return rc;
    if (n < 0) return set_error(FMM_ERR_ARG, "n < 0");
    if (n == 0) return 0;
    if (!pos || !mass || !acc) return set_error(FMM_ERR_ARG, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    if (int rc = fmm_build_tree(P, n, pos, mass, stream, tree)) return rc;
    fmm_tree *t = *tree;
    mark(t, 7, st);
    if (int rc = pm_forces_tree(P, mesh, t, acc, st)) return rc;  // deposits in Morton order
    mark(t, 8, st);
    if (int rc = run_forces(t, P, acc, st, 1)) return rc;
    if (t->timing) {
        (void)hipEventSynchronize(t->ev[8]);  // timing only
        t->stats.t_pm_ms = ev_ms(t, 7, 8);
    }
    return hip_check(hipGetLastError(), "hybrid");
}

int hybrid_forces(const fmm_params *P, int mesh, int64_t n, const double *pos, const double *mass, double *acc,
                  void *stream)
{
    static std::mutex mu;
    static fmm_tree *tree = nullptr;  // kept between calls: a steady-state call allocates nothing
    std::lock_guard<std::mutex> lk(mu);
    return fmm_hybrid_forces_tree(&tree, P, mesh, n, pos, mass, acc, stream);
}

int fmm_short_range_forces_batched(const fmm_params *per_box, int nbox, const int64_t *offsets, const double *pos,
                                   const double *mass, double *acc, void *stream)
{
    static std::mutex mu;
    static fmm_tree *forest = nullptr;  // reused across calls: steady-state calls allocate nothing
    std::lock_guard<std::mutex> lk(mu);
    if (int rc = fmm_build_tree_batched(per_box, nbox, offsets, pos, mass, stream, &forest)) return rc;
    if (forest->n > 0 && !acc) return set_error(FMM_ERR_ARG, "acc is NULL");
    return run_forces(forest, &per_box[0], acc, (hipStream_t)stream);
}

int fmm_set_memory_limit(uint64_t bytes)
{
    set_memory_limit(bytes);
    return 0;
}

int fmm_get_memory_use(uint64_t *bytes)
{
    if (!bytes) return set_error(FMM_ERR_ARG, "bytes is NULL");
    *bytes = memory_in_use();
    return 0;
}

void fmm_free_tree(fmm_tree *t)
{
    if (!t) return;
    DevBuf *bufs[] = {&t->keys[0], &t->keys[1], &t->idx[0], &t->idx[1], &t->xs, &t->ys, &t->zs, &t->ms, &t->perm,
                      &t->leaf_of, &t->rel32, &t->nearf, &t->cells, &t->leaves, &t->inner, &t->Mc, &t->Lc, &t->lhead,
                      &t->lcnt, &t->tstack, &t->counters, &t->scan_tmp, &t->nch, &t->flag, &t->boxoff,
                      &t->m2l_ctr, &t->m2l_pairs, &t->bbox, &t->wstate, &t->cfeat, &t->cellc, &t->mf_ne,
                      &t->mf_no, &t->mf_offe, &t->mf_offn, &t->mf_spos, &t->mf_sinks, &t->mf_csr, &t->mf_tot};
    for (DevBuf *b : bufs) free_buf(*b);
    free_buf(t->lord);
    for (int k = 0; k < kKinds; ++k) {
        free_buf(t->litems[k]);
        free_buf(t->lnext[k]);
    }
    if (t->gexec) (void)hipGraphExecDestroy(t->gexec);
    if (t->host) (void)hipHostFree(t->host);
    if (t->events_ready)
        for (auto &e : t->ev) (void)hipEventDestroy(e);
    if (t->bev_ready)
        for (auto &e : t->bev) (void)hipEventDestroy(e);
    if (t->lev_ready) {
        for (auto &e : t->lev) (void)hipEventDestroy(e);
        for (auto &e : t->p2p_t0) (void)hipEventDestroy(e);
        for (auto &e : t->p2p_t1) (void)hipEventDestroy(e);
    }
    if (t->aux) {
        (void)hipStreamSynchronize(t->aux);
        for (auto &e : t->dep) (void)hipEventDestroy(e);
        (void)hipStreamDestroy(t->aux);
    }
    delete t;
}

}  // extern "C"

namespace hfmm {
uint64_t cell_key_host(int level, int ix, int iy, int iz)
{
    uint64_t k = 1;
    for (int b = level - 1; b >= 0; --b)
        k = (k << 3) | ((uint64_t)((ix >> b) & 1) << 2) | ((uint64_t)((iy >> b) & 1) << 1) | (uint64_t)((iz >> b) & 1);
    return k;
}
}  // namespace hfmm
