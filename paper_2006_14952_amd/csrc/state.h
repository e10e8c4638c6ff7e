// The opaque tree handle: every device buffer of one box, grown on demand.
#pragma once
#include <vector>

#include "common.h"

namespace hfmm {
constexpr int kHostInts = 1024;
constexpr int kHostLevels = 512;  // tree build: level sizes mirrored at host[kHostLevels ...]
// Interaction list kinds: 0 M2L, 1 P2P, 2 handed to the children, 3 candidate pairs
// (training export), 4 M2L pairs of the learned selector (all orders; the order of each
// entry in a byte beside it).
constexpr int kKinds = 5;
constexpr int kKindCand = 3, kKindOrd = 4;
constexpr int kOrders = 7;  // learned selector: M2L orders 2 .. 8
}

struct fmm_tree {
    // shape
    int64_t n = 0;
    double box = 1.0;
    int ncrit = 32;
    int ncell = 0, nleaf = 0, nlevel = 0;  // levels 0 .. nlevel-1 are non-empty
    int nbox = 1;                          // roots: one per box of a batch
    std::vector<int> hboxoff;              // particle offsets of the boxes (host copy)
    std::vector<int> lvl_beg;              // cells of level l: lvl_beg[l] .. lvl_beg[l+1]-1
    std::vector<int> leaf_lvl;             // leaves of level l: leaves[leaf_lvl[l] .. leaf_lvl[l+1]-1]

    // particles, Morton order
    hfmm::DevBuf keys[2], idx[2];
    int sorted = 0;               // which of keys/idx holds the sorted order
    hfmm::DevBuf boxoff;          // int[nbox + 1] particle offsets of the boxes
    hfmm::DevBuf xs, ys, zs, ms;  // wrapped FP64 positions and masses
    hfmm::DevBuf perm;            // sorted index -> caller index
    hfmm::DevBuf leaf_of;         // sorted index -> leaf cell
    hfmm::DevBuf rel32;           // float4 (x - c_leaf, m) for the FP32 form
    hfmm::DevBuf nearf;           // near-field acceleration, 3 x n FP64 (SoA)

    // cells
    hfmm::DevBuf cells;           // Cell[ncell]
    hfmm::DevBuf leaves;          // int[nleaf]
    hfmm::DevBuf inner;           // int[ncell - nleaf]: the cells with children, level by level
    hfmm::DevBuf Mc, Lc;          // expansion coefficients, ncell x ncoef(p) (float or double)

    // interaction lists: per cell and list kind (hfmm::kKinds), a chain of 64-entry chunks;
    // head[k * ncell + c], cnt[k * ncell + c].  lcnt continues with the learned selector's
    // per-order counts, cnt[(kKinds + o - 2) * ncell + c] for order o.
    hfmm::DevBuf lhead, lcnt;
    hfmm::DevBuf litems[hfmm::kKinds], lnext[hfmm::kKinds];
    hfmm::DevBuf lord;                               // kind kKindOrd: the M2L order of each entry (byte)
    int lcap[hfmm::kKinds] = {0};                    // chunks (one more is allocated as overflow bin)
    int64_t lseg[hfmm::kOrders] = {0};               // learned: start of each order's pairs in m2l_pairs
    int trav_mode = 0;                               // mode of the last traversal
    hfmm::DevBuf tstack;                             // per-wave traversal stacks
    hfmm::DevBuf cellc;                              // packed 16-byte cell view for the traversal
    int stk_cap = 4096;                              // entries per wave (grows on overflow)
    int64_t n_m2l = 0, n_p2p = 0, n_visit = 0, p2p_pairs = 0;
    hfmm::DevBuf counters;                           // device counters

    // scratch
    hfmm::DevBuf scan_tmp, nch, flag;
    hfmm::DevBuf m2l_ctr, m2l_pairs;  // flattened M2L pairs (sink, item) for the pair kernel; its fill counter
    hfmm::DevBuf wstate;              // per traversal wave: chunk block in use of each list kind
    hfmm::DevBuf bbox;                // per cell: float4 lo, hi of its particles relative to the centre (leaves)
    // matrix-core M2L: per cell the entries it takes (ne) and the others (no), their
    // offsets, the sinks with such entries (compacted), the entries by sink (CSR), totals
    hfmm::DevBuf mf_ne, mf_no, mf_offe, mf_offn, mf_spos, mf_sinks, mf_csr, mf_tot;
    int64_t mf_n_other = 0;           // sizes of the last split (a recorded replay reuses them)
    int mf_nsink = 0;
    hfmm::DevBuf cfeat;               // learned selector: per-cell part of the features (float4)
    int *host = nullptr;  // pinned readback area (kHostInts ints)
    int last_p = -1, last_prec = -1;

    // second stream (default priority) for stages independent of the caller's stream
    hipStream_t aux = nullptr;
    hipEvent_t dep[4]{};
    hipEvent_t bev[hfmm::kMaxLevel + 1]{};  // tree build: one per level launch
    bool bev_ready = false;
    // traversal: the lists of level l's sinks are complete (lev); P2P launch of level l (timing)
    hipEvent_t lev[hfmm::kMaxLevel + 1]{}, p2p_t0[hfmm::kMaxLevel + 1]{}, p2p_t1[hfmm::kMaxLevel + 1]{};
    bool lev_ready = false;

    // recorded evaluation (fmm_short_range_forces_graph): the executable graph, what it was
    // recorded with, and the build it belongs to
    hipGraphExec_t gexec = nullptr;
    fmm_params gparams{};
    double *gacc = nullptr;
    hipStream_t gstream = nullptr;
    uint64_t build_serial = 0, gserial = 0, gmoves = 0;
    int64_t g_n_m2l = 0, g_n_p2p = 0, g_n_visit = 0;  // the recorded evaluation's counts
    int64_t g_by_order[hfmm::kOrders] = {0};
    uint64_t gmodel = 0;                              // selector model the graph was recorded with
    bool capturing = false;  // run_forces is being recorded: no host reads, no timing

    // timing
    int timing = 0;
    fmm_stats stats{};
    hipEvent_t ev[16]{};
    bool events_ready = false;
};

namespace hfmm {
int tree_build(fmm_tree *t, const fmm_params *P, int64_t n, const double *pos, const double *mass, int nbox,
               const int64_t *offsets, hipStream_t st);
// Called by the traversal after it has launched the kernel of sink level l on st: once that
// launch ends, the lists of the level's sinks are complete.  `side` is the stream the hook
// launches on; the traversal synchronises it before a rerun (whose lists replace these).
struct TravHook {
    int (*level)(void *ctx, int l, hipStream_t st);
    void *ctx;
    hipStream_t side;
};
int traverse(fmm_tree *t, const fmm_params *P, hipStream_t st, const TravHook *hook = nullptr);
struct MacModel;
int traverse_mode(fmm_tree *t, const fmm_params *P, int mode, double theta_max, const void *M, int mstride,
                  int mprec, const MacModel *model, hipStream_t st, const TravHook *hook = nullptr);
int upward(fmm_tree *t, const fmm_params *P, hipStream_t st);
int m2l(fmm_tree *t, const fmm_params *P, hipStream_t st);
int m2l_learned(fmm_tree *t, const fmm_params *P, hipStream_t st);
int downward_l2l(fmm_tree *t, const fmm_params *P, hipStream_t st);
int p2p(fmm_tree *t, const fmm_params *P, hipStream_t st);
// P2P of the sink leaves leaves[first .. first+count-1]; with err non-NULL the launch does
// nothing while *err is non-zero (lists of a traversal that overflowed)
int p2p_range(fmm_tree *t, const fmm_params *P, int first, int count, const int *err, hipStream_t st);
int p2p_bbox(fmm_tree *t, const fmm_params *P, hipStream_t st);  // before p2p (FP32 form): leaf boxes
bool fused_applies(const fmm_params *P);                            // schedule 2 serves these parameters
int p2p_m2l_fused_prepare(fmm_tree *t, const fmm_params *P, hipStream_t st);  // schedule 2: L, pairs, queue
int p2p_m2l_fused_launch(fmm_tree *t, const fmm_params *P, hipStream_t st);   // P2P + M2L, one launch
int l2p_combine(fmm_tree *t, const fmm_params *P, double *acc, int accumulate, hipStream_t st);
// FP32 M2L of order p in 4..8 on the matrix cores for pairs on one level; the other
// pairs are left in t->m2l_pairs, their number in *n_other (L zeroed by the caller)
int m2l_mfma_split_and_run(fmm_tree *t, int p, Split sp, int64_t *n_other, hipStream_t st);
uint64_t cell_key_host(int level, int ix, int iy, int iz);
}  // namespace hfmm
