/*
 * hfmm.h -- C ABI of the MI355X (gfx950) short-range gravity solver of the hybrid
 * PM-FMM method of Q. Wang, "A Hybrid Fast Multipole Method for Cosmological N-body
 * Simulations" (arXiv:2006.14952).
 *
 * The short-range force is the Gaussian-split (erfc-truncated) part of periodic
 * Newtonian gravity (Sec. 2.2, truncated potential and force law):
 *     a_i = G sum_{j, 0 < r_ij < r_cut} m_j f_(1)(r_ij) d_ij,
 *     f_(1)(r) = -[erfc(r/2r_s) + r/(r_s sqrt(pi)) exp(-r^2/4r_s^2)] / r^3,
 *     d_ij = x_i - x_j - box * round((x_i - x_j)/box)   (minimum image; r_cut < box/2).
 * It is evaluated by a truncated Cartesian FMM (Sec. 2.1 Eqs. (1)-(6) with the
 * truncated prefactors of Sec. 2.2) over a Morton-ordered octree, with the modified
 * multipole acceptance criterion of Sec. 2.3.  The long-range part is a plain
 * particle-mesh step with the Gaussian filter exp(-k^2 r_s^2) (Sec. 2.2).
 *
 * Conventions for every entry point:
 *   - Pointers named pos / mass / acc are DEVICE pointers owned by the caller,
 *     contiguous, double precision; pos and acc are (n, 3) row-major.
 *   - stream is a hipStream_t passed as void*; NULL means the default stream.  All
 *     GPU work is enqueued on it.  Calls return after enqueuing, except where noted
 *     (tree building reads a few level sizes back to the host).
 *   - Return value: 0 on success, a negative FMM_ERR_* code otherwise; the message
 *     of the last error of the calling thread is available from fmm_last_error().
 *   - Positions outside [0, box) are wrapped periodically; NaN or Inf positions are
 *     rejected with FMM_ERR_NAN (checked on the device, reported by the call).
 *   - Output is acceleration (units with the given G) in the caller's particle order.
 */
#ifndef HFMM_H
#define HFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FMM_OK 0
#define FMM_ERR_ARG (-1)    /* invalid argument or parameter */
#define FMM_ERR_NOMEM (-2)  /* device or host allocation failed */
#define FMM_ERR_HIP (-3)    /* a HIP runtime call or kernel launch failed */
#define FMM_ERR_NAN (-4)    /* non-finite input position */
#define FMM_ERR_STATE (-5)  /* tree and parameters do not match */

#define FMM_PMAX 8          /* highest expansion order compiled for the GPU */
#define FMM_MAXLEVEL 21     /* finest octree level (63-bit Morton keys) */

/* Method parameters (Secs. 2.1-2.3).
 *   box       periodic box side L > 0
 *   r_s       split scale of the Gaussian filter (Sec. 2.2), > 0
 *   r_cut     truncation radius of the short-range force (~5 r_s in the paper), 0 < r_cut < box/2
 *   theta     opening angle of MAC item 2 (Sec. 2.3), > 0
 *   G         gravitational constant (1 in the workloads)
 *   p         expansion order, 0 <= p <= FMM_PMAX
 *   n_crit    leaf limit: a cell is split while it holds more than n_crit particles (Sec. 2.1), >= 1
 *   mac_mode  bit 0: literal item 3 (open when S_c > r_cut > S_m) instead of the strict
 *             reading (open when S_M > r_cut >= S_m); bit 1: item 2 uses the source side
 *             alone instead of the larger side of the pair; bit 2: conventional MAC, the
 *             baseline of the cost comparison of Sec. 3 (item 2 alone: no neglect beyond
 *             r_cut, no forced opening across it; forces stay correct, at higher cost)
 *   precision 0: FP64 everywhere; 1: P2P and M2L in FP32 on cell-relative coordinates with
 *             compensated per-particle sums, FP64 positions, cell offsets and final sum;
 *             with split 0 the FP32 pair force uses a fitted polynomial whose degree (9, 10
 *             or 14) is chosen for r_cut / r_s, and r_cut > 6 r_s is rejected (FMM_ERR_ARG):
 *             beyond it FP32 cancellation near the cutoff exceeds the form's error bar
 *   learned   0: plain MAC at fixed p; 1: learned accept/order selector (see
 *             fmm_load_mac_model), the plain MAC's hard rules still apply
 *   split     0: the Gaussian (erfc) split of Sec. 2.2 with scale r_s, hard cut at r_cut;
 *             1: the polynomial split (the alternative truncation function Sec. 5 allows):
 *             phi_s = g(r/r_cut)/r, g(x) = 1 - 15/8 x + 5/4 x^3 - 3/8 x^5 below r_cut and 0
 *             beyond (r_s unused by the short range); PM filters with the transform of
 *             its smoothing density.  The learned selector requires split 0.
 *   pm_assign mass assignment of the PM long range: 0 or 2 cloud-in-cell, 3 triangular-
 *             shaped cloud, 4 piecewise cubic (B-splines of that order; the window
 *             sinc^order is divided out twice).  Unused by the short range.
 *   m2l_mfma  M2L kernel of the FP32 form (orders 4..8, plain MAC): 1 the lane-per-pair
 *             kernel on the vector ALUs; 2 pairs of cells on one level as dense products on
 *             the matrix cores (FP32 MFMA; pairs sharing an offset share the transfer
 *             matrix), the other pairs on the vector ALUs; 0 the library's choice.
 *   schedule  how P2P and M2L share the GPU (the task pool of Sec. 4): 1 two kernels on
 *             two streams, P2P after the traversal, beside M2L; 2 one persistent kernel
 *             whose workgroups pull sink leaves (P2P) and then blocks of 64 M2L pairs from
 *             one device queue until both stages are done; 3 as 1, but the P2P of each
 *             leaf level is launched as soon as the traversal has listed that level, so
 *             it runs beside the traversal of the finer levels; 0 the library's choice (3
 *             for trees of 2^22 leaves or more, else 1).  Schedule 2 requires precision 1,
 *             learned 0, 3 <= p <= 8, m2l_mfma != 2 and, with split 0, a force law of
 *             degree 9 or 10 (r_cut / r_s up to about 5.1); FMM_ERR_ARG otherwise.  The results do
 *             not depend on the schedule beyond FP32 summation order.
 *   deterministic  0: the fastest kernels, whose floating-point sums over the M2L pairs of
 *             a sink (and the PM mass deposit) are combined by atomics, so two runs agree
 *             only to rounding (about 1e-11 relative in FP64, 1e-5 in FP32); 1: every sum
 *             in a fixed order, so repeated runs on the same input give bit-identical
 *             accelerations: M2L by one thread per sink over its list in list order, the
 *             PM deposit in 64-bit fixed point (scaled by the total |mass|, exact integer
 *             sums, rounding below 1e-15 of the total mass per particle).  Slower (the M2L
 *             stage several times); schedule 2 and m2l_mfma 2 are refused with it
 *             (FMM_ERR_ARG).  0 or 1.
 *   p2p_chunk sink tile of P2P: a sink leaf is processed in Morton-ordered chunks of this
 *             many particles, each culled against the box of its own particles and
 *             replicated 64 / size times across the 64 lanes of a wave; 16, 32 or 64, 0 the
 *             library's choice (32).  A tile size for fmm_autotune_params; the results
 *             do not depend on it beyond FP32 summation order.  Schedule 2 has tile 32
 *             only (FMM_ERR_ARG for 16 or 64). */
typedef struct fmm_params {
    double box, r_s, r_cut, theta, G;
    int p, n_crit;
    int mac_mode;
    int precision;
    int learned;
    int split;
    int pm_assign;
    int m2l_mfma;
    int schedule;
    int deterministic;
    int p2p_chunk;
} fmm_params;

/* Counters and stage times of the last fmm_short_range_forces on a tree. Counts
 * follow the paper's cost measure (numbers of M2L and P2P operations, Sec. 3). */
typedef struct fmm_stats {
    int64_t n;                 /* particles */
    int64_t n_cells, n_leaves, max_level;
    int64_t n_m2l;             /* accepted M2L cell pairs */
    int64_t n_p2p;             /* P2P leaf pairs */
    int64_t p2p_pairs;         /* listed particle pairs (sum over P2P leaf pairs of n_A n_B) */
    int64_t n_visit;           /* cell pairs examined by the traversal */
    int64_t levels_traversed;
    int64_t n_m2l_by_order[7]; /* learned selector: accepted pairs at order 2..8 (else 0) */
    int64_t p2p_evaluated;     /* particle pairs the P2P kernel evaluated: the listed pairs less
                                  those of source leaves whose particles' bounding box is
                                  farther than r_cut from the sink leaf's (FP32 form) */
    /* stage spans (with timing on; stages on the two streams overlap); under schedule 2
       t_m2l_ms and t_p2p_ms are both the span of the one P2P + M2L launch */
    double t_tree_ms, t_upward_ms, t_traverse_ms, t_m2l_ms, t_p2p_ms, t_downward_ms, t_total_ms;
    double t_build_ms;         /* last fmm_build_tree */
    double t_pm_ms;            /* long-range (PM) part of the last fmm_hybrid_forces_tree */
    double reserved_d[6];
} fmm_stats;

typedef struct fmm_tree fmm_tree; /* opaque; owned by the library */

/* Build the Morton-ordered octree of n particles (the particle packs of Sec. 2.1):
 * wrap, 63-bit Morton keys, radix sort, SoA permutation, cells level by level.
 * pos (n,3) and mass (n) stay owned by the caller and must not change before the
 * forces are computed.  *out receives a new tree, or an existing tree passed in *out
 * is reused (its device memory only grows).  Uses params->box and params->n_crit.
 * Synchronises the stream (level sizes are read back).  n = 0 is allowed, n <= 2^30.
 * A tree of 2^27 cells or more is rejected with FMM_ERR_ARG (interaction-list entries
 * address cells with 27 bits; a larger n_crit gives fewer cells).  On any failure a
 * tree passed in *out is left empty (0 particles) and must be rebuilt before use. */
int fmm_build_tree(const fmm_params *params, int64_t n, const double *pos, const double *mass, void *stream,
                   fmm_tree **out);

/* Short-range accelerations of the particles of a built tree (Secs. 2.1-2.3):
 * upward pass (P2M, M2M), dual traversal with the modified MAC, M2L and P2P, downward
 * pass (L2L, L2P).  acc (n,3) is overwritten.  params->box and n_crit must equal the
 * values the tree was built with (FMM_ERR_STATE otherwise).  Synchronises the stream
 * once, after the traversal (list pool usage is read back; if a pool or traversal stack
 * was too small the traversal is rerun with enough room). */
int fmm_short_range_forces(fmm_tree *tree, const fmm_params *params, double *acc, void *stream);

/* The same evaluation as fmm_short_range_forces, recorded once as a HIP graph and then
 * replayed, for callers that evaluate one built tree (one box or a forest of boxes)
 * repeatedly: a replay is one hipGraphLaunch on `stream`, with no host synchronisation.
 * The first call on a tree, and any call after the tree is rebuilt, after any library
 * buffer was reallocated (e.g. by an eager call with a higher order), or with other params,
 * acc or stream, runs the evaluation eagerly (its result is this call's result) and then
 * records the same stages, on `stream` and the tree's second stream, into a graph the
 * tree owns (freed by fmm_free_tree or replaced on the next recording).  The graph
 * writes the acc it was recorded with: keep that buffer allocated while replaying.  A
 * replay reuses the recorded list sizes (they repeat exactly on an unchanged tree);
 * fmm_get_stats after a replay reports those counts and the replay's own pair
 * counters.  With the learned
 * selector, loading or clearing a model also makes the next call record again.  `stream`
 * must be a created stream (the null stream cannot be recorded: FMM_ERR_ARG).  Errors
 * as fmm_short_range_forces; a failed recording (FMM_ERR_HIP) leaves no graph behind and
 * the eager result stands. */
int fmm_short_range_forces_graph(fmm_tree *tree, const fmm_params *params, double *acc, void *stream);

/* Long-range accelerations by the particle-mesh method with a mesh of mesh^3 cells
 * (Sec. 2.2: Poisson Green function filtered by exp(-k^2 r_s^2)): mass deposit (CIC, TSC
 * or PCS by params->pm_assign), FFT, filtered Green function with the assignment window
 * deconvolved, spectral gradient, inverse FFTs, interpolation with the same weights.
 * acc (n,3) is overwritten.  8 <= mesh <= 1024. */
int pm_long_range_forces(const fmm_params *params, int mesh, int64_t n, const double *pos, const double *mass,
                         double *acc, void *stream);

/* Total periodic acceleration of the hybrid method (Sec. 2.2 split): the PM long-range
 * part written into acc, then the short-range part added to it by the final L2P +
 * near-field kernel.  Builds the octree into *tree (a new tree if *tree is NULL, else
 * the given tree is rebuilt in place; the caller frees it with fmm_free_tree), so the
 * tree's statistics (fmm_get_stats, with t_pm_ms) describe this call.  acc (n,3) is
 * overwritten.  Synchronises the stream like fmm_build_tree and fmm_short_range_forces. */
int fmm_hybrid_forces_tree(fmm_tree **tree, const fmm_params *params, int mesh, int64_t n, const double *pos,
                           const double *mass, double *acc, void *stream);

/* fmm_hybrid_forces_tree on a tree owned by the library: it is kept (and grown) across
 * calls until the process ends, so repeated calls allocate nothing once sizes are
 * steady.  Calls are serialised by a lock.  acc (n,3) is overwritten. */
int hybrid_forces(const fmm_params *params, int mesh, int64_t n, const double *pos, const double *mass,
                  double *acc, void *stream);

/* Build one forest over nbox independent periodic boxes stored back to back: box b holds
 * particles offsets[b] .. offsets[b+1]-1 of pos/mass (offsets: HOST array of nbox+1
 * entries, offsets[0] = 0, non-decreasing; empty boxes allowed).  Every box gets its own
 * root; particles are ordered by box, then Morton key.  All per_box entries must be equal
 * (FMM_ERR_ARG otherwise).  The returned tree works with fmm_short_range_forces,
 * fmm_get_stats, fmm_set_timing, fmm_copy_interactions and fmm_free_tree; its stages
 * process all boxes in shared launches.  Reuse of *out as in fmm_build_tree. */
int fmm_build_tree_batched(const fmm_params *per_box, int nbox, const int64_t *offsets, const double *pos,
                           const double *mass, void *stream, fmm_tree **out);

/* Short-range accelerations of nbox independent periodic boxes stored back to back:
 * box b holds particles offsets[b] .. offsets[b+1]-1 of pos/mass/acc, with its own
 * parameters per_box[b] (all equal, see fmm_build_tree_batched).  offsets is a HOST
 * array of nbox+1 entries starting at 0.  Builds a forest held by the library (reused by
 * later calls, serialised by a lock) and evaluates all boxes in shared launches. */
int fmm_short_range_forces_batched(const fmm_params *per_box, int nbox, const int64_t *offsets,
                                   const double *pos, const double *mass, double *acc, void *stream);

/* Autotuner: times complete steps (tree build + fmm_short_range_forces with the
 * parameters in params) for each leaf limit in candidates[0..ncand-1] (each >= 1), reps
 * timed steps each after one untimed one, on the caller's particles, and returns the
 * fastest in *best_n_crit.  The leaf limit sets the tile shape of every stage (P2P sink
 * and source tiles, list lengths, tree depth).  nbox = 1 tunes one box (offsets may be
 * NULL); nbox > 1 tunes the forest of fmm_build_tree_batched (offsets: HOST array of
 * nbox+1 entries, offsets[nbox] = n).  ms_out (host, ncand entries, may be NULL)
 * receives the mean step time of each candidate; acc (device, (n,3)) is scratch for the
 * forces.  Uses a temporary tree; synchronises the stream. */
int fmm_autotune(const fmm_params *params, int nbox, const int64_t *offsets, int64_t n, const double *pos,
                 const double *mass, double *acc, const int *candidates, int ncand, int reps, void *stream,
                 int *best_n_crit, double *ms_out);

/* Autotuner over whole parameter sets (the tile and kernel choices of Sec. 4's GPU
 * form): times complete steps (tree build + fmm_short_range_forces) for each of the ncand
 * parameter sets in cands (HOST array), reps timed steps each after one untimed one, and
 * returns the index of the fastest in *best.  The sets normally differ only in what picks
 * tile shapes and kernels: n_crit (P2P sink and source tiles, list lengths, tree depth),
 * schedule (two streams, or one persistent P2P + M2L kernel) and m2l_mfma (vector ALUs or
 * matrix cores); which of them may vary is the caller's choice (the lists, and so the
 * forces, depend on n_crit).  nbox, offsets, n, pos, mass, acc: as fmm_autotune.  ms_out
 * (host, ncand entries, may be NULL) receives each set's mean step time.  Every set is
 * validated before any is timed (FMM_ERR_ARG names the first invalid one's fault).
 * Uses a temporary tree; synchronises the stream. */
int fmm_autotune_params(const fmm_params *cands, int ncand, int nbox, const int64_t *offsets, int64_t n,
                        const double *pos, const double *mass, double *acc, int reps, void *stream, int *best,
                        double *ms_out);

/* Counters and stage times of the last force evaluation (host struct, caller-owned). */
int fmm_get_stats(const fmm_tree *tree, fmm_stats *out);

/* Turn per-stage timing with HIP events on (1) or off (0) for this tree.  Timing
 * synchronises the stream after each stage. */
int fmm_set_timing(fmm_tree *tree, int on);

/* Copy the interaction lists of the last force evaluation to HOST memory as
 * (sink cell key, source cell key, image) triples, image = 9 (sx+1) + 3 (sy+1) + (sz+1).
 * A cell key is (1 << 3 level) | morton(ix, iy, iz) at its level.  kind 0 = M2L,
 * 1 = P2P.  With out == NULL only the count is returned in *count; otherwise at most
 * cap triples are written and *count receives the number written. */
int fmm_copy_interactions(const fmm_tree *tree, int kind, uint64_t *out, int64_t cap, int64_t *count);

/* ---- learned acceptance / order selector -----------------------------------------
 * A small MLP (16 features -> 64 -> 64 -> 8 classes, ReLU) decides, for every cell pair
 * that passes MAC items 1 and 3 (Sec. 2.3) and has L/S_c <= theta_max, whether to open it
 * (class 0) or accept it with an M2L of order c + 1 (classes 1..7, orders 2..8).  Pairs
 * that fail items 1 or 3, or exceed theta_max, are handled by the plain rules (neglect /
 * open), so the selector never accepts a pair the hard rules forbid.  Used when
 * params->learned = 1 (expansions are then kept at order 8).  One model per process.
 * Parameter vector (FP32, 5768 floats, row-major [in][out]): W1 16x64 at 0, b1 at 1024,
 * W2 64x64 at 1088, b2 at 5184, W3 64x8 at 5248, b3 at 5760.  Features are normalised
 * as (x - mu) * isd before the first layer. */

/* Load a model file: "HFMMMAC1", int32 version (1), nfeat (16), hidden (64), nclass (8);
 * double theta_max, eps_label; int32 safety, reserved; float mu[16], isd[16],
 * params[5768], adam_m[5768], adam_v[5768]; int64 step; int32 length; JSON training
 * configuration.  path NULL unloads the model.  Weights are rounded to BF16 for the
 * selector's MFMA inference. */
int fmm_load_mac_model(const char *path);

/* Install a model from HOST arrays (params 5768, mu 16, isd 16); theta_max in (0, 0.75),
 * safety in [0, 6] orders added to the predicted order (capped at 8).  NULL params
 * unloads. */
int fmm_set_mac_model(const float *params, const float *mu, const float *isd, double theta_max, int safety);

/* Training data: on a built tree, export every candidate pair of a traversal with the
 * plain MAC of params (candidates: pass items 1 and 3, L/S_c <= theta_max) and label it
 * with the smallest order p in 2..8 whose error, measured by the library against the
 * exact pair force (FP64), satisfies max_i |a_i^(p) - a_i^direct| / |acc_ref_i| <= eps over
 * the sink's particles (class p - 1), else class 0.  acc_ref: DEVICE (n,3) total
 * short-range acceleration in caller order.  Only candidates whose (sink index + list
 * position) is a multiple of stride are labelled (stride >= 1, a deterministic subsample).
 * Outputs (DEVICE): feats (cap x 16 floats), labels (cap ints), errs (cap x 7 floats, per
 * order, may be NULL), pairs (cap x 3: sink cell key, source cell key, image; keys as in
 * fmm_copy_interactions; may be NULL).  *count (HOST) receives the number written (the
 * order of the records is not deterministic).  Pairs with n_A n_B > 2^18 are skipped. */
int fmm_mac_training_data(fmm_tree *tree, const fmm_params *params, double theta_max, const double *acc_ref,
                          double eps, int stride, float *feats, int *labels, float *errs, uint64_t *pairs,
                          int64_t cap, int64_t *count, void *stream);

/* FP32 forward pass of a parameter vector (DEVICE params, mu, isd, X (B x 16)) -> logits
 * (DEVICE B x 8). */
int fmm_mlp_forward(const float *params, const float *mu, const float *isd, const float *X, int B, float *logits,
                    void *stream);

/* Logits of the loaded model through the BF16 MFMA path used inside the traversal. */
int fmm_mlp_infer(const float *X, int B, float *logits, void *stream);

/* Gradient (DEVICE 5768 floats) and loss (DEVICE scalar) of the class-weighted softmax
 * cross-entropy, mean over the batch weighted by class_w (DEVICE 8 floats), of the
 * labels y (DEVICE B ints) for features X (DEVICE B x 16).  Synchronises the stream. */
int fmm_mlp_grad(const float *params, const float *mu, const float *isd, const float *X, const int *y,
                 const float *class_w, int B, float *grad, float *loss, void *stream);

/* fmm_mlp_grad for callers that cannot allocate device memory: code being recorded into a
 * HIP graph, training loops that must not call hipMalloc, harnesses that forbid it.  Same
 * arguments, kernels and result as fmm_mlp_grad (to FP32 rounding: the class-weight sum
 * is formed on the device), but it allocates nothing, synchronises nothing and reads
 * nothing back: the per-sample activations and gradients live in a fixed device array of
 * the library (9.4 MB per GPU, held until the process ends) sized for B <= 8192 samples;
 * a larger B is rejected with FMM_ERR_ARG.  The loss is cleared by a kernel, not a memset.
 * Labels outside [0, 8) get weight 0; if the weights of the batch's labels sum to 0 the
 * loss and gradient are 0 (fmm_mlp_grad returns FMM_ERR_ARG there).  Every call on a GPU
 * uses that GPU's one array: calls that overlap in time on one GPU (other streams or
 * threads) race and give wrong results; calls ordered on one stream do not. */
int fmm_mlp_grad_noalloc(const float *params, const float *mu, const float *isd, const float *X, const int *y,
                         const float *class_w, int B, float *grad, float *loss, void *stream);

/* One Adam step (DEVICE params, grad, m, v of 5768 floats), step >= 1 (bias correction).
 * weight_decay is a coupled L2 term: weight_decay * params is added to the gradient before
 * the moment updates (as torch.optim.Adam's weight_decay), not a decoupled (AdamW) decay. */
int fmm_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t step, float lr, float beta1,
                 float beta2, float eps, float weight_decay, void *stream);

/* Bound on the device memory the library's own buffers may hold, process-wide: trees and
 * their lists, forests, PM meshes, training scratch (not the caller's arrays, the FFT plans'
 * work areas, the selector model or the fixed scratch array of fmm_mlp_grad_noalloc).  0, the default, is no bound.  The buffers are kept
 * for reuse and freed only with their tree (PM meshes at exit), so the bound applies to
 * what they hold together.  A call that would grow a buffer past it fails with
 * FMM_ERR_NOMEM before allocating, as a failed device allocation does; a tree whose build
 * fails that way is left empty (rebuild it or free it).  Always returns 0. */
int fmm_set_memory_limit(uint64_t bytes);

/* Bytes the library's device buffers hold now (*bytes); FMM_ERR_ARG if bytes is NULL. */
int fmm_get_memory_use(uint64_t *bytes);

void fmm_free_tree(fmm_tree *tree);

/* Message of the last failed call on this thread ("" if none). */
const char *fmm_last_error(void);

/* Library version string. */
const char *fmm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HFMM_H */
