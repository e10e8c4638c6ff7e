// Dual tree traversal with the modified multipole acceptance criterion (Sec. 2.3).
//
// The dual traversal from the root pairs visits a cell pair (A, B) iff its parent pair
// was opened, and every decision depends on (A, B, image) alone.  It can therefore be
// run sink level by sink level: the pairs that a sink A meets are those its parent
// handed down ("open the sink"), expanded on the source side ("open the source").
// Each sink emits its M2L sources, its P2P sources (both leaves) and the pairs it hands
// to its children.  The set of pairs is exactly that of the recursive traversal.
//
// GPU form: one 64-lane wave per sink; a level's sinks are dealt round robin to a grid of
// as many waves as fit on the device at once.
// The wave takes up to 64 pending pairs at a time, decides them in parallel, appends
// the emitted pairs with ballots, and pushes opened sources' children on a per-wave
// stack (last in, first out).  Lists are chains of 64-entry chunks taken from pools
// with an atomic counter, so one pass and no host round trip per level is needed; a
// pool or stack that runs out is detected (the counter keeps the exact demand) and the
// traversal is rerun with enough room.  Per-sink list order is deterministic.
#include <string.h>

#include "mlp.h"
#include "state.h"

namespace hfmm {

// 0 = neglect (item 1), 1 = M2L (item 2), 2 = open (item 3 or item 2 failed).
// Distances are integers in units of u = box / 2^(l+1), l the finer level: every
// separation is below 2^23 and every squared distance below 2^50, so double precision
// holds them exactly and the comparisons are exact.
__device__ __forceinline__ int mac_decide(int4 a, int4 b, int s, const MacConst &mc)
{
    int la = xln_level(a.x), lb = xln_level(b.x);
    int l = la > lb ? la : lb;
    double wa = (double)(1 << (l - la)), wb = (double)(1 << (l - lb));
    double half = wa + wb, img = (double)(2 << l);
    double sh0 = (double)(s / 9 - 1), sh1 = (double)((s / 3) % 3 - 1), sh2 = (double)(s % 3 - 1);
    double R0 = (2.0 * xln_ix(a.x) + 1.0) * wa - (2.0 * xln_ix(b.x) + 1.0) * wb - sh0 * img;
    double R1 = (2.0 * a.y + 1.0) * wa - (2.0 * b.y + 1.0) * wb - sh1 * img;
    double R2 = (2.0 * a.z + 1.0) * wa - (2.0 * b.z + 1.0) * wb - sh2 * img;
    double A0 = fabs(R0), A1 = fabs(R1), A2 = fabs(R2);
    double g0 = fmax(A0 - half, 0.0), g1 = fmax(A1 - half, 0.0), g2 = fmax(A2 - half, 0.0);
    double sm2 = g0 * g0 + g1 * g1 + g2 * g2;
    double cut2 = ldexp(mc.cut2[0], 2 * l);  // equals (r_cut / u_l)^2 exactly
    double sc2 = R0 * R0 + R1 * R1 + R2 * R2;
    if (!(mc.mode & 4)) {  // truncated MAC; mode bit 2: conventional MAC, item 2 alone
        if (sm2 > cut2) return 0;
        double G0 = A0 + half, G1 = A1 + half, G2 = A2 + half;
        double sM2 = G0 * G0 + G1 * G1 + G2 * G2;
        bool straddle = (mc.mode & 1) ? (sc2 > cut2) : (sM2 > cut2);
        if (straddle) return 2;
    }
    double w = (mc.mode & 2) ? wb : fmax(wa, wb);
    if (4.0 * w * w <= mc.theta2 * sc2) return 1;
    return 2;
}

// Traversal modes: plain MAC; plain MAC plus export of candidate pairs; learned selector.
enum { kModePlain = 0, kModeExport = 1, kModeLearned = 2 };

struct TravArgs {
    const Cell *cells;
    int lbeg, ln, ncell;
    uint32_t *items[kKinds];
    int *next[kKinds];
    int cap[kKinds];
    int *pool;       // chunk counter of list kind k at pool[k * kPoolStride] (chunks handed out)
    int *wstate;     // per wave w: [kKinds] next chunk, [kKinds] end of its block, kept across levels
    int *head, *cnt; // [kKinds][ncell]
    unsigned char *ord;  // kind kKindOrd: the M2L order of each entry
    int *ocnt;           // learned: entries of order o of sink c at ocnt[(o - 2) * ncell + c]
    uint32_t *stack; // per-wave stacks when they do not fit in LDS
    int stk_cap;
    int *err;        // bit 0: stack overflow, bit 1: pool overflow
    unsigned long long *counters;  // [0] visits, [1] listed particle pairs (P2P kernel), [2] M2L, [3] P2P
    // candidate pairs / learned selector
    double theta_max2;             // candidates have (L/S_c)^2 <= theta_max2
    double box, rs, rcut;
    const float4 *cf;              // learned: per-cell part of the features (cell_features)
    const MacModel *model;
    const int4 *cellc;  // the first 16 bytes of every cell, packed (what the traversal reads)
};

constexpr int kChunkBlock = 32;   // chunks taken from a pool per atomic
constexpr int kPoolStride = 32;   // ints between the pool counters (one 128-byte line each)
constexpr int kCandQ = 128;       // learned: ring of candidate pairs (at most 63 wait between steps)

struct ListState {
    int head, cur, fill, tot;
};

// Next free chunk of list k.  Each wave takes kChunkBlock chunks per atomic and hands
// them out itself; the unused rest of its block passes to the wave with the same index
// in the next level's launch.  So the counters see one atomic per kChunkBlock chunks and
// no burst when a level starts (same-address atomics are serialised in the L2).  All
// list state is wave-uniform and kept in scalar registers.
__device__ __forceinline__ int new_chunk(const TravArgs &a, int k, int *bnext, int *bend, int lane)
{
    if (bnext[k] == bend[k]) {
        int c = 0;
        if (lane == 0) c = atomicAdd(&a.pool[k * kPoolStride], kChunkBlock);
        c = __builtin_amdgcn_readfirstlane(c);
        bnext[k] = c;
        bend[k] = c + kChunkBlock;
    }
    int c = bnext[k]++;
    if (c >= a.cap[k]) {  // out of room: write into the spare chunk, report, rerun later
        if (lane == 0) atomicOr(a.err, 2);
        c = a.cap[k];
    }
    return c;
}

// Append `item` of every lane with `pred` to list k, in lane order.  Chunks are taken
// only when an entry needs them, so a chain never ends in an empty chunk.  ORD: the
// byte `ob` is stored beside the entry (list kind kKindOrd).
template <bool ORD = false>
__device__ __forceinline__ void emit(const TravArgs &a, int k, ListState &L, int *bnext, int *bend, bool pred,
                                     uint32_t item, uint64_t lt, int lane, unsigned char ob = 0)
{
    uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    int m = __popcll(mask);
    int rank = __popcll(mask & lt);
    if (L.cur < 0 || L.fill == kChunk) {
        int c = new_chunk(a, k, bnext, bend, lane);
        if (L.cur < 0) L.head = c;
        else if (lane == 0) a.next[k][L.cur] = c;
        L.cur = c;
        L.fill = 0;
    }
    int room = kChunk - L.fill;
    if (pred && rank < room) {
        const size_t at = (size_t)L.cur * kChunk + L.fill + rank;
        a.items[k][at] = item;
        if (ORD) a.ord[at] = ob;
    }
    if (m > room) {
        int c = new_chunk(a, k, bnext, bend, lane);
        if (lane == 0) a.next[k][L.cur] = c;
        L.cur = c;
        if (pred && rank >= room) {
            const size_t at = (size_t)c * kChunk + rank - room;
            a.items[k][at] = item;
            if (ORD) a.ord[at] = ob;
        }
        L.fill = m - room;
    } else {
        L.fill += m;
    }
    L.tot += m;
}

// Full MAC evaluation for the candidate logic: code as mac_decide, plus whether item 3
// forced the opening and (L / S_c)^2.
struct MacEval {
    int code;
    bool straddle;
    double q2;
};

__device__ __forceinline__ MacEval mac_eval(int4 a, int4 b, int s, const MacConst &mc)
{
    MacEval r;
    PairGeo g = pair_geo(a, b, s);
    double cut2 = ldexp(mc.cut2[0], 2 * g.l);
    double w = (mc.mode & 2) ? g.wb : fmax(g.wa, g.wb);
    r.q2 = 4.0 * w * w / g.sc2;
    r.straddle = false;
    if (!(mc.mode & 4)) {  // truncated MAC; mode bit 2: conventional MAC, item 2 alone
        if (g.sm2 > cut2) {
            r.code = 0;
            return r;
        }
        r.straddle = (mc.mode & 1) ? (g.sc2 > cut2) : (g.sM2 > cut2);
        if (r.straddle) {
            r.code = 2;
            return r;
        }
    }
    r.code = (4.0 * w * w <= mc.theta2 * g.sc2) ? 1 : 2;
    return r;
}

// Sinks t = blockIdx.x, blockIdx.x + gridDim.x, ... of one level.
template <int MODE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MODE == kModeLearned ? 3 : 4))) void k_traverse(TravArgs a, MacConst mc)
{
    __shared__ short mlp_act[MODE == kModeLearned ? 64 * 64 : 1];
    __shared__ uint32_t cand_q[MODE == kModeLearned ? kCandQ : 1];

    const int lane = threadIdx.x;
    const uint64_t lt = (1ull << lane) - 1ull;
    // per-wave stack of pairs still to decide, in device memory (L2 resident); measured as
    // fast as an LDS stack, and it leaves the LDS to the learned selector
    uint32_t *stk = a.stack + (size_t)blockIdx.x * a.stk_cap;
    const int scap = a.stk_cap;
    const int4 *cellc = a.cellc;
    unsigned long long visits = 0, nm2l = 0, np2p = 0;
    unsigned nord[kOrders] = {0, 0, 0, 0, 0, 0, 0};  // learned: this wave's M2L pairs per order
    int bnext[kKinds], bend[kKinds];
    int *ws = a.wstate + (size_t)blockIdx.x * 2 * kKinds;
#pragma unroll
    for (int k = 0; k < kKinds; ++k) {
        bnext[k] = __builtin_amdgcn_readfirstlane(ws[k]);
        bend[k] = __builtin_amdgcn_readfirstlane(ws[kKinds + k]);
    }
    for (int t = xcd_order(blockIdx.x, gridDim.x); t < a.ln; t += gridDim.x) {
        const int A = a.lbeg + t;
        const int4 ga = cellc[A];
        const int parentA = a.cells[A].parent;
        const bool leafA = xln_nchild(ga.x) == 0;
        const int lvA = xln_level(ga.x);
        const bool root = lvA == 0;  // a root meets the 27 periodic images of itself
        int ninh = 27, ichunk = 0;
        if (root && a.cells[A].end == a.cells[A].beg) ninh = 0;  // empty box of a batch: nothing to do
        if (!root) {
            ninh = a.cnt[2 * a.ncell + parentA];
            ichunk = a.head[2 * a.ncell + parentA];
        }
        double mA0 = 0.0;
        if (MODE == kModeLearned) mA0 = a.cf[A].x;
        ListState Ls[kKinds];
#pragma unroll
        for (int k = 0; k < kKinds; ++k) Ls[k] = ListState{-1, -1, 0, 0};
        unsigned oc[kOrders] = {0, 0, 0, 0, 0, 0, 0};  // learned: this sink's M2L pairs per order
        int sp = 0;
        int qhead = 0, qtail = 0;  // learned: queue of candidate pairs awaiting the selector
        bool failed = false;
        // the inherited pairs go onto the stack first, so every step takes a full batch of
        // 64 while that many are pending (opened sources push their children on top)
        if (ninh > scap) {
            if (lane == 0) atomicOr(a.err, 1);
            continue;
        }
        if (root) {
            if (lane < ninh) stk[lane] = (uint32_t)A << 5 | (uint32_t)lane;
        } else {
            for (int e0 = 0; e0 < ninh; e0 += kChunk) {
                if (e0 > 0) ichunk = a.next[2][ichunk];
                if (e0 + lane < ninh) stk[e0 + lane] = a.items[2][(size_t)ichunk * kChunk + lane];
            }
        }
        sp = ninh;
        __syncthreads();  // the copied entries are written before they are popped

        // Lists and stack for decided pairs of the lanes with `valid`: `m2l_ord` >= 2 puts
        // the pair on an M2L list (order m2l_ord in learned mode, else plain), `opened`
        // hands it to P2P, to the children of A, or opens the source.  Returns false if
        // the stack overflowed.
        auto finish = [&](bool valid, uint32_t it, int4 gb, int m2l_ord, bool opened) __attribute__((always_inline))
            -> bool {
            const int lvB = xln_level(gb.x);
            const bool leafB = xln_nchild(gb.x) == 0;
            const bool is_m2l = valid && m2l_ord >= 2;
            opened = valid && opened;
            const bool is_p2p = opened && leafA && leafB;
            const bool is_pd = opened && !is_p2p && !leafA && (lvA <= lvB || leafB);
            const bool open_src = opened && !is_p2p && !is_pd;
            if (MODE == kModeLearned) {
                emit<true>(a, kKindOrd, Ls[kKindOrd], bnext, bend, is_m2l, it, lt, lane, (unsigned char)m2l_ord);
            } else {
                emit(a, 0, Ls[0], bnext, bend, is_m2l, it, lt, lane);
            }
            emit(a, 1, Ls[1], bnext, bend, is_p2p, it, lt, lane);
            emit(a, 2, Ls[2], bnext, bend, is_pd, it, lt, lane);
            const int nch = open_src ? xln_nchild(gb.x) : 0;
            const int incl = wave_incl_sum(nch);
            const int tot = __builtin_amdgcn_readlane(incl, 63);
            if (tot > 0) {
                if (sp + tot > scap) {
                    if (lane == 0) atomicOr(a.err, 1);
                    return false;
                }
                if (nch > 0) {
                    const int off = sp + incl - nch;
                    const int s = (int)(it & 31);
                    for (int q = 0; q < nch; ++q) stk[off + q] = (uint32_t)(gb.w + q) << 5 | (uint32_t)s;
                }
                sp += tot;
                __syncthreads();  // pushes complete before the next pop reads them
            }
            return true;
        };

        for (;;) {
            // next batch: a flush of the candidate queue (learned: when 64 wait, or when
            // nothing else is left), else up to 64 pairs from the stack
            int kk = 0, fk = 0;
            uint32_t it = 0;
            if (MODE == kModeLearned && qtail - qhead >= 64) {
                fk = 64;
            } else if (sp > 0) {
                kk = sp < 64 ? sp : 64;
                sp -= kk;
                if (lane < kk) it = stk[sp + lane];
            } else if (MODE == kModeLearned && qtail > qhead) {
                fk = qtail - qhead;
            } else {
                break;
            }
            bool valid, opened;
            int ord;
            int4 gb = make_int4(0, 0, 0, 0);
            if (MODE == kModeLearned && fk > 0) {
                // the selector decides fk queued candidates at once (features, MLP on the
                // matrix cores, order decoding); not accepted means opened
                __syncthreads();  // queued entries are written before other lanes read them
                valid = lane < fk;
                it = valid ? cand_q[(qhead + lane) & (kCandQ - 1)] : 0u;
                qhead += fk;
                const int B = (int)(it >> 5), s = (int)(it & 31);
                float fv[kFeat];
                for (int q = 0; q < kFeat; ++q) fv[q] = 0.0f;
                if (valid) {
                    gb = cellc[B];
                    PairGeo g = pair_geo(ga, gb, s);
                    pair_features(g, lvA, xln_level(gb.x), a.box, a.rs, a.rcut, mA0, a.cf[B], fv);
                }
                float lg[kCls];
                mlp_logits_wave(a.model->w, fv, mlp_act, lg);
                ord = valid ? decode_order(lg, a.model->safety) : 0;
                opened = ord < 2;
#pragma unroll
                for (int o = 0; o < kOrders; ++o) oc[o] += __popcll(__ballot(valid && ord == o + 2));
            } else {
                visits += kk;
                valid = lane < kk;
                int d = 0;
                bool cand = false;
                const int B = (int)(it >> 5), s = (int)(it & 31);
                if (valid) {
                    gb = cellc[B];
                    if (MODE == kModePlain) {
                        d = mac_decide(ga, gb, s, mc);
                    } else {
                        MacEval ev = mac_eval(ga, gb, s, mc);
                        d = ev.code;
                        cand = d != 0 && !ev.straddle && ev.q2 <= a.theta_max2;
                    }
                }
                if (MODE == kModeExport) emit(a, kKindCand, Ls[kKindCand], bnext, bend, cand, it, lt, lane);
                if (MODE == kModeLearned) {
                    // candidates wait in the queue; the rest are pruned (d = 0) or opened
                    const uint64_t cm = __ballot(cand);
                    if (cand) cand_q[(qtail + __popcll(cm & lt)) & (kCandQ - 1)] = it;
                    qtail += __popcll(cm);
                    valid = valid && !cand;
                    ord = 0;
                    opened = d != 0;
                } else {
                    ord = d == 1 ? 2 : 0;
                    opened = d == 2;
                }
            }
            if (!finish(valid, it, gb, ord, opened)) {
                failed = true;
                break;
            }
        }
        if (failed) continue;
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < kKinds; ++k) {
                a.head[k * a.ncell + A] = Ls[k].head;
                a.cnt[k * a.ncell + A] = Ls[k].tot;
            }
        }
        if (MODE == kModeLearned) {
            nm2l += Ls[kKindOrd].tot;
#pragma unroll
            for (int o = 0; o < kOrders; ++o) {
                if (lane == 0) a.ocnt[(size_t)o * a.ncell + A] = (int)oc[o];
                nord[o] += oc[o];
            }
        } else {
            nm2l += Ls[0].tot;
        }
        np2p += Ls[1].tot;
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < kKinds; ++k) {
            ws[k] = bnext[k];
            ws[kKinds + k] = bend[k];
        }
        atomicAdd(&a.counters[0], visits);
        atomicAdd(&a.counters[2], nm2l);
        atomicAdd(&a.counters[3], np2p);
        if (MODE == kModeLearned)
            for (int k = 0; k < kOrders; ++k) atomicAdd(&a.counters[16 + k], (unsigned long long)nord[k]);
    }
}

void mac_setup(const fmm_params *P, MacConst &mc)
{
    for (int l = 0; l <= kMaxLevel; ++l) {
        double u = ldexp(P->box, -(l + 1));
        mc.cut2[l] = (P->r_cut * P->r_cut) / (u * u);
    }
    mc.theta2 = P->theta * P->theta;
    mc.mode = P->mac_mode;
    mc.pad = 0;
}

// Waves of one traversal kernel that fit on the device at once.  Sinks are dealt to the
// waves statically, so the grid is never larger than this: a second partial round of
// waves would only lengthen the tail of each level.
template <int MODE> static int resident_waves()
{
    static int cached = 0;
    if (cached == 0) {
        int dev = 0, ncu = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_traverse<MODE>, 64, 0) != hipSuccess)
            return 4096;
        cached = (ncu > 0 ? ncu : 1) * (per > 0 ? per : 1);
    }
    return cached;
}

static int resident_waves(int mode)
{
    if (mode == kModePlain) return resident_waves<kModePlain>();
    if (mode == kModeExport) return resident_waves<kModeExport>();
    return resident_waves<kModeLearned>();
}

// The traversal's 16-byte view of each cell, packed: the random cell reads of the traversal
// then touch half as many cache lines (8 sibling cells per 128-byte line).
__global__ void k_pack_cells(const Cell *__restrict__ cells, int ncell, int4 *__restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncell) out[c] = reinterpret_cast<const int4 *>(cells)[2 * (size_t)c];
}

// Per-cell part of the selector's features, from the scaled multipoles (stride `stride`).
template <class T>
__global__ void k_cell_features(const T *__restrict__ M, int stride, int ncell, float4 *__restrict__ cf)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncell) cf[c] = cell_features<T>(M + (size_t)c * stride);
}

constexpr int kPoolByte = 256;
constexpr int kCounterBytes = kPoolByte + kKinds * kPoolStride * 4;
static_assert(kCounterBytes <= kHostInts * 4, "counter readback exceeds the pinned area");

// Wave w starts with chunks [w kChunkBlock, (w+1) kChunkBlock) of every list kind, and
// the counters start past those blocks: no wave needs an atomic for its first block.
__global__ void k_wstate_init(int *ws, int nw, int *pool)
{
    int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < nw)
        for (int k = 0; k < kKinds; ++k) {
            ws[(size_t)w * 2 * kKinds + k] = w * kChunkBlock;
            ws[(size_t)w * 2 * kKinds + kKinds + k] = (w + 1) * kChunkBlock;
        }
    if (w == 0)
        for (int k = 0; k < kKinds; ++k) pool[k * kPoolStride] = nw * kChunkBlock;
}

static int ensure_pools(fmm_tree *t, const int *want)
{
    for (int k = 0; k < kKinds; ++k) {
        if (want[k] <= t->lcap[k]) continue;
        int cap = want[k] + want[k] / 4 + 64;
        if (int rc = grow(t->litems[k], (size_t)(cap + 1) * kChunk * 4) | grow(t->lnext[k], (size_t)(cap + 1) * 4))
            return rc;
        if (k == kKindOrd)
            if (int rc = grow(t->lord, (size_t)(cap + 1) * kChunk)) return rc;
        t->lcap[k] = cap;
    }
    return 0;
}

// mode: kModePlain / kModeExport / kModeLearned.  For the last two, theta_max bounds the
// candidates, M/mstride/mprec give the multipoles used by the features, model the
// selector (learned only).
int traverse_mode(fmm_tree *t, const fmm_params *P, int mode, double theta_max, const void *M, int mstride,
                  int mprec, const MacModel *model, hipStream_t st, const TravHook *hook)
{
    MacConst mc;
    mac_setup(P, mc);
    const int ncell = t->ncell;
    // lcnt: kKinds list sizes, then the learned selector's per-order counts
    const size_t ncnt = (size_t)(kKinds + (mode == kModeLearned ? kOrders : 0)) * ncell;
    int rc = grow(t->lhead, (size_t)kKinds * ncell * 4) | grow(t->lcnt, (size_t)(kKinds + kOrders) * ncell * 4) |
             grow(t->counters, kCounterBytes);
    if (rc) return rc;
    // list kinds written in this mode get room for their expected size plus the partly
    // used chunk block each wave may hold at the end
    int want[kKinds];
    const int slack = resident_waves(mode) * kChunkBlock + 64;
    for (int k = 0; k < kKinds; ++k) want[k] = 0;
    want[1] = slack + 8 * t->nleaf;
    want[2] = slack + 2 * ncell;
    if (mode == kModeLearned) {
        want[kKindOrd] = slack + 4 * ncell;
    } else {
        want[0] = slack + 2 * ncell;
        if (mode == kModeExport) want[kKindCand] = slack + 2 * ncell;
    }
    if ((rc = ensure_pools(t, want))) return rc;
    if ((rc = grow(t->cellc, (size_t)ncell * sizeof(int4)))) return rc;
    k_pack_cells<<<(ncell + 255) / 256, 256, 0, st>>>(ptr<Cell>(t->cells), ncell, ptr<int4>(t->cellc));
    if (mode == kModeLearned) {
        if (!M || mstride < 20) return set_error(FMM_ERR_ARG, "learned traversal: multipoles of order >= 3 needed");
        if ((rc = grow(t->cfeat, (size_t)ncell * sizeof(float4)))) return rc;
        if (mprec)
            k_cell_features<float><<<(ncell + 63) / 64, 64, 0, st>>>(static_cast<const float *>(M), mstride, ncell,
                                                                    ptr<float4>(t->cfeat));
        else
            k_cell_features<double><<<(ncell + 63) / 64, 64, 0, st>>>(static_cast<const double *>(M), mstride, ncell,
                                                                     ptr<float4>(t->cfeat));
    }
    for (int attempt = 0; attempt < 4; ++attempt) {
        int nw = 1;
        for (int l = 0; l < t->nlevel; ++l) {
            int ln = t->lvl_beg[l + 1] - t->lvl_beg[l];
            nw = ln > nw ? ln : nw;
        }
        // measured: below about a million cells the plain traversal runs faster on two
        // thirds of the resident waves (2M box 3.05 -> 2.83 ms, 64-box forest 3.47 -> 3.23 ms;
        // the upward pass shares the GPU), above it on all of them (16.7M box 14.6 ms on all,
        // 17.6 ms on two thirds)
        const int cap = mode == kModePlain && ncell < (1 << 20) ? resident_waves(mode) * 2 / 3 : resident_waves(mode);
        nw = nw < cap ? nw : cap;
        if ((rc = grow(t->tstack, (size_t)nw * t->stk_cap * 4))) return rc;
        if ((rc = grow(t->wstate, (size_t)nw * 2 * kKinds * sizeof(int)))) return rc;
        // counters: [0..3] 64-bit stats, err at byte 96, 64-bit M2L counts per learned order
        // at byte 128, P2P evaluated pairs at byte 192, pool counters from byte kPoolByte
        unsigned char *cb = ptr<unsigned char>(t->counters);
        if ((rc = zero_async(cb, kCounterBytes, st))) return rc;  // a kernel: also valid inside a recorded graph
        k_wstate_init<<<(nw + 255) / 256, 256, 0, st>>>(ptr<int>(t->wstate), nw,
                                                        reinterpret_cast<int *>(cb + kPoolByte));
        if ((rc = zero_async(t->lcnt.p, ncnt * 4, st))) return rc;
        TravArgs a;
        a.cells = ptr<Cell>(t->cells);
        a.ncell = ncell;
        for (int k = 0; k < kKinds; ++k) {
            a.items[k] = ptr<uint32_t>(t->litems[k]);
            a.next[k] = ptr<int>(t->lnext[k]);
            a.cap[k] = t->lcap[k];
        }
        a.counters = reinterpret_cast<unsigned long long *>(cb);
        a.pool = reinterpret_cast<int *>(cb + kPoolByte);
        a.wstate = ptr<int>(t->wstate);
        a.err = reinterpret_cast<int *>(cb + 96);
        a.head = ptr<int>(t->lhead);
        a.cnt = ptr<int>(t->lcnt);
        a.ord = ptr<unsigned char>(t->lord);
        a.ocnt = ptr<int>(t->lcnt) + (size_t)kKinds * ncell;
        a.stack = ptr<uint32_t>(t->tstack);
        a.stk_cap = t->stk_cap;
        a.theta_max2 = theta_max * theta_max;
        a.box = P->box;
        a.rs = P->r_s;
        a.rcut = P->r_cut;
        a.cf = ptr<float4>(t->cfeat);
        a.model = model;
        a.cellc = ptr<int4>(t->cellc);
        for (int l = 0; l < t->nlevel; ++l) {
            a.lbeg = t->lvl_beg[l];
            a.ln = t->lvl_beg[l + 1] - a.lbeg;
            int g = a.ln < nw ? a.ln : nw;
            if (mode == kModePlain) k_traverse<kModePlain><<<g, 64, 0, st>>>(a, mc);
            else if (mode == kModeExport) k_traverse<kModeExport><<<g, 64, 0, st>>>(a, mc);
            else k_traverse<kModeLearned><<<g, 64, 0, st>>>(a, mc);
            if (hook)
                if ((rc = hook->level(hook->ctx, l, st))) return rc;
        }
        if ((rc = hip_check(hipGetLastError(), "traversal"))) return rc;
        // Being recorded: the tree and parameters are those of the evaluation just run, whose
        // pools and stacks fitted; the lists, their sizes and every wave's use of pool blocks
        // and stack (sinks are dealt statically) repeat exactly, so no readback is needed.
        if (t->capturing) return 0;
        if ((rc = hip_check(hipMemcpyAsync(t->host, cb, kCounterBytes, hipMemcpyDeviceToHost, st), "counters")))
            return rc;
        if ((rc = hip_check(hipStreamSynchronize(st), "traversal sync"))) return rc;
        unsigned long long c64[4];
        int pools[kKinds], err;
        memcpy(c64, t->host, 32);
        for (int k = 0; k < kKinds; ++k)  // kinds this mode does not write keep their size
            pools[k] = want[k] ? t->host[kPoolByte / 4 + k * kPoolStride] : 0;
        memcpy(&err, (char *)t->host + 96, 4);
        if (err == 0) {
            unsigned long long ord[kOrders];
            memcpy(ord, (char *)t->host + 128, sizeof(ord));
            for (int k = 0; k < kOrders; ++k) t->stats.n_m2l_by_order[k] = mode == kModeLearned ? (int64_t)ord[k] : 0;
            t->n_visit = (int64_t)c64[0];
            t->n_m2l = (int64_t)c64[2];
            t->n_p2p = (int64_t)c64[3];
            t->trav_mode = mode;
            return 0;
        }
        // what the hook launched read the counters the rerun clears: let it end first
        if (hook && hook->side)
            if ((rc = hip_check(hipStreamSynchronize(hook->side), "traversal side stream"))) return rc;
        if (err & 1) t->stk_cap *= 4;  // a wave's stack overflowed: larger stacks, rerun
        if (err & 2)
            if ((rc = ensure_pools(t, pools))) return rc;
    }
    return set_error(FMM_ERR_NOMEM, "traversal did not fit after resizing");
}

int traverse(fmm_tree *t, const fmm_params *P, hipStream_t st, const TravHook *hook)
{
    return traverse_mode(t, P, kModePlain, 0.0, nullptr, 0, 0, nullptr, st, hook);
}

}  // namespace hfmm
