// Dual tree traversal with the modified multipole acceptance criterion (Sec. 2.3).
//
// The dual traversal from the root pairs visits a cell pair (A, B) iff its parent pair
// was opened, and every decision depends on (A, B, image) alone.  It can therefore be
// run sink level by sink level: the pairs that a sink A meets are those its parent
// handed down ("open the sink"), expanded on the source side ("open the source").
// Each sink emits its M2L sources, its P2P sources (both leaves) and the pairs it hands
// to its children.  The set of pairs is exactly that of the recursive traversal.
//
// GPU form: one 64-lane wave per sink (persistent waves pull sinks from a counter).
// The wave takes up to 64 pending pairs at a time, decides them in parallel, appends
// the emitted pairs with ballots, and pushes opened sources' children on a per-wave
// stack (last in, first out).  Lists are chains of 64-entry chunks taken from pools
// with an atomic counter, so one pass and no host round trip per level is needed; a
// pool or stack that runs out is detected (the counter keeps the exact demand) and the
// traversal is rerun with enough room.  Per-sink list order is deterministic.
#include <string.h>

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
    if (sm2 > cut2) return 0;
    double sc2 = R0 * R0 + R1 * R1 + R2 * R2;
    double G0 = A0 + half, G1 = A1 + half, G2 = A2 + half;
    double sM2 = G0 * G0 + G1 * G1 + G2 * G2;
    bool straddle = (mc.mode & 1) ? (sc2 > cut2) : (sM2 > cut2);
    if (straddle) return 2;
    double w = (mc.mode & 2) ? wb : fmax(wa, wb);
    if (4.0 * w * w <= mc.theta2 * sc2) return 1;
    return 2;
}

struct TravArgs {
    const Cell *cells;
    int lbeg, ln, ncell;
    uint32_t *items[3];
    int *next[3];
    int cap[3];
    int *pool;       // [3] chunk counters (chunks handed out, in blocks of kChunkBlock)
    int *head, *cnt; // [3][ncell]
    uint32_t *stack; // per-wave stacks when they do not fit in LDS
    int stk_cap;
    int *err;        // bit 0: stack overflow, bit 1: pool overflow
    unsigned long long *counters;  // [0] visits, [1] listed particle pairs (P2P kernel), [2] M2L, [3] P2P
};

constexpr int kChunkBlock = 16;   // chunks taken from a pool per atomic
constexpr int kLdsStack = 2048;   // entries of the in-LDS traversal stack

struct ListState {
    int head, cur, fill, tot;
};

// Next free chunk of list k.  Each wave takes kChunkBlock chunks per atomic and hands
// them out itself, so the pool counters see one atomic per 16 chunks.  All list state
// is wave-uniform and kept in scalar registers.
__device__ __forceinline__ int new_chunk(const TravArgs &a, int k, int *bnext, int *bend, int lane)
{
    if (bnext[k] == bend[k]) {
        int c = 0;
        if (lane == 0) c = atomicAdd(&a.pool[k], kChunkBlock);
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
// only when an entry needs them, so a chain never ends in an empty chunk.
__device__ __forceinline__ void emit(const TravArgs &a, int k, ListState &L, int *bnext, int *bend, bool pred,
                                     uint32_t item, uint64_t lt, int lane)
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
    if (pred && rank < room) a.items[k][(size_t)L.cur * kChunk + L.fill + rank] = item;
    if (m > room) {
        int c = new_chunk(a, k, bnext, bend, lane);
        if (lane == 0) a.next[k][L.cur] = c;
        L.cur = c;
        if (pred && rank >= room) a.items[k][(size_t)c * kChunk + rank - room] = item;
        L.fill = m - room;
    } else {
        L.fill += m;
    }
    L.tot += m;
}

__device__ __forceinline__ int wave_incl_scan(int v, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// Sinks t = blockIdx.x, blockIdx.x + gridDim.x, ... of one level.
template <bool GLOBAL_STACK>
__global__ __launch_bounds__(64) void k_traverse(TravArgs a, MacConst mc)
{
    __shared__ uint32_t lds_stack[GLOBAL_STACK ? 1 : kLdsStack];
    const int lane = threadIdx.x;
    const uint64_t lt = (1ull << lane) - 1ull;
    uint32_t *stk = GLOBAL_STACK ? a.stack + (size_t)blockIdx.x * a.stk_cap : lds_stack;
    const int scap = GLOBAL_STACK ? a.stk_cap : kLdsStack;
    const int4 *cell4 = reinterpret_cast<const int4 *>(a.cells);  // two int4 per cell
    unsigned long long visits = 0, nm2l = 0, np2p = 0;
    int bnext[3] = {0, 0, 0}, bend[3] = {0, 0, 0};
    for (int t = blockIdx.x; t < a.ln; t += gridDim.x) {
        const int A = a.lbeg + t;
        const int4 ga = cell4[2 * A];
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
        ListState Ls[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) Ls[k] = ListState{-1, -1, 0, 0};
        int sp = 0, ip = 0;
        bool failed = false;
        for (;;) {
            int kk;
            uint32_t it = 0;
            if (sp > 0) {
                kk = sp < 64 ? sp : 64;
                sp -= kk;
                if (lane < kk) it = stk[sp + lane];
            } else if (ip < ninh) {
                kk = ninh - ip < 64 ? ninh - ip : 64;
                if (lane < kk)
                    it = root ? ((uint32_t)A << 5 | (uint32_t)(ip + lane)) : a.items[2][(size_t)ichunk * kChunk + lane];
                ip += kk;
                if (!root && ip < ninh) ichunk = a.next[2][ichunk];
            } else {
                break;
            }
            visits += kk;
            const bool valid = lane < kk;
            int d = 0;
            int4 gb = make_int4(0, 0, 0, 0);
            const int B = (int)(it >> 5), s = (int)(it & 31);
            if (valid) {
                gb = cell4[2 * B];
                d = mac_decide(ga, gb, s, mc);
            }
            const int lvB = xln_level(gb.x);
            const bool leafB = xln_nchild(gb.x) == 0;
            bool is_m2l = d == 1;
            bool is_p2p = d == 2 && leafA && leafB;
            bool is_pd = d == 2 && !is_p2p && !leafA && (lvA <= lvB || leafB);
            bool open_src = d == 2 && !is_p2p && !is_pd;
            emit(a, 0, Ls[0], bnext, bend, is_m2l, it, lt, lane);
            emit(a, 1, Ls[1], bnext, bend, is_p2p, it, lt, lane);
            emit(a, 2, Ls[2], bnext, bend, is_pd, it, lt, lane);
            int nch = open_src ? xln_nchild(gb.x) : 0;
            int incl = wave_incl_scan(nch, lane);
            int tot = __builtin_amdgcn_readlane(incl, 63);
            if (tot > 0) {
                if (sp + tot > scap) {
                    if (lane == 0) atomicOr(a.err, 1);
                    failed = true;
                    break;
                }
                if (nch > 0) {
                    int off = sp + incl - nch;
                    for (int q = 0; q < nch; ++q) stk[off + q] = (uint32_t)(gb.w + q) << 5 | (uint32_t)s;
                }
                sp += tot;
                __syncthreads();  // pushes complete before the next pop reads them
            }
        }
        if (failed) continue;
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                a.head[k * a.ncell + A] = Ls[k].head;
                a.cnt[k * a.ncell + A] = Ls[k].tot;
            }
        }
        nm2l += Ls[0].tot;
        np2p += Ls[1].tot;
    }
    if (lane == 0) {
        atomicAdd(&a.counters[0], visits);
        atomicAdd(&a.counters[2], nm2l);
        atomicAdd(&a.counters[3], np2p);
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

constexpr int kTravWaves = 8192;

static int ensure_pools(fmm_tree *t, const int want[3])
{
    for (int k = 0; k < 3; ++k) {
        if (want[k] <= t->lcap[k]) continue;
        int cap = want[k] + want[k] / 4 + 64;
        if (int rc = grow(t->litems[k], (size_t)(cap + 1) * kChunk * 4) | grow(t->lnext[k], (size_t)(cap + 1) * 4))
            return rc;
        t->lcap[k] = cap;
    }
    return 0;
}

int traverse(fmm_tree *t, const fmm_params *P, hipStream_t st)
{
    MacConst mc;
    mac_setup(P, mc);
    const int ncell = t->ncell;
    int rc = grow(t->lhead, (size_t)3 * ncell * 4) | grow(t->lcnt, (size_t)3 * ncell * 4) | grow(t->counters, 256);
    if (rc) return rc;
    int want[3] = {2 * ncell + 64 * kChunkBlock, 8 * t->nleaf + 64 * kChunkBlock, 2 * ncell + 64 * kChunkBlock};
    if ((rc = ensure_pools(t, want))) return rc;
    for (int attempt = 0; attempt < 4; ++attempt) {
        int nw = 1;
        for (int l = 0; l < t->nlevel; ++l) {
            int ln = t->lvl_beg[l + 1] - t->lvl_beg[l];
            nw = ln > nw ? ln : nw;
        }
        nw = nw < kTravWaves ? nw : kTravWaves;
        if (t->global_stack && (rc = grow(t->tstack, (size_t)nw * t->stk_cap * 4))) return rc;
        // counters: [0..3] 64-bit stats, then int pool[3], err, sink counters per level
        unsigned char *cb = ptr<unsigned char>(t->counters);
        hipMemsetAsync(cb, 0, 256, st);
        hipMemsetAsync(t->lcnt.p, 0, (size_t)3 * ncell * 4, st);
        TravArgs a;
        a.cells = ptr<Cell>(t->cells);
        a.ncell = ncell;
        for (int k = 0; k < 3; ++k) {
            a.items[k] = ptr<uint32_t>(t->litems[k]);
            a.next[k] = ptr<int>(t->lnext[k]);
            a.cap[k] = t->lcap[k];
        }
        a.counters = reinterpret_cast<unsigned long long *>(cb);
        a.pool = reinterpret_cast<int *>(cb + 32);
        a.err = reinterpret_cast<int *>(cb + 44);
        a.head = ptr<int>(t->lhead);
        a.cnt = ptr<int>(t->lcnt);
        a.stack = ptr<uint32_t>(t->tstack);
        a.stk_cap = t->stk_cap;
        for (int l = 0; l < t->nlevel; ++l) {
            a.lbeg = t->lvl_beg[l];
            a.ln = t->lvl_beg[l + 1] - a.lbeg;
            int g = a.ln < nw ? a.ln : nw;
            if (t->global_stack) k_traverse<true><<<g, 64, 0, st>>>(a, mc);
            else k_traverse<false><<<g, 64, 0, st>>>(a, mc);
        }
        if ((rc = hip_check(hipGetLastError(), "traversal"))) return rc;
        hipMemcpyAsync(t->host, cb, 48, hipMemcpyDeviceToHost, st);
        if ((rc = hip_check(hipStreamSynchronize(st), "traversal sync"))) return rc;
        unsigned long long c64[4];
        int c32[4];
        memcpy(c64, t->host, 32);
        memcpy(c32, (char *)t->host + 32, 16);
        int err = c32[3];
        if (err == 0) {
            t->n_visit = (int64_t)c64[0];
            t->n_m2l = (int64_t)c64[2];
            t->n_p2p = (int64_t)c64[3];
            return 0;
        }
        if (err & 1) {  // LDS stack too small for this input: per-wave stacks in device memory
            if (t->global_stack) t->stk_cap *= 4;
            t->global_stack = true;
        }
        if (err & 2) {
            int need[3] = {c32[0], c32[1], c32[2]};
            if ((rc = ensure_pools(t, need))) return rc;
        }
    }
    return set_error(FMM_ERR_NOMEM, "traversal did not fit after resizing");
}

}  // namespace hfmm
