// Stage entry points of the expansion operators: precision dispatch.  The kernels are
// in expand_impl.h and are instantiated in expand_f32.hip and expand_f64.hip.
#include "state.h"

namespace hfmm {
template <class T> int upward_t(fmm_tree *t, int p, hipStream_t st);
template <class T>
int m2l_t(fmm_tree *t, int p, Split sp, int learned, int pstore, int accumulate, int mfma, int det, hipStream_t st);

static Split split_of(const fmm_params *P) { return Split{P->split ? P->r_cut : P->r_s, P->split}; }
static int flatten_learned(fmm_tree *t, hipStream_t st);
template <class T> int l2l_t(fmm_tree *t, int p, hipStream_t st);
template <class T> int l2p_t(fmm_tree *t, int p, double G, double *acc, int accumulate, hipStream_t st);

int upward(fmm_tree *t, const fmm_params *P, hipStream_t st)
{
    return P->precision ? upward_t<float>(t, P->p, st) : upward_t<double>(t, P->p, st);
}

// The FP32 M2L kernel: fmm_params.m2l_mfma 2 = matrix cores for same-level pairs, 1 = vector
// ALUs, 0 = the library's choice (the vector ALUs).
static int use_mfma(const fmm_params *P) { return P->m2l_mfma == 2; }

// deterministic mode: the thread-per-sink kernel, which sums each sink's pairs in list
// order in registers (no atomics)
int m2l(fmm_tree *t, const fmm_params *P, hipStream_t st)
{
    return P->precision ? m2l_t<float>(t, P->p, split_of(P), 0, P->p, 0, use_mfma(P), P->deterministic, st)
                        : m2l_t<double>(t, P->p, split_of(P), 0, P->p, 0, 0, P->deterministic, st);
}

// Learned selector: coefficients stored at order 8; the pairs accepted at order o are
// contracted at that order and added up.
int m2l_learned(fmm_tree *t, const fmm_params *P, hipStream_t st)
{
    if (int rc = zero_async(t->Lc.p, (size_t)t->ncell * ncoef(8) * (P->precision ? 4 : 8), st)) return rc;
    if (!P->deterministic)
        if (int rc = flatten_learned(t, st)) return rc;
    for (int o = 2; o <= 8; ++o) {
        int rc = P->precision ? m2l_t<float>(t, o, split_of(P), 1, 8, 1, 0, P->deterministic, st)
                              : m2l_t<double>(t, o, split_of(P), 1, 8, 1, 0, P->deterministic, st);
        if (rc) return rc;
    }
    return 0;
}

// Flattens the chunked M2L list of `kind` into (sink, item) pairs, each sink's pairs
// contiguous (the pair kernel reduces runs of one sink; the order of the sinks is free).
// A wave takes 64 sinks: a wave scan of their list sizes, one atomic reservation of the
// total in the output, then each sink's chunks are copied 64 items at a time.  `npair`
// (the list total counted by the traversal) bounds every write.
__global__ __launch_bounds__(64) void k_flatten_pairs(const int *__restrict__ head, const int *__restrict__ cnt,
                                                      const uint32_t *__restrict__ items, const int *__restrict__ next,
                                                      int ncell, int *__restrict__ ctr, int2 *__restrict__ out,
                                                      int npair)
{
    const int lane = threadIdx.x;
    for (int A0 = blockIdx.x * 64; A0 < ncell; A0 += gridDim.x * 64) {
        const int A = A0 + lane;
        const int nl = A < ncell ? cnt[A] : 0;
        const int hd = nl > 0 ? head[A] : 0;
        const int incl = wave_incl_sum(nl);
        const int total = __builtin_amdgcn_readlane(incl, 63);
        if (total == 0) continue;
        int base = 0;
        if (lane == 63) base = atomicAdd(ctr, total);
        base = __shfl(base, 63, 64);
        const int excl = incl - nl;
        for (int j = 0; j < 64; ++j) {
            const int nj = __shfl(nl, j, 64);
            if (nj == 0) continue;
            const int oj = base + __shfl(excl, j, 64);
            int chunk = __shfl(hd, j, 64);
            for (int e0 = 0; e0 < nj; e0 += kChunk) {
                if (e0 > 0) chunk = next[chunk];
                const int e = e0 + lane, o = oj + e;
                if (e < nj && o < npair) out[o] = make_int2(A0 + j, (int)items[(size_t)chunk * kChunk + lane]);
            }
        }
    }
}

// The learned selector's list (entries of mixed order, the order in a byte beside each)
// as (sink, item) pairs in one segment per order, each sink's pairs of one order
// contiguous.  A wave takes 64 sinks: per order, a wave scan of the sinks' counts and one
// atomic reservation in that order's segment; then each sink's chunks are copied, every
// entry to the next place of its order (lane rank among the chunk's entries of that
// order).  seg/nseg bound every write.
struct OrderSegs {
    long long seg[kOrders], n[kOrders];
};

__global__ __launch_bounds__(64) void k_flatten_learned(const int *__restrict__ head, const int *__restrict__ cnt,
                                                        const int *__restrict__ ocnt, const uint32_t *__restrict__ items,
                                                        const unsigned char *__restrict__ ord,
                                                        const int *__restrict__ next, int ncell, int *__restrict__ ctr,
                                                        OrderSegs sg, int2 *__restrict__ out)
{
    const int lane = threadIdx.x;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int A0 = blockIdx.x * 64; A0 < ncell; A0 += gridDim.x * 64) {
        const int A = A0 + lane;
        const int nl = A < ncell ? cnt[A] : 0;
        if (__ballot(nl > 0) == 0) continue;
        const int hd = nl > 0 ? head[A] : 0;
        int excl[kOrders], base[kOrders];
#pragma unroll
        for (int o = 0; o < kOrders; ++o) {
            const int c = nl > 0 ? ocnt[(size_t)o * ncell + A] : 0;
            const int incl = wave_incl_sum(c);
            excl[o] = incl - c;
            const int total = __builtin_amdgcn_readlane(incl, 63);
            int b = 0;
            if (lane == 63 && total > 0) b = atomicAdd(&ctr[o], total);
            base[o] = __shfl(b, 63, 64);
        }
        for (int j = 0; j < 64; ++j) {
            const int nj = __shfl(nl, j, 64);
            if (nj == 0) continue;
            int pos[kOrders];
#pragma unroll
            for (int o = 0; o < kOrders; ++o) pos[o] = base[o] + __shfl(excl[o], j, 64);
            int chunk = __shfl(hd, j, 64);
            for (int e0 = 0; e0 < nj; e0 += kChunk) {
                if (e0 > 0) chunk = next[chunk];
                const bool v = e0 + lane < nj;
                const size_t at = (size_t)chunk * kChunk + lane;
                const int ob = v ? (int)ord[at] - 2 : -1;
                const uint32_t it = v ? items[at] : 0u;
#pragma unroll
                for (int o = 0; o < kOrders; ++o) {
                    const uint64_t m = __ballot(ob == o);
                    if (ob == o) {
                        const long long r = (long long)pos[o] + __popcll(m & lt);
                        if (r < sg.n[o]) out[sg.seg[o] + r] = make_int2(A0 + j, (int)it);
                    }
                    pos[o] += __popcll(m);
                }
            }
        }
    }
}

static int flatten_learned(fmm_tree *t, hipStream_t st)
{
    const int ncell = t->ncell;
    OrderSegs sg;
    long long tot = 0;
    for (int o = 0; o < kOrders; ++o) {
        sg.seg[o] = tot;
        sg.n[o] = t->stats.n_m2l_by_order[o];
        t->lseg[o] = tot;
        tot += sg.n[o];
    }
    if (tot == 0) return 0;
    if (tot > 0x7fffffff) return set_error(FMM_ERR_ARG, "too many M2L pairs (%lld)", tot);
    if (int rc = grow(t->m2l_ctr, 256) | grow(t->m2l_pairs, (size_t)tot * 8)) return rc;
    if (int rc = zero_async(t->m2l_ctr.p, kOrders * 4, st)) return rc;
    const size_t off = (size_t)kKindOrd * ncell;
    const int nw = (ncell + 63) / 64;
    const int g = nw < 16384 ? nw : 16384;
    k_flatten_learned<<<g, 64, 0, st>>>(ptr<int>(t->lhead) + off, ptr<int>(t->lcnt) + off,
                                        ptr<int>(t->lcnt) + (size_t)kKinds * ncell, ptr<uint32_t>(t->litems[kKindOrd]),
                                        ptr<unsigned char>(t->lord), ptr<int>(t->lnext[kKindOrd]), ncell,
                                        ptr<int>(t->m2l_ctr), sg, ptr<int2>(t->m2l_pairs));
    return hip_check(hipGetLastError(), "flatten learned pairs");
}

int flatten_pairs(fmm_tree *t, int kind, int64_t npair, hipStream_t st)
{
    const int ncell = t->ncell;
    if (npair > 0x7fffffff) return set_error(FMM_ERR_ARG, "too many M2L pairs for one list (%lld)", (long long)npair);
    const size_t off = (size_t)kind * ncell;
    if (int rc = grow(t->m2l_ctr, 256) | grow(t->m2l_pairs, (size_t)npair * 8)) return rc;
    if (int rc = zero_async(t->m2l_ctr.p, 4, st)) return rc;
    const int nw = (ncell + 63) / 64;
    const int g = nw < 16384 ? nw : 16384;
    k_flatten_pairs<<<g, 64, 0, st>>>(ptr<int>(t->lhead) + off, ptr<int>(t->lcnt) + off, ptr<uint32_t>(t->litems[kind]),
                                      ptr<int>(t->lnext[kind]), ncell, ptr<int>(t->m2l_ctr), ptr<int2>(t->m2l_pairs),
                                      (int)npair);
    return hip_check(hipGetLastError(), "flatten pairs");
}

int downward_l2l(fmm_tree *t, const fmm_params *P, hipStream_t st)
{
    return P->precision ? l2l_t<float>(t, P->p, st) : l2l_t<double>(t, P->p, st);
}

int l2p_combine(fmm_tree *t, const fmm_params *P, double *acc, int accumulate, hipStream_t st)
{
    return P->precision ? l2p_t<float>(t, P->p, P->G, acc, accumulate, st)
                        : l2p_t<double>(t, P->p, P->G, acc, accumulate, st);
}

}  // namespace hfmm
