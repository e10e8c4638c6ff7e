// Stage entry points of the expansion operators: precision dispatch.  The kernels are
// in expand_impl.h and are instantiated in expand_f32.hip and expand_f64.hip.
#include "state.h"

namespace hfmm {
template <class T> int upward_t(fmm_tree *t, int p, hipStream_t st);
template <class T> int m2l_t(fmm_tree *t, int p, double rs, int kind, int pstore, int accumulate, hipStream_t st);
template <class T> int l2l_t(fmm_tree *t, int p, hipStream_t st);
template <class T> int l2p_t(fmm_tree *t, int p, double G, double *acc, int accumulate, hipStream_t st);

int upward(fmm_tree *t, const fmm_params *P, hipStream_t st)
{
    return P->precision ? upward_t<float>(t, P->p, st) : upward_t<double>(t, P->p, st);
}

int m2l(fmm_tree *t, const fmm_params *P, hipStream_t st)
{
    return P->precision ? m2l_t<float>(t, P->p, P->r_s, 0, P->p, 0, st) : m2l_t<double>(t, P->p, P->r_s, 0, P->p, 0, st);
}

// Learned selector: coefficients stored at order 8; the pairs accepted at order o (list
// kind 4 + o - 2) are contracted at that order and added up.
int m2l_learned(fmm_tree *t, const fmm_params *P, hipStream_t st)
{
    hipMemsetAsync(t->Lc.p, 0, (size_t)t->ncell * ncoef(8) * (P->precision ? 4 : 8), st);
    for (int o = 2; o <= 8; ++o) {
        int rc = P->precision ? m2l_t<float>(t, o, P->r_s, 4 + o - 2, 8, 1, st)
                              : m2l_t<double>(t, o, P->r_s, 4 + o - 2, 8, 1, st);
        if (rc) return rc;
    }
    return 0;
}

// Flattens the chunked M2L list of `kind` into (sink, item) pairs ordered by sink.
__global__ __launch_bounds__(64) void k_flatten_pairs(const int *__restrict__ head, const int *__restrict__ cnt,
                                                      const uint32_t *__restrict__ items, const int *__restrict__ next,
                                                      const int *__restrict__ off, int ncell, int2 *__restrict__ out)
{
    const int lane = threadIdx.x;
    for (int A = blockIdx.x; A < ncell; A += gridDim.x) {
        const int nl = cnt[A];
        if (nl == 0) continue;
        int chunk = head[A];
        const int o = off[A];
        for (int e0 = 0; e0 < nl; e0 += kChunk) {
            if (e0 > 0) chunk = next[chunk];
            if (e0 + lane < nl) out[o + e0 + lane] = make_int2(A, (int)items[(size_t)chunk * kChunk + lane]);
        }
    }
}

int flatten_pairs(fmm_tree *t, int kind, int64_t npair, hipStream_t st)
{
    const int ncell = t->ncell;
    if (npair > 0x7fffffff) return set_error(FMM_ERR_ARG, "too many M2L pairs for one list (%lld)", (long long)npair);
    const size_t off = (size_t)kind * ncell;
    if (int rc = grow(t->m2l_off, (size_t)ncell * 4) | grow(t->m2l_pairs, (size_t)npair * 8)) return rc;
    if (int rc = scan_exclusive(ptr<int>(t->lcnt) + off, ptr<int>(t->m2l_off), ncell, nullptr, st, t->scan_tmp))
        return rc;
    const int g = ncell < 65536 ? ncell : 65536;
    k_flatten_pairs<<<g, 64, 0, st>>>(ptr<int>(t->lhead) + off, ptr<int>(t->lcnt) + off, ptr<uint32_t>(t->litems[kind]),
                                      ptr<int>(t->lnext[kind]), ptr<int>(t->m2l_off), ncell, ptr<int2>(t->m2l_pairs));
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
