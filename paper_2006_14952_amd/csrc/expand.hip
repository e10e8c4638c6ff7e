// Stage entry points of the expansion operators: precision dispatch.  The kernels are
// in expand_impl.h and are instantiated in expand_f32.hip and expand_f64.hip.
#include "state.h"

namespace hfmm {
template <class T> int upward_t(fmm_tree *t, int p, hipStream_t st);
template <class T> int m2l_t(fmm_tree *t, int p, double rs, hipStream_t st);
template <class T> int l2l_t(fmm_tree *t, int p, hipStream_t st);
template <class T> int l2p_t(fmm_tree *t, int p, double G, double *acc, hipStream_t st);

int upward(fmm_tree *t, const fmm_params *P, hipStream_t st)
{
    return P->precision ? upward_t<float>(t, P->p, st) : upward_t<double>(t, P->p, st);
}

int m2l(fmm_tree *t, const fmm_params *P, hipStream_t st)
{
    return P->precision ? m2l_t<float>(t, P->p, P->r_s, st) : m2l_t<double>(t, P->p, P->r_s, st);
}

int downward_l2l(fmm_tree *t, const fmm_params *P, hipStream_t st)
{
    return P->precision ? l2l_t<float>(t, P->p, st) : l2l_t<double>(t, P->p, st);
}

int l2p_combine(fmm_tree *t, const fmm_params *P, double *acc, hipStream_t st)
{
    return P->precision ? l2p_t<float>(t, P->p, P->G, acc, st) : l2p_t<double>(t, P->p, P->G, acc, st);
}

}  // namespace hfmm
