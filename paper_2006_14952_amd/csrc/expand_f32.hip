// FP32 instantiation of the expansion operators (one translation unit per precision).
#include "expand_impl.h"

namespace hfmm {
template int upward_t<float>(fmm_tree *, int, hipStream_t);
template int m2l_t<float>(fmm_tree *, int, Split, int, int, int, int, int, hipStream_t);
template int l2l_t<float>(fmm_tree *, int, hipStream_t);
template int l2p_t<float>(fmm_tree *, int, double, double *, int, hipStream_t);
}  // namespace hfmm
