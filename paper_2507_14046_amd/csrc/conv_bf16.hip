// Conv kernels instantiated for the PREC_BF16 operand mode.
#include "conv_impl.h"

namespace d2ip {
void conv_fwd_bf16(const ConvFwd& a, hipStream_t s) { conv_detail::conv_fwd_mode<PREC_BF16>(a, s); }
void conv_wgrad_bf16(const ConvWgrad& a, hipStream_t s) {
  conv_detail::conv_wgrad_mode<PREC_BF16>(a, s);
}
}  // namespace d2ip
