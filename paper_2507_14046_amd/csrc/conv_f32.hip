// Conv kernels instantiated for the PREC_F32 operand mode.
#include "conv_impl.h"

namespace d2ip {
void conv_fwd_f32(const ConvFwd& a, hipStream_t s) { conv_detail::conv_fwd_mode<PREC_F32>(a, s); }
void conv_wgrad_f32(const ConvWgrad& a, hipStream_t s) {
  conv_detail::conv_wgrad_mode<PREC_F32>(a, s);
}
}  // namespace d2ip
