// ChangeType conversions (Sec. 3) fused with the layout change: f64, f32,
// f16 and bf16 storage, narrowing with round to nearest even, widening exact.
#include "kernels.hpp"

namespace lm {

hipError_t launch_conv(const TileArgs& a, uint32_t unit, uint32_t grid, uint32_t lds, hipStream_t st) {
  // unit: the destination column size, the element (ES_DST) or 1 (Bytesplit)
#define LM_CONV(CV)                                                          \
  case CV:                                                                   \
    if (unit == (uint32_t)ConvInfo<CV>::ES_DST) return launch_k<1, CV, ConvInfo<CV>::ES_DST>(a, grid, lds, st); \
    if (unit == 1) return launch_k<1, CV, 1>(a, grid, lds, st);              \
    break;
  switch (a.conv) {
    LM_CONV(CV_F64_F32)
    LM_CONV(CV_F32_F64)
    LM_CONV(CV_F32_F16)
    LM_CONV(CV_F32_BF16)
    LM_CONV(CV_F64_F16)
    LM_CONV(CV_F64_BF16)
    LM_CONV(CV_F16_F32)
    LM_CONV(CV_BF16_F32)
    LM_CONV(CV_F16_F64)
    LM_CONV(CV_BF16_F64)
    default: break;
  }
#undef LM_CONV
  return hipErrorInvalidValue;
}

}  // namespace lm
