// ChangeType conversions fused with the layout change.
#include "kernels.hpp"

namespace lm {

hipError_t launch_conv(const TileArgs& a, uint32_t unit, uint32_t grid, uint32_t lds, hipStream_t st) {
  if (a.conv == CV_F64_F32) {
    if (unit == 4) return launch_k<1, CV_F64_F32, 4>(a, grid, lds, st);
    if (unit == 1) return launch_k<1, CV_F64_F32, 1>(a, grid, lds, st);
  } else if (a.conv == CV_F32_F64) {
    if (unit == 8) return launch_k<1, CV_F32_F64, 8>(a, grid, lds, st);
    if (unit == 1) return launch_k<1, CV_F32_F64, 1>(a, grid, lds, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lm
