// Raw layout copies (no value conversion), units of 1, 2, 4 or 8 bytes.
#include "kernels.hpp"

namespace lm {

hipError_t launch_raw(const TileArgs& a, uint32_t unit, uint32_t grid, uint32_t lds, hipStream_t st) {
  switch (unit) {
    case 1: return launch_k<0, 0, 1>(a, grid, lds, st);
    case 2: return launch_k<0, 0, 2>(a, grid, lds, st);
    case 4: return launch_k<0, 0, 4>(a, grid, lds, st);
    case 8: return launch_k<0, 0, 8>(a, grid, lds, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lm
