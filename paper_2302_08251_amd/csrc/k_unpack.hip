// Unpack BitPackedIntSoA / BitPackedFloatSoA streams into a physical layout.
#include "kernels.hpp"

namespace lm {

#define LM_UNPACK(CD, ES)                                              \
  case CD:                                                             \
    if (unit == ES) return launch_k<3, CD, ES>(a, grid, lds, st);      \
    if (unit == 1) return launch_k<3, CD, 1>(a, grid, lds, st);        \
    break;

hipError_t launch_unpack(const TileArgs& a, uint32_t unit, uint32_t grid, uint32_t lds, hipStream_t st) {
  switch (a.codec) {
    case CD_U8:
      if (unit == 1) return launch_k<3, CD_U8, 1>(a, grid, lds, st);
      break;
    case CD_I8:
      if (unit == 1) return launch_k<3, CD_I8, 1>(a, grid, lds, st);
      break;
    LM_UNPACK(CD_U16, 2)
    LM_UNPACK(CD_I16, 2)
    LM_UNPACK(CD_U32, 4)
    LM_UNPACK(CD_I32, 4)
    LM_UNPACK(CD_U64, 8)
    LM_UNPACK(CD_I64, 8)
    LM_UNPACK(CD_F32, 4)
    LM_UNPACK(CD_F64, 8)
  }
  return hipErrorInvalidValue;
}

}  // namespace lm
