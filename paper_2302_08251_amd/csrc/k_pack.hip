// Pack into BitPackedIntSoA / BitPackedFloatSoA streams.
#include "kernels.hpp"

namespace lm {

hipError_t launch_pack(const TileArgs& a, uint32_t grid, uint32_t lds, hipStream_t st) {
  switch (a.codec) {
    case CD_U8: return launch_k<2, CD_U8, 4>(a, grid, lds, st);
    case CD_I8: return launch_k<2, CD_I8, 4>(a, grid, lds, st);
    case CD_U16: return launch_k<2, CD_U16, 4>(a, grid, lds, st);
    case CD_I16: return launch_k<2, CD_I16, 4>(a, grid, lds, st);
    case CD_U32: return launch_k<2, CD_U32, 4>(a, grid, lds, st);
    case CD_I32: return launch_k<2, CD_I32, 4>(a, grid, lds, st);
    case CD_U64: return launch_k<2, CD_U64, 4>(a, grid, lds, st);
    case CD_I64: return launch_k<2, CD_I64, 4>(a, grid, lds, st);
    case CD_F32: return launch_k<2, CD_F32, 4>(a, grid, lds, st);
    case CD_F64: return launch_k<2, CD_F64, 4>(a, grid, lds, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lm
