// Pack into BitPackedIntSoA / BitPackedFloatSoA streams.
#include "kernels.hpp"

namespace lm {

hipError_t launch_pack(const TileArgs& a, uint32_t grid, uint32_t lds, hipStream_t st) {
  // the benchmarked float formats get compile-time encoders
  if (a.codec == CD_F32 && !a.dst.rne) {
    const uint32_t E = a.dst.exp_bits, M = a.dst.man_bits;
    if (E == 8 && M == 7) return launch_k<2, CD_F32, PF_E8M7>(a, grid, lds, st);
    if (E == 5 && M == 10) return launch_k<2, CD_F32, PF_E5M10>(a, grid, lds, st);
    if (E == 8 && M == 15) return launch_k<2, CD_F32, PF_E8M15>(a, grid, lds, st);
  }
  switch (a.codec) {
    case CD_U8: return launch_k<2, CD_U8, PF_RUNTIME>(a, grid, lds, st);
    case CD_I8: return launch_k<2, CD_I8, PF_RUNTIME>(a, grid, lds, st);
    case CD_U16: return launch_k<2, CD_U16, PF_RUNTIME>(a, grid, lds, st);
    case CD_I16: return launch_k<2, CD_I16, PF_RUNTIME>(a, grid, lds, st);
    case CD_U32: return launch_k<2, CD_U32, PF_RUNTIME>(a, grid, lds, st);
    case CD_I32: return launch_k<2, CD_I32, PF_RUNTIME>(a, grid, lds, st);
    case CD_U64: return launch_k<2, CD_U64, PF_RUNTIME>(a, grid, lds, st);
    case CD_I64: return launch_k<2, CD_I64, PF_RUNTIME>(a, grid, lds, st);
    case CD_F32: return launch_k<2, CD_F32, PF_RUNTIME>(a, grid, lds, st);
    case CD_F64: return launch_k<2, CD_F64, PF_RUNTIME>(a, grid, lds, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lm
