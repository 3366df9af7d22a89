// Raw layout copies of records with 4-byte leaves (f32 / i32 / u32).
// Full-chunk stores of the raw copies: non-temporal at device scope (sc1 nt).
// Measured: +0.6 % over the 36 layout pairs; the pack, unpack and batch
// kernels lose with it and keep nt alone.
#define LM_STORE_POLICY 18
#include "kernels.hpp"

namespace lm {

hipError_t launch_raw4(const TileArgs& a, uint32_t variant, uint32_t grid, uint32_t lds, hipStream_t st) {
  switch (variant) {
    case RV_DIRECT_ES: return launch_raw_rv<4, RV_DIRECT_ES>(a, grid, lds, st);
    case RV_DIRECT_1: return launch_raw_rv<4, RV_DIRECT_1>(a, grid, lds, st);
    case RV_MERGE: return launch_raw_rv<4, RV_MERGE>(a, grid, lds, st);
    case RV_SPLIT: return launch_raw_rv<4, RV_SPLIT>(a, grid, lds, st);
    case RV_SPLIT_FUSED: return launch_raw_fused<4, RV_SPLIT_FUSED>(a, grid, lds, st);
    case RV_MERGE_FUSED: return launch_raw_fused<4, RV_MERGE_FUSED>(a, grid, lds, st);
    case RV_LINE_ES: return launch_raw_line<4, RV_LINE_ES>(a, grid, lds, st);
    case RV_LINE_1: return launch_raw_line<4, RV_LINE_1>(a, grid, lds, st);
    case RV_LINE_SPLIT: return launch_raw_line<4, RV_LINE_SPLIT>(a, grid, lds, st);
    case RV_LINE_MERGE: return launch_raw_line<4, RV_LINE_MERGE>(a, grid, lds, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lm
