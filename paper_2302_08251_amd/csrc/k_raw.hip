// Raw layout copies (no value conversion) of records with 1, 2 or 8 byte
// leaves; 4-byte leaves are in k_raw4.hip.
// Full-chunk stores of the raw copies: non-temporal at device scope (sc1 nt).
// Measured: +0.6 % over the 36 layout pairs; the pack, unpack and batch
// kernels lose with it and keep nt alone.
#define LM_STORE_POLICY 18
#include "kernels.hpp"

namespace lm {

uint32_t raw_variant(const TileArgs& a, uint32_t leaf_bytes) {
  if (a.mode == RM_LINE) {
    if (a.src.cs == a.dst.cs) return a.dst.cs == leaf_bytes && leaf_bytes > 1 ? RV_LINE_ES : RV_LINE_1;
    return a.dst.cs == 1 ? RV_LINE_SPLIT : RV_LINE_MERGE;
  }
  if (a.mode == RM_MERGE) return RV_MERGE;
  if (a.mode == RM_SPLIT) return RV_SPLIT;
  if (a.mode == RM_MERGE_FUSED) return RV_MERGE_FUSED;
  if (a.mode == RM_SPLIT_FUSED) return RV_SPLIT_FUSED;
  return a.src.cs == leaf_bytes && leaf_bytes > 1 ? RV_DIRECT_ES : RV_DIRECT_1;
}

template <int ES>
static hipError_t launch_es(const TileArgs& a, uint32_t rv, uint32_t grid, uint32_t lds, hipStream_t st) {
  switch (rv) {
    case RV_DIRECT_ES: return launch_raw_rv<ES, RV_DIRECT_ES>(a, grid, lds, st);
    case RV_DIRECT_1: return launch_raw_rv<ES, RV_DIRECT_1>(a, grid, lds, st);
    case RV_MERGE: return launch_raw_rv<ES, RV_MERGE>(a, grid, lds, st);
    case RV_SPLIT: return launch_raw_rv<ES, RV_SPLIT>(a, grid, lds, st);
    case RV_SPLIT_FUSED: return launch_raw_fused<ES, RV_SPLIT_FUSED>(a, grid, lds, st);
    case RV_MERGE_FUSED: return launch_raw_fused<ES, RV_MERGE_FUSED>(a, grid, lds, st);
    case RV_LINE_ES: return launch_raw_line<ES, RV_LINE_ES>(a, grid, lds, st);
    case RV_LINE_1: return launch_raw_line<ES, RV_LINE_1>(a, grid, lds, st);
    case RV_LINE_SPLIT: return launch_raw_line<ES, RV_LINE_SPLIT>(a, grid, lds, st);
    case RV_LINE_MERGE: return launch_raw_line<ES, RV_LINE_MERGE>(a, grid, lds, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_raw(const TileArgs& a, uint32_t leaf_bytes, uint32_t variant, uint32_t grid, uint32_t lds,
                      hipStream_t st) {
  switch (leaf_bytes) {
    case 1:
      if (variant == RV_LINE_1) return launch_raw_line<1, RV_LINE_1>(a, grid, lds, st);
      return launch_raw_rv<1, RV_DIRECT_1>(a, grid, lds, st);
    case 2: return launch_es<2>(a, variant, grid, lds, st);
    case 4: return launch_raw4(a, variant, grid, lds, st);
    case 8: return launch_es<8>(a, variant, grid, lds, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lm
