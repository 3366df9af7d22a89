// Work items of the persistent batched copy.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace lm {

struct BatchItem {
  TileArgs args;   // the view's single-launch plan (tile size shared by the batch)
  uint32_t unit;     // leaf bytes of the record (1, 2, 4, 8)
  uint32_t variant;  // raw-copy variant (RawVariant)
  uint32_t pad[2];
};

// tile_view: view index of every tile (total_tiles entries), or null
hipError_t launch_batch(const BatchItem* items, const uint32_t* prefix, const uint32_t* tile_view,
                        uint32_t total_tiles, uint32_t n_views, uint32_t grid, uint32_t lds, hipStream_t st);

}  // namespace lm
