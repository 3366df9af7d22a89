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

// The views of one leaf size (contiguous after the host's ordering) and
// their tiles [t_begin, t_end) of the batch's tile space: one kernel, compiled
// for that leaf size only, moves them.
struct BatchGroup {
  uint32_t unit;              // leaf bytes
  uint32_t t_begin, t_end;    // tiles
  uint32_t v_begin, v_end;    // views
  uint32_t lds;               // the largest LDS of the group's views
  uint32_t tile_map;          // 1: each XCD takes a contiguous run of the group's tiles
};

// tile_view: view index of every tile of the batch, or null (then each
// workgroup searches the prefix sums)
hipError_t launch_batch(const BatchItem* items, const uint32_t* prefix, const uint32_t* tile_view,
                        const BatchGroup& g, uint32_t grid, hipStream_t st);

}  // namespace lm
