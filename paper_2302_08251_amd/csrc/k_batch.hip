// Persistent batched copy: one launch per leaf size moves the tiles of many
// views with mixed mapping pairs.  The global tile index space is the concatenation of
// every view's tiles (prefix sums in `prefix`); workgroup b takes tiles
// b, b + G, b + 2G, ... so consecutive tiles of one view spread over all
// XCDs and every workgroup gets the same number of tiles.  The per-tile work
// is the single-view tile engine, selected by the view's leaf size and copy
// variant with wave-uniform branches; the host orders views by variant so
// that a workgroup walks through one variant's tiles at a time.
#include "batch.hpp"
#include "kernels.hpp"

namespace lm {

template <int ES>
__global__ __launch_bounds__(kThreads) void k_batch(const BatchItem* __restrict__ items,
                                                   const uint32_t* __restrict__ prefix,
                                                   const uint32_t* __restrict__ tile_view, const BatchGroup g) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  uint32_t v = g.v_begin;
  const uint32_t nt_all = g.t_end - g.t_begin;
  const bool xmap = g.tile_map && gridDim.x >= nt_all;
  for (uint32_t b = blockIdx.x; b < nt_all; b += gridDim.x) {
    const uint32_t t = g.t_begin + (xmap ? xcd_tile(b, nt_all) : b);
    // view holding tile t: prefix[v] <= t < prefix[v + 1].  With one
    // workgroup per tile the host's tile -> view table answers in one load;
    // a persistent workgroup visits its tiles in increasing order and
    // gallops forward from the last view, then bisects.
    if (tile_view) {
      v = tile_view[t];
    } else if (prefix[v + 1] <= t) {
      uint32_t step = 1, lo = v + 1, hi = v + 1;
      while (hi < g.v_end && prefix[hi + 1] <= t) {
        lo = hi + 1;
        hi = hi + step;
        step *= 2;
        if (hi >= g.v_end) hi = g.v_end - 1;
      }
      while (lo < hi) {  // smallest u in [lo, hi] with prefix[u + 1] > t
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid + 1] <= t) lo = mid + 1;
        else hi = mid;
      }
      v = lo;
    }
    const BatchItem& it = items[v];
    const uint64_t i0 = (uint64_t)(t - prefix[v]) * it.args.tile;
    const uint64_t left = it.args.src.n - i0;
    const uint32_t nt = left < (uint64_t)it.args.tile ? (uint32_t)left : it.args.tile;
    tile_raw_any<ES>(it.args, it.variant, i0, nt, lds);
    __syncthreads();
  }
}

hipError_t launch_batch(const BatchItem* items, const uint32_t* prefix, const uint32_t* tile_view,
                        const BatchGroup& g, uint32_t grid, hipStream_t st) {
  // the table is used when every workgroup takes a single tile
  const uint32_t* tv = grid >= g.t_end - g.t_begin ? tile_view : nullptr;
  switch (g.unit) {
    case 1: hipLaunchKernelGGL(k_batch<1>, dim3(grid), dim3(kThreads), g.lds, st, items, prefix, tv, g); break;
    case 2: hipLaunchKernelGGL(k_batch<2>, dim3(grid), dim3(kThreads), g.lds, st, items, prefix, tv, g); break;
    case 4: hipLaunchKernelGGL(k_batch<4>, dim3(grid), dim3(kThreads), g.lds, st, items, prefix, tv, g); break;
    case 8: hipLaunchKernelGGL(k_batch<8>, dim3(grid), dim3(kThreads), g.lds, st, items, prefix, tv, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lm
