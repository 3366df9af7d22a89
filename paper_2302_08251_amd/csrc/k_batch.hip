// Persistent batched copy: one launch moves the tiles of many views with
// mixed mapping pairs.  The global tile index space is the concatenation of
// every view's tiles (prefix sums in `prefix`); workgroup b takes tiles
// b, b + G, b + 2G, ... so consecutive tiles of one view spread over all
// XCDs and every workgroup gets the same number of tiles.  The per-tile work
// is the single-view tile engine, selected by the view's leaf size and copy
// variant with wave-uniform branches; the host orders views by variant so
// that a workgroup walks through one variant's tiles at a time.
#include "batch.hpp"
#include "kernels.hpp"

namespace lm {

__global__ __launch_bounds__(kThreads) void k_batch(const BatchItem* __restrict__ items,
                                                   const uint32_t* __restrict__ prefix,
                                                   const uint32_t* __restrict__ tile_view, uint32_t total_tiles,
                                                   uint32_t n_views) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  uint32_t v = 0;
  for (uint32_t t = blockIdx.x; t < total_tiles; t += gridDim.x) {
    // view holding tile t: prefix[v] <= t < prefix[v + 1].  With one
    // workgroup per tile the host's tile -> view table answers in one load;
    // a persistent workgroup visits its tiles in increasing order and
    // gallops forward from the last view, then bisects.
    if (tile_view) {
      v = tile_view[t];
    } else if (prefix[v + 1] <= t) {
      uint32_t step = 1, lo = v + 1, hi = v + 1;
      while (hi < n_views && prefix[hi + 1] <= t) {
        lo = hi + 1;
        hi = hi + step;
        step *= 2;
        if (hi >= n_views) hi = n_views - 1;
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
    switch (it.unit) {
      case 1: tile_raw_any<1>(it.args, it.variant, i0, nt, lds); break;
      case 2: tile_raw_any<2>(it.args, it.variant, i0, nt, lds); break;
      case 4: tile_raw_any<4>(it.args, it.variant, i0, nt, lds); break;
      default: tile_raw_any<8>(it.args, it.variant, i0, nt, lds); break;
    }
    __syncthreads();
  }
}

hipError_t launch_batch(const BatchItem* items, const uint32_t* prefix, const uint32_t* tile_view,
                        uint32_t total_tiles, uint32_t n_views, uint32_t grid, uint32_t lds, hipStream_t st) {
  // the table is used when every workgroup takes a single tile
  const uint32_t* tv = grid >= total_tiles ? tile_view : nullptr;
  hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kThreads), lds, st, items, prefix, tv, total_tiles, n_views);
  return hipGetLastError();
}

}  // namespace lm
