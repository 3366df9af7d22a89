// Zero fill of every mapped byte of a view: a copy from a NULL view (Sec. 3
// Null: loads give zero).  The destination is walked in 16-byte chunks as
// in Phase B; bytes that no record maps (AoSoA padding lanes) keep their
// contents.  Zero is the code of 0 in every integer and float format, so
// computed destinations are filled through their storage layout.
#include "kernels.hpp"

namespace lm {

template <int U, int DL>
__global__ __launch_bounds__(kThreads) void k_zero(const TileArgs a) {
  constexpr int NU = 16 / U;
  constexpr uint32_t FULL = (1u << NU) - 1u;
  for (uint32_t t = blockIdx.x; t < a.ntiles_lo; t += gridDim.x) {
    const uint64_t i0 = (uint64_t)t * a.tile;
    const uint64_t left = a.dst.n - i0;
    const uint32_t nt = left < (uint64_t)a.tile ? (uint32_t)left : a.tile;
    for_dst_chunks(a.dst, i0, nt, [&](__amdgpu_buffer_rsrc_t rs, uint32_t seg, uint32_t off, int x0, uint32_t len) {
      const uint32_t w[4] = {0u, 0u, 0u, 0u};
      uint32_t valid = 0;
#pragma unroll
      for (int k = 0; k < NU; ++k) {
        const int x = x0 + k * U;
        bool ok = x >= 0 && x < (int)len;
        if constexpr (DL != LY_STREAM) {  // stream words: every byte up to the tile's last word
          uint32_t r, b;
          dst_inv<DL>(a.dst, seg, ok ? (uint32_t)x : 0u, r, b);
          ok = ok && r < nt;
        }
        valid |= (uint32_t)ok << k;
      }
      store_chunk<U>(rs, off, w, valid, FULL);
    });
  }
}

template <int U>
static hipError_t launch_zero_u(const TileArgs& a, uint32_t grid, hipStream_t st) {
  switch (a.dst.layout) {
    case LY_AOS: hipLaunchKernelGGL((k_zero<U, LY_AOS>), dim3(grid), dim3(kThreads), 0, st, a); break;
    case LY_PLANAR: hipLaunchKernelGGL((k_zero<U, LY_PLANAR>), dim3(grid), dim3(kThreads), 0, st, a); break;
    case LY_AOSOA: hipLaunchKernelGGL((k_zero<U, LY_AOSOA>), dim3(grid), dim3(kThreads), 0, st, a); break;
    default: hipLaunchKernelGGL((k_zero<U, LY_STREAM>), dim3(grid), dim3(kThreads), 0, st, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_zero(const TileArgs& a, uint32_t unit, uint32_t grid, hipStream_t st) {
  switch (unit) {
    case 1: return launch_zero_u<1>(a, grid, st);
    case 2: return launch_zero_u<2>(a, grid, st);
    case 4: return launch_zero_u<4>(a, grid, st);
    case 8: return launch_zero_u<8>(a, grid, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lm
