// Tile kernels: one workgroup per tile (or a persistent grid looping over
// tiles).  The (destination, source) layout pair is resolved once per tile
// by a wave-uniform branch into a fully specialised Phase B loop.
#pragma once
#include "tile_engine.hpp"

namespace lm {

#define LM_LAYOUT_PAIRS(CALL)                                   \
  switch (d.layout * 3u + s.layout) {                           \
    case 0: CALL(LY_AOS, LY_AOS); break;                        \
    case 1: CALL(LY_AOS, LY_PLANAR); break;                     \
    case 2: CALL(LY_AOS, LY_AOSOA); break;                      \
    case 3: CALL(LY_PLANAR, LY_AOS); break;                     \
    case 4: CALL(LY_PLANAR, LY_PLANAR); break;                  \
    case 5: CALL(LY_PLANAR, LY_AOSOA); break;                   \
    case 6: CALL(LY_AOSOA, LY_AOS); break;                      \
    case 7: CALL(LY_AOSOA, LY_PLANAR); break;                   \
    default: CALL(LY_AOSOA, LY_AOSOA); break;                   \
  }

template <int U>
__device__ __forceinline__ void phase_b_raw(const Side& s, const Side& d, uint64_t i0, uint32_t nt,
                                            const uint8_t* lds) {
#define LM_CALL(DL, SL) store_raw<U, DL, SL>(s, d, i0, nt, lds)
  LM_LAYOUT_PAIRS(LM_CALL)
#undef LM_CALL
}

template <int CONV, int U>
__device__ __forceinline__ void phase_b_conv(const Side& s, const Side& d, uint64_t i0, uint32_t nt,
                                             const uint8_t* lds) {
#define LM_CALL(DL, SL) store_conv<CONV, U, DL, SL>(s, d, i0, nt, lds)
  LM_LAYOUT_PAIRS(LM_CALL)
#undef LM_CALL
}

template <int CODEC>
__device__ __forceinline__ void phase_b_pack(const Side& s, const Side& d, uint64_t i0, uint32_t nt,
                                             const uint8_t* lds) {
  switch (s.layout) {
    case LY_AOS: store_pack<CODEC, LY_AOS>(s, d, i0, nt, lds); break;
    case LY_PLANAR: store_pack<CODEC, LY_PLANAR>(s, d, i0, nt, lds); break;
    default: store_pack<CODEC, LY_AOSOA>(s, d, i0, nt, lds); break;
  }
}

template <int CODEC, int U>
__device__ __forceinline__ void phase_b_unpack(const Side& s, const Side& d, uint64_t i0, uint32_t nt,
                                               const uint8_t* lds) {
  switch (d.layout) {
    case LY_AOS: store_unpack<CODEC, U, LY_AOS>(s, d, i0, nt, lds); break;
    case LY_PLANAR: store_unpack<CODEC, U, LY_PLANAR>(s, d, i0, nt, lds); break;
    default: store_unpack<CODEC, U, LY_AOSOA>(s, d, i0, nt, lds); break;
  }
}

// kind: 0 raw, 1 conversion, 2 pack, 3 unpack
template <int KIND, int P0, int U>
__global__ __launch_bounds__(kThreads) void k_tile(const TileArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  for (uint32_t t = blockIdx.x; t < a.ntiles_lo; t += gridDim.x) {
    const uint64_t i0 = (uint64_t)t * a.tile;
    const uint64_t left = a.src.n - i0;
    const uint32_t nt = left < (uint64_t)a.tile ? (uint32_t)left : a.tile;
    load_tile(a.src, i0, nt, lds);
    wait_tile_loads();
    if constexpr (KIND == 0) phase_b_raw<U>(a.src, a.dst, i0, nt, lds);
    else if constexpr (KIND == 1) phase_b_conv<P0, U>(a.src, a.dst, i0, nt, lds);
    else if constexpr (KIND == 2) phase_b_pack<P0>(a.src, a.dst, i0, nt, lds);
    else phase_b_unpack<P0, U>(a.src, a.dst, i0, nt, lds);
    __syncthreads();
  }
}

// Host launchers (one per kernel family, defined in the k_*.hip files).
hipError_t launch_raw(const TileArgs& a, uint32_t unit, uint32_t grid, uint32_t lds, hipStream_t st);
hipError_t launch_conv(const TileArgs& a, uint32_t unit, uint32_t grid, uint32_t lds, hipStream_t st);
hipError_t launch_pack(const TileArgs& a, uint32_t grid, uint32_t lds, hipStream_t st);
hipError_t launch_unpack(const TileArgs& a, uint32_t unit, uint32_t grid, uint32_t lds, hipStream_t st);

template <int KIND, int P0, int U>
inline hipError_t launch_k(const TileArgs& a, uint32_t grid, uint32_t lds, hipStream_t st) {
  hipLaunchKernelGGL((k_tile<KIND, P0, U>), dim3(grid), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

}  // namespace lm
