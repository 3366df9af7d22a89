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

// Raw-copy variants: how the source tile reaches Phase B (see RawMode) and
// the unit of Phase B.
enum RawVariant : uint32_t {
  RV_DIRECT_ES = 0,  // same column size on both sides: leaf elements
  RV_DIRECT_1 = 1,   // both sides Bytesplit: bytes
  RV_MERGE = 2,      // Bytesplit source -> element columns
  RV_SPLIT = 3,      // element columns -> Bytesplit destination
  RV_SPLIT_FUSED = 4,  // RV_SPLIT without the canonical image
  RV_MERGE_FUSED = 5,  // RV_MERGE without the canonical image
  // line-owner writes into single-blob planes off the line grid (RM_LINE),
  // by how the destination planes are built:
  RV_LINE_ES = 6,      //   element columns on both sides
  RV_LINE_1 = 7,       //   byte columns on both sides
  RV_LINE_SPLIT = 8,   //   element columns -> byte planes, transposed in registers
  RV_LINE_MERGE = 9,   //   byte columns -> element planes
};

template <int RV>
constexpr bool is_line_variant() {
  return RV == RV_LINE_ES || RV == RV_LINE_1 || RV == RV_LINE_SPLIT || RV == RV_LINE_MERGE;
}

// Phase B for one destination layout DL from an LDS image of layout SL, with
// the item loop form FORM (see load_tile).
template <int U, int DL, int SL, int COLRUN, int FORM, typename G>
__device__ __forceinline__ void phase_b_dl(const G& s, const Side& d, uint64_t i0, uint32_t nt, const uint8_t* lds) {
  if constexpr (COLRUN && DL == LY_AOS) {
    store_identity<U, FORM>(s, d, i0, nt, lds);  // AoS image of the same record: identical bytes
  } else if constexpr (COLRUN && SL != LY_AOS) {
    store_colrun<U, DL, SL, FORM>(s, d, i0, nt, lds);
  } else {
    store_raw<U, DL, SL, FORM>(s, d, i0, nt, lds);
  }
}

// One tile of a raw copy of records whose leaves are ES bytes, from a source
// of layout SL: verbatim source image, an optional relayout through a
// canonical planar image when exactly one side is a Bytesplit, then Phase B.
template <int ES, int RV, int DL, int COLRUN, int SL>
__device__ __forceinline__ void tile_raw_sl(const TileArgs& a, uint64_t i0, uint32_t nt, uint8_t* lds) {
  // loop forms (measured): element copies take the run-time-layout loops in
  // Phase B, and in Phase A when the source is one segment (AoS, AoSoA)
  constexpr int FORM_A = RV == RV_DIRECT_ES && (SL == LY_AOS || SL == LY_AOSOA) ? 1 : 0;
  constexpr int FORM_B = RV == RV_DIRECT_ES ? 1 : 0;
  if constexpr (is_line_variant<RV>()) {
    // the tile and its halo: the records up to the end of the tile's last line
    const uint64_t left = a.src.n - i0;
    const uint32_t nl = left < (uint64_t)(nt + a.halo) ? (uint32_t)left : nt + a.halo;
    load_tile<SL, 0>(a.src, i0, nl, lds);
    wait_tile_loads();
    if constexpr (RV == RV_LINE_SPLIT) {
      store_split_lines16<ES, SL>(a.src, a.dst, i0, nt, nl, lds);
    } else if constexpr (RV == RV_LINE_ES) {
      store_lines16<ES>(a.dst, i0, nt, nl, a.src.ncols,
                        [&](uint32_t r, uint32_t c) { return read_col16<ES, SL>(a.src, lds, r, c); });
    } else if constexpr (RV == RV_LINE_1) {
      store_lines16<1>(a.dst, i0, nt, nl, a.src.ncols,
                       [&](uint32_t r, uint32_t c) { return read_col16<1, SL>(a.src, lds, r, c); });
    } else {  // byte columns merged into element planes
      store_lines16<ES>(a.dst, i0, nt, nl, a.src.ncols / ES,
                        [&](uint32_t r, uint32_t f) { return read_merge16<ES, SL>(a.src, lds, r, f); });
    }
    return;
  }
  load_tile<SL, FORM_A>(a.src, i0, nt, lds);
  wait_tile_loads();
  if constexpr (RV == RV_SPLIT_FUSED) {
    if (DL == LY_AOSOA && (a.dst.lanes & 15u)) store_split_fused<ES, SL, DL>(a.src, a.dst, i0, nt, lds);  // runs of 4 records
    else store_split_fused16<ES, SL, DL>(a.src, a.dst, i0, nt, lds);
  } else if constexpr (RV == RV_MERGE_FUSED) {
    store_merge_fused<ES, SL, DL>(a.src, a.dst, i0, nt, lds);
  } else if constexpr (RV == RV_MERGE || RV == RV_SPLIT) {
    uint8_t* can = lds + a.can_off;
    if constexpr (RV == RV_MERGE && DL == LY_AOS) {
      if (a.can_off == 0u) relayout_merge_aos_inplace<ES, SL, kMergeInPlaceItems<ES>>(a.src, nt, lds, a.can);
      else relayout_merge_aos<ES, SL>(a.src, nt, lds, can, a.can);
    } else if constexpr (RV == RV_MERGE) {
      relayout_merge<ES, SL>(a.src, nt, lds, can, a.can);
    } else {
      relayout_split<ES, SL>(a.src, nt, lds, can, a.can);
    }
    __syncthreads();
    // the canonical image: the destination's AoS record image (merge into
    // AoS) or planes of elements (merge) or bytes (split)
    constexpr int CL = (RV == RV_MERGE && DL == LY_AOS) ? LY_AOS : LY_PLANAR;
    phase_b_dl<RV == RV_MERGE ? ES : 1, DL, CL, COLRUN, 0>(a.can, a.dst, i0, nt, can);
  } else {
    phase_b_dl<RV == RV_DIRECT_ES ? ES : 1, DL, SL, COLRUN, FORM_B>(a.src, a.dst, i0, nt, lds);
  }
}

// The source layouts a variant can meet: a Bytesplit source (the merges)
// keeps byte columns in planes or AoSoA blocks; every other variant takes
// any physical layout.
template <int ES, int RV, int DL, int COLRUN>
__device__ __forceinline__ void tile_raw(const TileArgs& a, uint64_t i0, uint32_t nt, uint8_t* lds) {
  if constexpr (RV == RV_MERGE || RV == RV_MERGE_FUSED || RV == RV_LINE_MERGE) {
    if (a.src.layout == LY_AOSOA) tile_raw_sl<ES, RV, DL, COLRUN, LY_AOSOA>(a, i0, nt, lds);
    else tile_raw_sl<ES, RV, DL, COLRUN, LY_PLANAR>(a, i0, nt, lds);
  } else {
    switch (a.src.layout) {
      case LY_AOS: tile_raw_sl<ES, RV, DL, COLRUN, LY_AOS>(a, i0, nt, lds); break;
      case LY_PLANAR: tile_raw_sl<ES, RV, DL, COLRUN, LY_PLANAR>(a, i0, nt, lds); break;
      default: tile_raw_sl<ES, RV, DL, COLRUN, LY_AOSOA>(a, i0, nt, lds); break;
    }
  }
}

// Runtime selection of the variant (batched copies).
template <int ES>
__device__ __forceinline__ void tile_raw_any(const TileArgs& a, uint32_t rv, uint64_t i0, uint32_t nt, uint8_t* lds) {
#define LM_DL(RV, DL)                                                        \
  if (a.dst.layout == DL) {                                                  \
    if (a.colrun) tile_raw<ES, RV, DL, 1>(a, i0, nt, lds);                   \
    else tile_raw<ES, RV, DL, 0>(a, i0, nt, lds);                            \
    return;                                                                  \
  }
#define LM_RV(RV) \
  if (rv == RV) { LM_DL(RV, LY_AOS) LM_DL(RV, LY_PLANAR) LM_DL(RV, LY_AOSOA) }
#define LM_RVF(RV) \
  if (rv == RV) {                                                            \
    if (a.dst.layout == LY_AOSOA) tile_raw<ES, RV, LY_AOSOA, 0>(a, i0, nt, lds); \
    else tile_raw<ES, RV, LY_PLANAR, 0>(a, i0, nt, lds);                     \
    return;                                                                  \
  }
#define LM_RVL(RV) \
  if (rv == RV) {                                                            \
    tile_raw<ES, RV, LY_PLANAR, 0>(a, i0, nt, lds);                          \
    return;                                                                  \
  }
  if constexpr (ES == 1) {
    LM_RV(RV_DIRECT_1)
    LM_RVL(RV_LINE_1)
  } else {
    LM_RV(RV_DIRECT_ES)
    LM_RV(RV_DIRECT_1)
    LM_RV(RV_MERGE)
    LM_RV(RV_SPLIT)
    LM_RVF(RV_SPLIT_FUSED)
    LM_RVF(RV_MERGE_FUSED)
    LM_RVL(RV_LINE_ES)
    LM_RVL(RV_LINE_1)
    LM_RVL(RV_LINE_SPLIT)
    LM_RVL(RV_LINE_MERGE)
  }
#undef LM_RVL
#undef LM_RVF
#undef LM_RV
#undef LM_DL
}

template <int CONV, int U>
__device__ __forceinline__ void phase_b_conv(const Side& s, const Side& d, uint64_t i0, uint32_t nt,
                                             const uint8_t* lds) {
#define LM_CALL(DL, SL) store_conv<CONV, U, DL, SL>(s, d, i0, nt, lds)
  LM_LAYOUT_PAIRS(LM_CALL)
#undef LM_CALL
}

template <int CODEC, int FMT>
__device__ __forceinline__ void phase_b_pack(const Side& s, const Side& d, uint64_t i0, uint32_t nt,
                                             const uint8_t* lds, uint32_t* words, uint32_t wstride) {
  switch (s.layout) {
    case LY_AOS: store_pack<CODEC, FMT, LY_AOS>(s, d, i0, nt, lds, words, wstride); break;
    case LY_PLANAR: store_pack<CODEC, FMT, LY_PLANAR>(s, d, i0, nt, lds, words, wstride); break;
    default: store_pack<CODEC, FMT, LY_AOSOA>(s, d, i0, nt, lds, words, wstride); break;
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

// Raw copies, one kernel per (leaf bytes, variant, destination layout,
// column-run flag) so that each kernel holds only the Phase B bodies it runs.
template <int ES, int RV, int DL, int COLRUN>
__global__ __launch_bounds__(kThreads) void k_raw(const TileArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  for (uint32_t t = blockIdx.x; t < a.ntiles_lo; t += gridDim.x) {
    const uint64_t i0 = (uint64_t)t * a.tile;
    const uint64_t left = a.src.n - i0;
    const uint32_t nt = left < (uint64_t)a.tile ? (uint32_t)left : a.tile;
    tile_raw<ES, RV, DL, COLRUN>(a, i0, nt, lds);
    __syncthreads();
  }
}

// kind: 1 conversion, 2 pack, 3 unpack.  P0: the conversion (Conv) or the
// codec (Codec); U: the destination unit in bytes (conversion, unpack) or the
// compile-time float format (pack, PackFmt).
template <int KIND, int P0, int U>
__global__ __launch_bounds__(kThreads) void k_tile(const TileArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  for (uint32_t t = blockIdx.x; t < a.ntiles_lo; t += gridDim.x) {
    const uint64_t i0 = (uint64_t)t * a.tile;
    const uint64_t left = a.src.n - i0;
    const uint32_t nt = left < (uint64_t)a.tile ? (uint32_t)left : a.tile;
    // pack: the stream-word image of the tile (one plane of tile * B / 32
    // words per field) follows the source image in LDS (can_off 0: none, every
    // field's codes are stored from registers)
    uint32_t* words = (uint32_t*)(lds + a.can_off);
    const uint32_t wstride = (a.tile * a.dst.bits) >> 5;
    if constexpr (KIND == 2) {
      if (a.can_off) pack_clear_words(words, a.dst.ncols * wstride);  // 0: no word image
    }
    // streaming loads for packs and conversions from f32 or narrower (see load_tile)
    if constexpr (KIND == 3) load_tile<LY_STREAM, 0, false>(a.src, i0, nt, lds);
    else if constexpr (KIND == 1 && ConvInfo<P0>::ES_SRC > 4) load_tile<-1, 0, false>(a.src, i0, nt, lds);
    else load_tile(a.src, i0, nt, lds);
    wait_tile_loads();
    if constexpr (KIND == 1) phase_b_conv<P0, U>(a.src, a.dst, i0, nt, lds);
    else if constexpr (KIND == 2) phase_b_pack<P0, U>(a.src, a.dst, i0, nt, lds, words, wstride);
    else phase_b_unpack<P0, U>(a.src, a.dst, i0, nt, lds);
    __syncthreads();
  }
}

// Host launchers (one per kernel family, defined in the k_*.hip files).
hipError_t launch_raw(const TileArgs& a, uint32_t leaf_bytes, uint32_t variant, uint32_t grid, uint32_t lds,
                      hipStream_t st);
hipError_t launch_raw4(const TileArgs& a, uint32_t variant, uint32_t grid, uint32_t lds, hipStream_t st);
uint32_t raw_variant(const TileArgs& a, uint32_t leaf_bytes);
hipError_t launch_conv(const TileArgs& a, uint32_t unit, uint32_t grid, uint32_t lds, hipStream_t st);
hipError_t launch_pack(const TileArgs& a, uint32_t grid, uint32_t lds, hipStream_t st);
hipError_t launch_unpack(const TileArgs& a, uint32_t unit, uint32_t grid, uint32_t lds, hipStream_t st);
hipError_t launch_zero(const TileArgs& a, uint32_t unit, uint32_t grid, hipStream_t st);
hipError_t launch_xpose(const XposeArgs& a, uint32_t unit, uint32_t grid, uint32_t lds, hipStream_t st);
hipError_t launch_mixed(const MixArgs& a, uint32_t grid, hipStream_t st);
hipError_t launch_generic(const GenArgs& a, uint32_t grid, hipStream_t st);
hipError_t launch_pack_planar(const PlanarPackArgs& a, uint32_t grid, hipStream_t st);

template <int KIND, int P0, int U>
inline hipError_t launch_k(const TileArgs& a, uint32_t grid, uint32_t lds, hipStream_t st) {
  hipLaunchKernelGGL((k_tile<KIND, P0, U>), dim3(grid), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

template <int ES, int RV>
inline hipError_t launch_raw_fused(const TileArgs& a, uint32_t grid, uint32_t lds, hipStream_t st) {
  if (a.dst.layout == LY_AOSOA) hipLaunchKernelGGL((k_raw<ES, RV, LY_AOSOA, 0>), dim3(grid), dim3(kThreads), lds, st, a);
  else hipLaunchKernelGGL((k_raw<ES, RV, LY_PLANAR, 0>), dim3(grid), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

template <int ES, int RV>
inline hipError_t launch_raw_line(const TileArgs& a, uint32_t grid, uint32_t lds, hipStream_t st) {
  hipLaunchKernelGGL((k_raw<ES, RV, LY_PLANAR, 0>), dim3(grid), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

template <int ES, int RV>
inline hipError_t launch_raw_rv(const TileArgs& a, uint32_t grid, uint32_t lds, hipStream_t st) {
#define LM_L(DL)                                                                                  \
  if (a.dst.layout == DL) {                                                                       \
    if (a.colrun) hipLaunchKernelGGL((k_raw<ES, RV, DL, 1>), dim3(grid), dim3(kThreads), lds, st, a); \
    else hipLaunchKernelGGL((k_raw<ES, RV, DL, 0>), dim3(grid), dim3(kThreads), lds, st, a);          \
    return hipGetLastError();                                                                     \
  }
  LM_L(LY_AOS)
  LM_L(LY_PLANAR)
  LM_L(LY_AOSOA)
#undef LM_L
  return hipErrorInvalidValue;
}

}  // namespace lm
