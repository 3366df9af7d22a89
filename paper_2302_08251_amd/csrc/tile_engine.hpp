// Tile engine for layout-aware copy, ChangeType conversion and bit packing
// on gfx950 (LLAMA, arXiv 2302.08251: layout-aware copy Sec. 1, computed
// mappings Sec. 3, AoS / SoA / AoSoA Sec. 5).
//
// One workgroup moves one tile of records [i0, i0 + nt):
//   Phase A  the source side's segments for the tile are copied verbatim into
//            LDS with direct buffer->LDS 128-bit loads (one 1 KiB group of 64
//            lanes per wave instruction, contiguous in HBM).
//   Phase B  each lane owns a 16-byte chunk of a destination segment (so the
//            store is one coalesced 128-bit buffer store), inverts the
//            destination mapping for every unit of the chunk to (record,
//            byte of record), and gathers that unit from LDS through the
//            source mapping's tile-local address function.
// All global accesses go through buffer resources whose range is the blob
// the mapping uses, so an access outside the blob is dropped by hardware.
// Per-lane offsets are 32-bit; only the per-segment scalar base is 64-bit.
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace lm {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
typedef __attribute__((address_space(3))) void lds_void;

constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit format, gfx9 family
// Cache policy of full-chunk stores: non-temporal (streaming).  Device code is
// compiled per translation unit, so a unit may define LM_STORE_POLICY before
// including this header to choose another policy for its own kernels.
#ifndef LM_STORE_POLICY
#define LM_STORE_POLICY 2
#endif
constexpr int kStoreNT = LM_STORE_POLICY;
constexpr int kLoadStream = 3;          // cache policy: a load of data read once (sc0 nt: no L1, streaming)

__device__ __forceinline__ uint32_t wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}
__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }
__device__ __forceinline__ uint32_t num_waves() { return blockDim.x >> 6; }

// The tile of workgroup b (of n, one per tile) when each of the 8 XCDs takes
// a contiguous run of the tiles: workgroup b runs on XCD b mod 8, so
// neighbouring tiles share that XCD's L2 (lines they both touch are fetched
// from HBM once).
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
  const uint32_t x = b & 7u, k = b >> 3, q = n >> 3, r = n & 7u;
  return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t x, const Div& d) {
  return d.pow2 ? (x >> d.sh) : __umulhi(x, d.m);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint64_t bytes) {
  const uint32_t nr = bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)nr, kRsrcWord3);
}

// ---------------------------------------------------------------------------
// Segment geometry of one side for a tile
// ---------------------------------------------------------------------------

struct SegGeo {
  uint32_t nseg;  // segments of the tile
  uint32_t len;   // bytes per segment (equal for all segments)
};

// The segment helpers take the side's layout as a template argument when
// the caller knows it (L >= 0), so that no layout switch is left in the item
// loops; L = -1 reads it from the side.
template <int L>
__device__ __forceinline__ uint32_t layout_of(const Side& s) {
  return L >= 0 ? (uint32_t)L : s.layout;
}

template <int L = -1>
__device__ __forceinline__ SegGeo seg_geo(const Side& s, uint32_t nt) {
  switch (layout_of<L>(s)) {
    case LY_AOS: return {1u, nt * s.rec_bytes};
    case LY_AOSOA: return {1u, fdiv(nt + s.lanes - 1, s.div_L) * s.lanes * s.rec_bytes};
    case LY_PLANAR: return {s.ncols, nt * s.cs};
    default: return {s.ncols, ((nt * s.bits + 31u) >> 5) * 4u};
  }
}

// Byte offset, within its blob, where segment `seg` of the tile at i0 starts.
template <int L = -1>
__device__ __forceinline__ uint64_t seg_start(const Side& s, uint32_t seg, uint64_t i0) {
  switch (layout_of<L>(s)) {
    case LY_AOS:
    case LY_AOSOA: return i0 * s.rec_bytes;
    case LY_PLANAR: return (s.mb ? 0ull : s.n * s.cs * seg) + i0 * s.cs;
    default: return (i0 * s.bits) >> 3;
  }
}

template <int L = -1>
__device__ __forceinline__ const void* seg_blob(const Side& s, uint32_t seg) {
  const uint32_t l = layout_of<L>(s);
  const bool per_col = l == LY_STREAM || (l == LY_PLANAR && s.mb);
  return per_col ? s.blob[seg] : s.blob[0];
}

// LDS offset of segment `seg`'s allocation.  The data starts at
// seg_lds + (start mod 16), so a 16-byte aligned global chunk lands on a
// 16-byte aligned LDS chunk.
template <int L = -1>
__device__ __forceinline__ uint32_t seg_lds(const Side& s, uint32_t seg) {
  const uint32_t l = layout_of<L>(s);
  return (l == LY_PLANAR || l == LY_STREAM) ? seg * s.lds_stride : 0u;
}

// Start phase (mod 16) of planar column c of a single-blob side.
template <typename G>
__device__ __forceinline__ uint32_t planar_phase(const G& s, uint32_t c) {
  return s.mb ? 0u : ((s.n_mod16 * s.cs * c) & 15u);
}

// Divisor for a run-time d >= 1 built on the device once per tile (one
// 32-bit division), so that the item loops split an item index into
// (segment, group) with one multiply-high: fdiv(x, div) = x / d exactly
// while x * d < 2^32, which every item loop below satisfies.
__device__ __forceinline__ Div make_div_dev(uint32_t d) {
  Div r;
  r.d = d;
  r.pow2 = (d & (d - 1u)) == 0u ? 1u : 0u;
  r.sh = r.pow2 ? (uint32_t)__builtin_ctz(d) : 0u;
  r.m = r.pow2 ? 0u : 0xFFFFFFFFu / d + 1u;
  return r;
}

// ---------------------------------------------------------------------------
// Phase A: source tile -> LDS, verbatim
// ---------------------------------------------------------------------------

// Two forms of the item loops, chosen per kernel family by measurement on
// the MI355X.  FORM 0: the layout fixed at compile time and one divisor per
// tile; this is much faster for the many byte planes of a Bytesplit side.
// FORM 1: the layout read at run time and a division per item; this is about
// 4 % faster for element copies between AoS, SoA and AoSoA.
//
// STREAM: the loads stream past L1 with the streaming L2 hint (sc0 nt), for
// data read once; measured faster for copies (+2.5 % over the 36 layout
// pairs) and packs (+10-20 %), slower for unpacks of narrow codes (-10-20 %)
// and f64 sources of a conversion, which keep the default policy.
template <int LT = -1, int FORM = 0, bool STREAM = true>
__device__ __forceinline__ void load_tile(const Side& s, uint64_t i0, uint32_t nt, uint8_t* lds) {
  constexpr int L = FORM ? -1 : LT;
  const SegGeo g = seg_geo<L>(s, nt);
  const uint32_t w = wave_id(), nw = num_waves(), lane = lane_id();
  const uint32_t gps = (g.len + 15u + 1023u) >> 10;  // groups of 64 chunks per segment
  const Div dg = make_div_dev(gps);
  const uint32_t items = g.nseg * gps;
  // per-column blobs only for SoA-MB and streams: otherwise one blob, its
  // pointer loaded once for the tile (a scalar load per item, waited on
  // before the item's load could issue, cost single-blob Bytesplit sources
  // 6 %: Bytesplit -> SoA-SB 5.72 -> 6.09 TB/s)
  const uint32_t lay = layout_of<L>(s);
  const bool per_col = lay == LY_STREAM || (lay == LY_PLANAR && s.mb);
  const uint8_t* const blob0 = (const uint8_t*)s.blob[0];
  for (uint32_t it = w; it < items; it += nw) {
    const uint32_t seg = FORM ? it / gps : fdiv(it, dg);
    const uint32_t grp = it - seg * gps;
    const uint64_t start = seg_start<L>(s, seg, i0);
    const uint32_t phase = (uint32_t)start & 15u;
    const uint64_t abase = start - phase;
    const uint8_t* base = per_col ? (const uint8_t*)s.blob[seg] : blob0;
    const auto rs = make_rsrc(base + abase, s.blob_size - abase);
    const uint32_t chunk = grp * 64u + lane;
    if (chunk * 16u < phase + g.len) {
      if (abase + chunk * 16ull + 16ull <= s.blob_size) {
        lds_void* to = (lds_void*)(lds + seg_lds<L>(s, seg) + grp * 1024u);
        if constexpr (STREAM) __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, to, 16, chunk * 16u, 0, 0, kLoadStream);
        else __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, to, 16, chunk * 16u, 0, 0, 0);
      } else {
        // The chunk crosses the end of the blob.  Buffer range checks work on
        // whole dwords, so a blob size that is not a multiple of 4 would zero
        // the last bytes: fetch this chunk byte by byte instead.
        uint8_t* out = lds + seg_lds<L>(s, seg) + chunk * 16u;
        const uint64_t left = s.blob_size - (abase + chunk * 16ull);
        for (uint32_t k = 0; k < 16u && k < left; ++k)
          out[k] = __builtin_amdgcn_raw_buffer_load_b8(rs, chunk * 16u + k, 0, 0);
      }
    }
  }
}

__device__ __forceinline__ void wait_tile_loads() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Mapping functions on tile-local coordinates
// ---------------------------------------------------------------------------

// Destination inverse: byte x of destination segment `seg` holds byte b of
// the stored record image of tile-local record r.
template <int DL>
__device__ __forceinline__ void dst_inv(const Side& d, uint32_t seg, uint32_t x, uint32_t& r,
                                        uint32_t& b) {
  if constexpr (DL == LY_AOS) {
    r = fdiv(x, d.div_S);
    b = x - r * d.rec_bytes;
  } else if constexpr (DL == LY_PLANAR) {
    r = x >> d.log2cs;
    b = seg * d.cs + (x & (d.cs - 1u));
  } else {  // LY_AOSOA: block, column, lane, byte
    const uint32_t blk = fdiv(x, d.div_LS);
    const uint32_t y = x - blk * (d.lanes * d.rec_bytes);
    const uint32_t c = fdiv(y, d.div_Lcs);
    const uint32_t z = y - c * (d.lanes * d.cs);
    r = blk * d.lanes + (z >> d.log2cs);
    b = c * d.cs + (z & (d.cs - 1u));
  }
}

// Source forward: LDS offset of byte b of the stored record image of
// tile-local record r (G is a Side or the Geo of a canonical image).
template <int SL, typename G>
__device__ __forceinline__ uint32_t src_addr(const G& s, uint32_t r, uint32_t b) {
  if constexpr (SL == LY_AOS) {
    return r * s.rec_bytes + b;
  } else if constexpr (SL == LY_PLANAR) {
    const uint32_t c = b >> s.log2cs;
    return c * s.lds_stride + planar_phase(s, c) + r * s.cs + (b & (s.cs - 1u));
  } else {  // LY_AOSOA
    const uint32_t c = b >> s.log2cs;
    const uint32_t blk = fdiv(r, s.div_L);
    const uint32_t lane = r - blk * s.lanes;
    return blk * (s.lanes * s.rec_bytes) + c * (s.lanes * s.cs) + lane * s.cs + (b & (s.cs - 1u));
  }
}

template <int U>
__device__ __forceinline__ uint64_t lds_read(const uint8_t* lds, uint32_t a) {
  if constexpr (U == 1) return lds[a];
  else if constexpr (U == 2) return *(const uint16_t*)(lds + a);
  else if constexpr (U == 4) return *(const uint32_t*)(lds + a);
  else return *(const uint64_t*)(lds + a);
}

// Store `nunits` units of U bytes of a 16-byte chunk; full chunks go out as
// one 128-bit store, partial ones unit by unit.
template <int U>
__device__ __forceinline__ void store_chunk(__amdgpu_buffer_rsrc_t rs, uint32_t off, const uint32_t (&w)[4],
                                            uint32_t valid, uint32_t full_mask) {
  // full chunk: one 128-bit store; partial: whole dwords, then single units
  if (valid == full_mask) {
    u32x4 v = {w[0], w[1], w[2], w[3]};
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, off, 0, kStoreNT);
    return;
  }
  if constexpr (U < 4) {
    // dwords whose units are all valid go out whole
    constexpr uint32_t PER = 4 / U, M = (1u << PER) - 1u;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (((valid >> (q * PER)) & M) == M) __builtin_amdgcn_raw_buffer_store_b32(w[q], rs, off + 4u * q, 0, 0);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (((valid >> (q * PER)) & M) == M) valid &= ~(M << (q * PER));
  }
#pragma unroll
  for (int t = 0; t < 16 / U; ++t) {
    if (!((valid >> t) & 1u)) continue;
    const uint32_t byte = t * U;
    if constexpr (U == 1) {
      __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(w[byte >> 2] >> ((byte & 3u) * 8u)), rs, off + byte, 0, 0);
    } else if constexpr (U == 2) {
      __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(w[byte >> 2] >> ((byte & 3u) * 8u)), rs, off + byte, 0, 0);
    } else if constexpr (U == 4) {
      __builtin_amdgcn_raw_buffer_store_b32(w[byte >> 2], rs, off + byte, 0, 0);
    } else {
      u32x2 v = {w[byte >> 2], w[(byte >> 2) + 1]};
      __builtin_amdgcn_raw_buffer_store_b64(v, rs, off + byte, 0, 0);
    }
  }
}

template <int U>
__device__ __forceinline__ void put_unit(uint32_t (&w)[4], int t, uint64_t v) {
  if constexpr (U == 8) {
    w[2 * t] = (uint32_t)v;
    w[2 * t + 1] = (uint32_t)(v >> 32);
  } else if constexpr (U == 4) {
    w[t] = (uint32_t)v;
  } else {
    const uint32_t byte = t * U;
    w[byte >> 2] |= ((uint32_t)v & ((1u << (8 * U)) - 1u)) << ((byte & 3u) * 8u);
  }
}

// Iterates over the 16-byte chunks of the destination segments of a tile,
// one group of 64 chunks per wave at a time; `body(rs, seg, chunk, x0, len)`
// handles one chunk whose first byte is segment byte x0 (negative for the
// bytes before a misaligned segment start).
template <int LT = -1, int FORM = 0, typename Body>
__device__ __forceinline__ void for_dst_chunks(const Side& d, uint64_t i0, uint32_t nt, Body&& body) {
  constexpr int L = FORM ? -1 : LT;
  const SegGeo g = seg_geo<L>(d, nt);
  const uint32_t w = wave_id(), nw = num_waves(), lane = lane_id();
  const uint32_t gps = (g.len + 15u + 1023u) >> 10;
  const Div dg = make_div_dev(gps);
  const uint32_t items = g.nseg * gps;
  for (uint32_t it = w; it < items; it += nw) {
    const uint32_t seg = FORM ? it / gps : fdiv(it, dg);
    const uint32_t grp = it - seg * gps;
    const uint64_t start = seg_start<L>(d, seg, i0);
    const uint32_t phase = (uint32_t)start & 15u;
    const uint64_t abase = start - phase;
    const auto rs = make_rsrc((const uint8_t*)seg_blob<L>(d, seg) + abase, d.blob_size - abase);
    const uint32_t chunk = grp * 64u + lane;
    const int x0 = (int)(chunk * 16u) - (int)phase;
    if (x0 < (int)g.len) body(rs, seg, chunk * 16u, x0, g.len);
  }
}

// ---------------------------------------------------------------------------
// Phase B, raw copy: units of U = min(source column, destination column) bytes
// ---------------------------------------------------------------------------

template <int U, int DL, int SL, int FORM = 0, typename G>
__device__ __forceinline__ void store_raw(const G& s, const Side& d, uint64_t i0, uint32_t nt,
                                          const uint8_t* lds);

// ---------------------------------------------------------------------------
// In-LDS relayout between Bytesplit byte columns and element columns
// (Sec. 3 Bytesplit).  Four consecutive records of one field form a 4 x ES
// byte block.  MERGE reads the block from ES byte columns (four bytes each)
// and writes four elements into the field's plane of a canonical planar
// image; SPLIT reads four elements and writes ES four-byte words into the
// byte planes.  A 4 x 4 byte block is transposed with eight v_perm_b32.
// Consecutive lanes take consecutive blocks, so the canonical image is
// written (MERGE, SPLIT) and the planar source read (SPLIT) without bank
// conflicts.
// ---------------------------------------------------------------------------

// out[j] byte k = in[k] byte j
__device__ __forceinline__ void transpose4x4(const uint32_t (&in)[4], uint32_t (&out)[4]) {
  const uint32_t t01 = __builtin_amdgcn_perm(in[1], in[0], 0x05010400u);
  const uint32_t t23 = __builtin_amdgcn_perm(in[3], in[2], 0x05010400u);
  const uint32_t u01 = __builtin_amdgcn_perm(in[1], in[0], 0x07030602u);
  const uint32_t u23 = __builtin_amdgcn_perm(in[3], in[2], 0x07030602u);
  out[0] = __builtin_amdgcn_perm(t23, t01, 0x05040100u);
  out[1] = __builtin_amdgcn_perm(t23, t01, 0x07060302u);
  out[2] = __builtin_amdgcn_perm(u23, u01, 0x05040100u);
  out[3] = __builtin_amdgcn_perm(u23, u01, 0x07060302u);
}

// bytes of byte column c for tile-local records r .. r+3 (r a multiple of 4)
template <int SL>
__device__ __forceinline__ uint32_t read_run4(const Side& s, const uint8_t* lds, uint32_t r, uint32_t c) {
  const uint32_t a = src_addr<SL>(s, r, c);
  const bool contiguous = SL == LY_PLANAR || (SL == LY_AOSOA && (s.lanes & 3u) == 0u);
  if (contiguous) {
    if ((a & 3u) == 0u) return *(const uint32_t*)(lds + a);
    // a misaligned run (plane start not 4-byte aligned): two aligned dwords
    // (inside the plane's 16-byte slack) and a byte funnel shift
    const uint32_t al = a & ~3u;
    return __builtin_amdgcn_alignbyte(*(const uint32_t*)(lds + al + 4u), *(const uint32_t*)(lds + al), a & 3u);
  }
  uint32_t w = 0;
#pragma unroll
  for (uint32_t j = 0; j < 4; ++j) w |= (uint32_t)lds[src_addr<SL>(s, r + j, c)] << (8u * j);
  return w;
}

// four elements (ES bytes each) of field f for records r .. r+3, as dwords:
// e[j * ES/4 + h] is dword h of element j (ES = 4, 8); for ES = 2, e[0], e[1]
// hold elements (0, 1) and (2, 3)
template <int ES, int SL>
__device__ __forceinline__ void read_elems4(const Side& s, const uint8_t* lds, uint32_t r, uint32_t f,
                                            uint32_t (&e)[ES]) {
  const uint32_t a = src_addr<SL>(s, r, f * ES);
  const bool contiguous = SL == LY_PLANAR || (SL == LY_AOSOA && (s.lanes & 3u) == 0u);
  if constexpr (ES == 2) {
    if (contiguous && (a & 7u) == 0u) {
      const u32x2 v = *(const u32x2*)(lds + a);
      e[0] = v.x;
      e[1] = v.y;
    } else {
      uint32_t h[4];
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j) h[j] = *(const uint16_t*)(lds + src_addr<SL>(s, r + j, f * 2));
      e[0] = h[0] | (h[1] << 16);
      e[1] = h[2] | (h[3] << 16);
    }
  } else {
    constexpr int DW = ES / 4;  // dwords per element
    if (contiguous && (a & 15u) == 0u) {
#pragma unroll
      for (int q = 0; q < DW; ++q) {
        const u32x4 v = *(const u32x4*)(lds + a + 16u * q);
        e[4 * q + 0] = v.x;
        e[4 * q + 1] = v.y;
        e[4 * q + 2] = v.z;
        e[4 * q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j)
#pragma unroll
        for (int h = 0; h < DW; ++h) e[j * DW + h] = *(const uint32_t*)(lds + src_addr<SL>(s, r + j, f * ES) + 4u * h);
    }
  }
}

// write NB bytes (dwords w[]) to LDS offset a, with the widest accesses its
// alignment allows
template <int NB>
__device__ __forceinline__ void lds_write(uint8_t* lds, uint32_t a, const uint32_t* w) {
  if constexpr (NB >= 16) {
    if ((a & 15u) == 0u) {
#pragma unroll
      for (int q = 0; q < NB / 16; ++q)
        *(u32x4*)(lds + a + 16 * q) = u32x4{w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]};
      return;
    }
  }
  if ((a & 3u) == 0u) {
#pragma unroll
    for (int q = 0; q < NB / 4; ++q) *(uint32_t*)(lds + a + 4 * q) = w[q];
  } else if ((a & 1u) == 0u) {
#pragma unroll
    for (int q = 0; q < NB / 2; ++q) *(uint16_t*)(lds + a + 2 * q) = (uint16_t)(w[q >> 1] >> (16 * (q & 1)));
  } else {
#pragma unroll
    for (int q = 0; q < NB; ++q) lds[a + q] = (uint8_t)(w[q >> 2] >> (8 * (q & 3)));
  }
}

// The canonical planes sit at the same phase (mod 16) as the destination's
// planes (geometry `cg`), so Phase B moves whole aligned 16-byte chunks.
template <int ES, int SL>
__device__ __forceinline__ void relayout_merge(const Side& s, uint32_t nt, const uint8_t* lds, uint8_t* can,
                                               const Geo& cg) {
  const uint32_t F = s.ncols / ES;
  const uint32_t quads = (nt + 3u) >> 2;
  const Div dq = make_div_dev(quads);
  const uint32_t items = F * quads;
  for (uint32_t q = threadIdx.x; q < items; q += blockDim.x) {
    const uint32_t f = fdiv(q, dq);
    const uint32_t r = (q - f * quads) * 4u;
    const uint32_t a = f * cg.lds_stride + planar_phase(cg, f) + r * ES;
    uint32_t out[ES];  // the 4 elements, as ES dwords in memory order
    if constexpr (ES == 2) {
      const uint32_t b0 = read_run4<SL>(s, lds, r, 2 * f), b1 = read_run4<SL>(s, lds, r, 2 * f + 1);
      out[0] = __builtin_amdgcn_perm(b1, b0, 0x05010400u);
      out[1] = __builtin_amdgcn_perm(b1, b0, 0x07030602u);
    } else {
      constexpr int DW = ES / 4;
#pragma unroll
      for (int h = 0; h < DW; ++h) {  // bytes 4h .. 4h+3 of the elements
        uint32_t in[4], o[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) in[k] = read_run4<SL>(s, lds, r, f * ES + 4 * h + k);
        transpose4x4(in, o);
#pragma unroll
        for (int j = 0; j < 4; ++j) out[j * DW + h] = o[j];
      }
    }
    lds_write<4 * ES>(can, a, out);
  }
}

template <int ES, int SL>
__device__ __forceinline__ void relayout_split(const Side& s, uint32_t nt, const uint8_t* lds, uint8_t* can,
                                               const Geo& cg) {
  const uint32_t F = s.ncols;
  const uint32_t quads = (nt + 3u) >> 2;
  const Div dq = make_div_dev(quads);
  const uint32_t items = F * quads;
  for (uint32_t q = threadIdx.x; q < items; q += blockDim.x) {
    const uint32_t f = fdiv(q, dq);
    const uint32_t r = (q - f * quads) * 4u;
    uint32_t e[ES];
    read_elems4<ES, SL>(s, lds, r, f, e);
    uint32_t col[ES];  // col[k]: byte k of records r..r+3
    if constexpr (ES == 2) {
      col[0] = __builtin_amdgcn_perm(e[1], e[0], 0x06040200u);
      col[1] = __builtin_amdgcn_perm(e[1], e[0], 0x07050301u);
    } else {
      constexpr int DW = ES / 4;
#pragma unroll
      for (int h = 0; h < DW; ++h) {
        uint32_t in[4], o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) in[j] = e[j * DW + h];
        transpose4x4(in, o);
#pragma unroll
        for (int k = 0; k < 4; ++k) col[4 * h + k] = o[k];
      }
    }
#pragma unroll
    for (int k = 0; k < ES; ++k) {
      const uint32_t c = f * ES + k;
      lds_write<4>(can, c * cg.lds_stride + planar_phase(cg, c) + r, &col[k]);
    }
  }
}

// ---------------------------------------------------------------------------
// Phase B over column runs: when every destination chunk holds 16/cs
// consecutive records of one column and the source keeps those records
// contiguous too (planar, or AoSoA with 16-byte column runs), a chunk is one
// LDS read and one 128-bit store.  Other chunks take the unit-by-unit path.
// ---------------------------------------------------------------------------

// MERGE into an AoS destination: the elements go straight into the
// destination's own record image (record r at r * S, field f at f * ES), so
// Phase B is a plain 16-byte copy of that image.  Work items are (quad of
// records, field) with the field fastest: the four element writes of a wave
// then land on neighbouring words.
template <int ES, int SL>
__device__ __forceinline__ void relayout_merge_aos(const Side& s, uint32_t nt, const uint8_t* lds, uint8_t* can,
                                                   const Geo& cg) {
  const uint32_t F = cg.ncols;
  const uint32_t items = ((nt + 3u) >> 2) * F;
  for (uint32_t it = threadIdx.x; it < items; it += blockDim.x) {
    const uint32_t q = fdiv(it, cg.div_L);  // div_L holds the field count here
    const uint32_t f = it - q * F;
    const uint32_t r = 4u * q;
    uint32_t out[ES];  // the 4 elements, as ES dwords in memory order
    if constexpr (ES == 2) {
      const uint32_t b0 = read_run4<SL>(s, lds, r, 2 * f), b1 = read_run4<SL>(s, lds, r, 2 * f + 1);
      out[0] = __builtin_amdgcn_perm(b1, b0, 0x05010400u);
      out[1] = __builtin_amdgcn_perm(b1, b0, 0x07030602u);
    } else {
      constexpr int DW = ES / 4;
#pragma unroll
      for (int h = 0; h < DW; ++h) {
        uint32_t in[4], o[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) in[k] = read_run4<SL>(s, lds, r, f * ES + 4 * h + k);
        transpose4x4(in, o);
#pragma unroll
        for (int j = 0; j < 4; ++j) out[j * DW + h] = o[j];
      }
    }
    uint8_t* base = can + r * cg.rec_bytes + f * ES;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint8_t* e = base + j * cg.rec_bytes;
      if constexpr (ES == 2) *(uint16_t*)e = (uint16_t)(out[j >> 1] >> (16 * (j & 1)));
      else if constexpr (ES == 4) *(uint32_t*)e = out[j];
      else *(u32x2*)e = u32x2{out[2 * j], out[2 * j + 1]};
    }
  }
}

// The same merge into the AoS record image, in place over the source image:
// every thread first reads and transposes all its (quad, field) items into
// registers (at most MAXI), then, after a barrier, writes them over the byte
// planes.  The tile then needs one LDS image instead of two, which lets more
// workgroups share a CU.  The host picks this form (canonical image offset
// 0) when quads * fields <= MAXI * threads.
template <int ES, int SL, int MAXI>
__device__ __forceinline__ void relayout_merge_aos_inplace(const Side& s, uint32_t nt, uint8_t* lds, const Geo& cg) {
  const uint32_t F = cg.ncols;
  const uint32_t items = ((nt + 3u) >> 2) * F;
  uint32_t out[MAXI][ES];  // per item: the 4 elements, as ES dwords in memory order
#pragma unroll
  for (int k = 0; k < MAXI; ++k) {
    const uint32_t it = threadIdx.x + (uint32_t)k * blockDim.x;
    if (it >= items) break;
    const uint32_t q = fdiv(it, cg.div_L);  // div_L holds the field count here
    const uint32_t f = it - q * F;
    const uint32_t r = 4u * q;
    if constexpr (ES == 2) {
      const uint32_t b0 = read_run4<SL>(s, lds, r, 2 * f), b1 = read_run4<SL>(s, lds, r, 2 * f + 1);
      out[k][0] = __builtin_amdgcn_perm(b1, b0, 0x05010400u);
      out[k][1] = __builtin_amdgcn_perm(b1, b0, 0x07030602u);
    } else {
      constexpr int DW = ES / 4;
#pragma unroll
      for (int h = 0; h < DW; ++h) {
        uint32_t in[4], o[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) in[c] = read_run4<SL>(s, lds, r, f * ES + 4 * h + c);
        transpose4x4(in, o);
#pragma unroll
        for (int j = 0; j < 4; ++j) out[k][j * DW + h] = o[j];
      }
    }
  }
  __syncthreads();  // every byte plane is read before any record is written over it
#pragma unroll
  for (int k = 0; k < MAXI; ++k) {
    const uint32_t it = threadIdx.x + (uint32_t)k * blockDim.x;
    if (it >= items) break;
    const uint32_t q = fdiv(it, cg.div_L);
    const uint32_t f = it - q * F;
    uint8_t* base = lds + 4u * q * cg.rec_bytes + f * ES;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint8_t* e = base + j * cg.rec_bytes;
      if constexpr (ES == 2) *(uint16_t*)e = (uint16_t)(out[k][j >> 1] >> (16 * (j & 1)));
      else if constexpr (ES == 4) *(uint32_t*)e = out[k][j];
      else *(u32x2*)e = u32x2{out[k][2 * j], out[k][2 * j + 1]};
    }
  }
}

template <int U, int DL, int SL, typename G>
__device__ __forceinline__ void raw_chunk(const G& s, const Side& d, uint32_t nt, const uint8_t* lds,
                                          __amdgpu_buffer_rsrc_t rs, uint32_t seg, uint32_t off, int x0,
                                          uint32_t len) {
  constexpr int NU = 16 / U;
  constexpr uint32_t FULL = (1u << NU) - 1u;
  uint32_t w[4] = {0u, 0u, 0u, 0u};
  uint32_t valid = 0;
#pragma unroll
  for (int t = 0; t < NU; ++t) {
    const int x = x0 + t * U;
    bool ok = x >= 0 && x < (int)len;
    uint32_t r, b;
    dst_inv<DL>(d, seg, ok ? (uint32_t)x : 0u, r, b);
    ok = ok && r < nt;
    if (ok) put_unit<U>(w, t, lds_read<U>(lds, src_addr<SL>(s, r, b)));
    valid |= (uint32_t)ok << t;
  }
  store_chunk<U>(rs, off, w, valid, FULL);
}

template <int U, int DL, int SL, int FORM, typename G>
__device__ __forceinline__ void store_raw(const G& s, const Side& d, uint64_t i0, uint32_t nt,
                                          const uint8_t* lds) {
  for_dst_chunks<DL, FORM>(d, i0, nt, [&](__amdgpu_buffer_rsrc_t rs, uint32_t seg, uint32_t off, int x0, uint32_t len) {
    raw_chunk<U, DL, SL>(s, d, nt, lds, rs, seg, off, x0, len);
  });
}

template <int U, int DL, int SL, int FORM = 0, typename G>
__device__ __forceinline__ void store_colrun(const G& s, const Side& d, uint64_t i0, uint32_t nt,
                                             const uint8_t* lds) {
  constexpr uint32_t NREC = 16 / U;
  for_dst_chunks<DL, FORM>(d, i0, nt, [&](__amdgpu_buffer_rsrc_t rs, uint32_t seg, uint32_t off, int x0, uint32_t len) {
    if (x0 >= 0 && x0 + 16 <= (int)len) {
      uint32_t r, b;
      dst_inv<DL>(d, seg, (uint32_t)x0, r, b);
      if (r + NREC <= nt) {
        const uint32_t a = src_addr<SL>(s, r, b);
        if (src_addr<SL>(s, r + NREC - 1u, b) - a == 16u - U) {
          u32x4 v;
          if ((a & 15u) == 0u) {
            v = *(const u32x4*)(lds + a);
          } else if ((a & 3u) == 0u) {
            const uint32_t* p = (const uint32_t*)(lds + a);
            v = u32x4{p[0], p[1], p[2], p[3]};
          } else {
            // five aligned dwords and byte funnel shifts; the fifth dword
            // starts inside the run and ends before the next 4-aligned
            // plane boundary, so it stays in this plane's allocation
            const uint32_t* p = (const uint32_t*)(lds + (a & ~3u));
            const uint32_t sh = a & 3u;
            const uint32_t d0 = p[0], d1 = p[1], d2 = p[2], d3 = p[3], d4 = p[4];
            v = u32x4{__builtin_amdgcn_alignbyte(d1, d0, sh), __builtin_amdgcn_alignbyte(d2, d1, sh),
                      __builtin_amdgcn_alignbyte(d3, d2, sh), __builtin_amdgcn_alignbyte(d4, d3, sh)};
          }
          __builtin_amdgcn_raw_buffer_store_b128(v, rs, off, 0, kStoreNT);
          return;
        }
      }
    }
    raw_chunk<U, DL, SL>(s, d, nt, lds, rs, seg, off, x0, len);
  });
}

// AoS image -> AoS destination of the same record: the LDS image and the
// destination segment hold the same bytes in the same order (tiles start on
// 16-byte boundaries), so whole chunks move as they are.
template <int U, int FORM = 0, typename G>
__device__ __forceinline__ void store_identity(const G& s, const Side& d, uint64_t i0, uint32_t nt,
                                               const uint8_t* lds) {
  for_dst_chunks<LY_AOS, FORM>(d, i0, nt, [&](__amdgpu_buffer_rsrc_t rs, uint32_t seg, uint32_t off, int x0, uint32_t len) {
    if (x0 + 16 <= (int)len) __builtin_amdgcn_raw_buffer_store_b128(*(const u32x4*)(lds + x0), rs, off, 0, kStoreNT);
    else raw_chunk<U, LY_AOS, LY_AOS>(s, d, nt, lds, rs, seg, off, x0, len);
  });
}

// ---------------------------------------------------------------------------
// Line-owner Phase B for single-blob planar destinations whose planes start
// off the 128-byte line grid (n * column bytes not a multiple of 128).  When
// two workgroups each write part of one line, the memory system merges the
// parts by a read-modify-write of the line; with planes off the grid every
// tile boundary of every plane would cost one.  Here each line of a plane is
// written whole by exactly one tile: the tile owns the plane's bytes from the
// first line boundary at or after its first record to the first one at or
// after its end (the plane's own start and end bound the first and last
// tile).  Its last line reaches up to 128 / cs records into the next tile,
// so the tile loads that many more records (the halo).  Lanes build 16-byte
// runs of one destination column in registers straight from the tile's
// source image and write 16-byte windows aligned to the destination, each
// joining the left neighbour's run and the lane's own (store_lines16,
// store_split_lines16).  Only lines shared by the end of one plane and the
// start of the next keep two writers.
// ---------------------------------------------------------------------------


// ---------------------------------------------------------------------------
// Fused relayout + store for Bytesplit pairs whose byte runs stay 4-byte
// aligned.  Work items are (field f, 64 blocks of 4 records); the field is
// wave-uniform, so every byte column a wave writes has a uniform buffer
// resource (also for multi-blob destinations).
//   split: 4 elements of field f (one 4 x ES byte block) are read from the
//          source tile, transposed, and the ES four-byte words are stored to
//          the destination byte columns: 256 contiguous bytes per column and
//          wave instruction.
//   merge: ES four-byte words (byte k of records r..r+3) are read from the
//          source byte columns, transposed into 4 elements and stored as one
//          4*ES-byte run of field f: 1 KiB contiguous per wave instruction.
// ---------------------------------------------------------------------------

// Column c of a planar or AoSoA side (cs = column size): the byte offset
// where the tile's run of that column starts (wave-uniform; tiles start on
// AoSoA block boundaries) and the offset of tile-local record r from there.
template <int DL>
__device__ __forceinline__ uint64_t col_base(const Side& d, uint64_t i0, uint32_t c) {
  if constexpr (DL == LY_PLANAR) return (d.mb ? 0ull : d.n * d.cs * c) + i0 * d.cs;
  else return i0 * d.rec_bytes + (uint64_t)c * d.lanes * d.cs;
}

template <int DL>
__device__ __forceinline__ uint32_t col_local(const Side& d, uint32_t r) {
  if constexpr (DL == LY_PLANAR) {
    return r * d.cs;
  } else {
    const uint32_t blk = fdiv(r, d.div_L);
    return blk * d.lanes * d.rec_bytes + (r - blk * d.lanes) * d.cs;
  }
}

template <int ES, int SL, int DL>
__device__ __forceinline__ void store_split_fused(const Side& s, const Side& d, uint64_t i0, uint32_t nt,
                                                  const uint8_t* lds) {
  const uint32_t F = s.ncols;
  const uint32_t quads = (nt + 3u) >> 2;
  // Single-blob byte planes start at c * n: with n % 4 != 0 a plane's runs
  // sit off the dword grid by ph = (c * n) % 4 bytes.  Lane l then writes
  // the aligned dword made of the last ph bytes of quad q - 1 (its left
  // neighbour's, via ds_bpermute) and its own first 4 - ph bytes.  So that
  // every such dword has a complete owner, a wave covers 63 writer quads and
  // lane 0 recomputes the quad just before them as a helper; only the
  // tile's first and last quads write single bytes.
  const bool shifted = DL == LY_PLANAR && !d.mb && (d.n & 3u);
  const uint32_t per = shifted ? 63u : 64u;
  const uint32_t gpf = (quads + per - 1u) / per;
  const uint32_t w0 = wave_id(), nw = num_waves(), lane = lane_id();
  const Div dg = make_div_dev(gpf);
  const uint32_t items = F * gpf;
  for (uint32_t it = w0; it < items; it += nw) {
    const uint32_t f = fdiv(it, dg);
    const int qi = (int)((it - f * gpf) * per + lane) - (shifted ? 1 : 0);
    // every lane takes part (the cross-lane read below needs its neighbour);
    // lanes outside the tile read record 0 and store nothing
    const bool act = qi >= 0 && qi < (int)quads;
    const uint32_t q = act ? (uint32_t)qi : 0u;
    const bool writer = act && !(shifted && lane == 0u);
    const uint32_t r = q * 4u;
    uint32_t e[ES];
    read_elems4<ES, SL>(s, lds, r, f, e);
    uint32_t col[ES];  // col[k]: byte k of records r..r+3
    if constexpr (ES == 2) {
      col[0] = __builtin_amdgcn_perm(e[1], e[0], 0x06040200u);
      col[1] = __builtin_amdgcn_perm(e[1], e[0], 0x07050301u);
    } else {
      constexpr int DW = ES / 4;
#pragma unroll
      for (int h = 0; h < DW; ++h) {
        uint32_t in[4], o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) in[j] = e[j * DW + h];
        transpose4x4(in, o);
#pragma unroll
        for (int k = 0; k < 4; ++k) col[4 * h + k] = o[k];
      }
    }
    const uint32_t nrec = !writer ? 0u : (nt - r < 4u ? nt - r : 4u);
#pragma unroll
    for (int k = 0; k < ES; ++k) {
      const uint32_t c = f * ES + k;
      const void* blob = (DL == LY_PLANAR && d.mb) ? d.blob[c] : d.blob[0];
      // the resource base is the run start aligned down to 16 bytes
      const uint64_t cb = col_base<DL>(d, i0, c);
      const uint64_t base = cb & ~15ull;
      const auto rs = make_rsrc((const uint8_t*)blob + base, d.blob_size - base);
      const uint32_t lo = (uint32_t)(cb - base) + col_local<DL>(d, r);
      const uint32_t ph = (uint32_t)cb & 3u;  // wave-uniform
      if (ph == 0u) {
        if (nrec == 4u) {
          __builtin_amdgcn_raw_buffer_store_b32(col[k], rs, lo, 0, 0);
        } else {
          for (uint32_t j = 0; j < nrec; ++j)
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(col[k] >> (8u * j)), rs, lo + j, 0, 0);
        }
      } else {
        const uint32_t prev = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((lane ? lane - 1u : 0u) * 4u), (int)col[k]);
        const uint32_t lead = 4u - ph;       // own bytes in the dword at lo - ph
        const bool has_prev = writer && q >= 1u;  // quad q - 1 is in the tile (it is lane l - 1's)
        if (has_prev && nrec >= lead) {
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_amdgcn_alignbyte(col[k], prev, lead), rs, lo - ph, 0, 0);
        } else if (writer) {  // tile's first quad, or a short last quad
          for (uint32_t j = 0; j < lead && j < nrec; ++j)
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(col[k] >> (8u * j)), rs, lo + j, 0, 0);
          if (has_prev)
            for (uint32_t j = 0; j < ph; ++j)
              __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(prev >> (8u * (lead + j))), rs, lo - ph + j, 0, 0);
        }
        // the tile's last quad: its last ph bytes have no owner in this tile
        if (writer && q + 1u == quads)
          for (uint32_t j = lead; j < nrec; ++j)
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(col[k] >> (8u * j)), rs, lo + j, 0, 0);
      }
    }
  }
}

// The 16-byte form of the split: a lane takes 16 consecutive records of one
// field and stores one 16-byte run per byte plane, so a wave writes 1 KiB
// contiguous per plane and store instruction.  Needs runs of 16 records per
// column (planar, or AoSoA with L % 16 == 0).  A single-blob plane whose
// start is off the 16-byte grid by ph bytes is written as aligned 16-byte
// windows: the last ph bytes of the left neighbour's run (ds_bpermute) and
// the lane's own first 16 - ph bytes.  As in the 4-byte form, lane 0 then
// recomputes the run just before the wave's 63 writer runs, and only a
// tile's first and last runs write single bytes.
__device__ __forceinline__ u32x4 funnel16(const u32x4& p, const u32x4& o, uint32_t ph) {
  // bytes [16 - ph, 32 - ph) of the 32-byte string p ++ o, for 0 < ph < 16
  const uint32_t d[8] = {p.x, p.y, p.z, p.w, o.x, o.y, o.z, o.w};
  const uint32_t sft = 16u - ph, dq = sft >> 2, rb = sft & 3u;
  u32x4 v;
  switch (dq) {  // wave-uniform
#define LM_F(Q)                                                                                  \
  case Q:                                                                                        \
    v = u32x4{__builtin_amdgcn_alignbyte(d[Q + 1], d[Q], rb), __builtin_amdgcn_alignbyte(d[Q + 2], d[Q + 1], rb), \
              __builtin_amdgcn_alignbyte(d[Q + 3], d[Q + 2], rb), __builtin_amdgcn_alignbyte(d[Q + 4], d[Q + 3], rb)}; \
    break;
    LM_F(0)
    LM_F(1)
    LM_F(2)
    default: LM_F(3)
#undef LM_F
  }
  return v;
}

template <int ES, int SL, int DL>
__device__ __forceinline__ void store_split_fused16(const Side& s, const Side& d, uint64_t i0, uint32_t nt,
                                                    const uint8_t* lds) {
  const uint32_t F = s.ncols;
  const uint32_t runs = (nt + 15u) >> 4;
  const bool shifted = DL == LY_PLANAR && !d.mb && (d.n & 15u);
  const uint32_t per = shifted ? 63u : 64u;
  const uint32_t gpf = (runs + per - 1u) / per;
  const uint32_t w0 = wave_id(), nw = num_waves(), lane = lane_id();
  const Div dg = make_div_dev(gpf);
  const uint32_t items = F * gpf;
  // cache policy of the full-window stores (measured): non-temporal from
  // multi-segment sources, plain from an AoS source
  constexpr int kPol = SL == LY_AOS ? 0 : kStoreNT;
  for (uint32_t it = w0; it < items; it += nw) {
    const uint32_t f = fdiv(it, dg);
    const int qi = (int)((it - f * gpf) * per + lane) - (shifted ? 1 : 0);
    const bool act = qi >= 0 && qi < (int)runs;
    const uint32_t q = act ? (uint32_t)qi : 0u;
    const bool writer = act && !(shifted && lane == 0u);
    const uint32_t r = q * 16u;
    uint32_t col[ES][4];  // col[k][m]: byte k of records r + 4m .. r + 4m + 3
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      uint32_t e[ES];
      read_elems4<ES, SL>(s, lds, r + 4u * m, f, e);
      if constexpr (ES == 2) {
        col[0][m] = __builtin_amdgcn_perm(e[1], e[0], 0x06040200u);
        col[1][m] = __builtin_amdgcn_perm(e[1], e[0], 0x07050301u);
      } else {
        constexpr int DW = ES / 4;
#pragma unroll
        for (int h = 0; h < DW; ++h) {
          uint32_t in[4], o[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) in[j] = e[j * DW + h];
          transpose4x4(in, o);
#pragma unroll
          for (int k = 0; k < 4; ++k) col[4 * h + k][m] = o[k];
        }
      }
    }
    const uint32_t nrec = !writer ? 0u : (nt - r < 16u ? nt - r : 16u);
#pragma unroll
    for (int k = 0; k < ES; ++k) {
      const uint32_t c = f * ES + k;
      const void* blob = (DL == LY_PLANAR && d.mb) ? d.blob[c] : d.blob[0];
      const uint64_t cb = col_base<DL>(d, i0, c);
      const uint64_t base = cb & ~15ull;
      const auto rs = make_rsrc((const uint8_t*)blob + base, d.blob_size - base);
      const uint32_t lo = (uint32_t)(cb - base) + col_local<DL>(d, r);
      const uint32_t ph = (uint32_t)cb & 15u;  // wave-uniform
      const u32x4 own = u32x4{col[k][0], col[k][1], col[k][2], col[k][3]};
      auto own_byte = [&](uint32_t j) { return (uint8_t)(col[k][j >> 2] >> (8u * (j & 3u))); };
      if (ph == 0u) {
        if (nrec == 16u) {
          __builtin_amdgcn_raw_buffer_store_b128(own, rs, lo, 0, kPol);
        } else {
          for (uint32_t j = 0; j < nrec; ++j) __builtin_amdgcn_raw_buffer_store_b8(own_byte(j), rs, lo + j, 0, 0);
        }
      } else {
        const int src_lane = (int)((lane ? lane - 1u : 0u) * 4u);
        const u32x4 prev = u32x4{(uint32_t)__builtin_amdgcn_ds_bpermute(src_lane, (int)own.x),
                                 (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane, (int)own.y),
                                 (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane, (int)own.z),
                                 (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane, (int)own.w)};
        const uint32_t lead = 16u - ph;       // own bytes in the window at lo - ph
        const bool has_prev = writer && q >= 1u;  // run q - 1 is in the tile (lane l - 1's)
        if (has_prev && nrec >= lead) {
          __builtin_amdgcn_raw_buffer_store_b128(funnel16(prev, own, ph), rs, lo - ph, 0, kPol);
        } else if (writer) {  // the tile's first run, or a short last run
          for (uint32_t j = 0; j < lead && j < nrec; ++j)
            __builtin_amdgcn_raw_buffer_store_b8(own_byte(j), rs, lo + j, 0, 0);
          if (has_prev)
            for (uint32_t j = 0; j < ph; ++j) {
              const uint32_t b = lead + j;  // byte of the neighbour's run
              __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(prev[b >> 2] >> (8u * (b & 3u))), rs, lo - ph + j, 0, 0);
            }
        }
        // the tile's last run: its last ph bytes have no owner in this tile
        if (writer && q + 1u == runs)
          for (uint32_t j = lead; j < nrec; ++j) __builtin_amdgcn_raw_buffer_store_b8(own_byte(j), rs, lo + j, 0, 0);
      }
    }
  }
}

// The 16-byte split with line-owner writes (single-blob byte planes off the
// line grid, see store_lines): the tile's source image holds its records and
// the halo (nl records), lanes take runs of 16 records of one field as in
// store_split_fused16, and the 16-byte window that starts ph bytes before a
// lane's run (ph = the plane's phase mod 16) is written when it lies inside
// the bytes the tile owns in that plane.  Window w joins the last ph bytes of
// run w - 1 (the left neighbour's) and the first 16 - ph bytes of run w; lane
// 0 of each wave only supplies its run to lane 1, and one window past the
// last run carries that run's last ph bytes.  No byte is written twice and
// every owned line is written whole; only the planes' ends use byte stores.
template <int ES, int SL>
__device__ __forceinline__ void store_split_lines16(const Side& s, const Side& d, uint64_t i0, uint32_t nt,
                                                    uint32_t nl, const uint8_t* lds) {
  const uint32_t F = s.ncols;
  const uint32_t runs = (nl + 15u) >> 4;
  const uint32_t wins = runs + 1u;
  const uint32_t gpf = (wins + 62u) / 63u;
  const uint32_t w0 = wave_id(), nw = num_waves(), lane = lane_id();
  const Div dg = make_div_dev(gpf);
  const uint32_t items = F * gpf;
  const bool first = i0 == 0, last = i0 + nt >= d.n;
  for (uint32_t it = w0; it < items; it += nw) {
    const uint32_t f = fdiv(it, dg);
    const int qi = (int)((it - f * gpf) * 63u + lane) - 1;
    const bool has = qi >= 0 && qi < (int)runs;  // a run of the tile's image
    const uint32_t q = qi >= 0 ? (uint32_t)qi : 0u;  // the lane's run and window
    const bool writer = lane != 0u && qi >= 0 && qi < (int)wins;
    const uint32_t r = has ? q * 16u : 0u;
    uint32_t col[ES][4];  // col[k][m]: byte k of records r + 4m .. r + 4m + 3
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      uint32_t e[ES];
      read_elems4<ES, SL>(s, lds, r + 4u * m, f, e);
      if constexpr (ES == 2) {
        col[0][m] = __builtin_amdgcn_perm(e[1], e[0], 0x06040200u);
        col[1][m] = __builtin_amdgcn_perm(e[1], e[0], 0x07050301u);
      } else {
        constexpr int DW = ES / 4;
#pragma unroll
        for (int h = 0; h < DW; ++h) {
          uint32_t in[4], o[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) in[j] = e[j * DW + h];
          transpose4x4(in, o);
#pragma unroll
          for (int k = 0; k < 4; ++k) col[4 * h + k][m] = o[k];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < ES; ++k) {
      const uint32_t c = f * ES + k;
      const uint64_t p0 = d.n * c, pe = p0 + d.n;  // byte plane c in the blob
      const uint64_t t0 = p0 + i0, te = t0 + nt;
      const uint64_t b0 = first ? t0 : (t0 + 127u) & ~127ull;
      uint64_t b1 = last ? pe : (te + 127u) & ~127ull;
      if (b1 > pe) b1 = pe;
      const uint32_t ph = (uint32_t)t0 & 15u;  // wave-uniform
      const u32x4 own = has ? u32x4{col[k][0], col[k][1], col[k][2], col[k][3]} : u32x4{0u, 0u, 0u, 0u};
      const int src_lane = (int)((lane ? lane - 1u : 0u) * 4u);
      const u32x4 prev = u32x4{(uint32_t)__builtin_amdgcn_ds_bpermute(src_lane, (int)own.x),
                               (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane, (int)own.y),
                               (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane, (int)own.z),
                               (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane, (int)own.w)};
      if (!writer) continue;
      const uint64_t ws = t0 + 16ull * q - ph;  // the window, 16-byte aligned
      if (ws >= b1 || ws + 16u <= b0) continue;
      const uint64_t base = ws & ~127ull;
      const auto rs = make_rsrc((const uint8_t*)d.blob[0] + base, d.blob_size - base);
      const uint32_t lo = (uint32_t)(ws - base);
      if (ws >= b0 && ws + 16u <= b1) {
        __builtin_amdgcn_raw_buffer_store_b128(ph ? funnel16(prev, own, ph) : own, rs, lo, 0, kStoreNT);
      } else {
        for (uint32_t j = 0; j < 16u; ++j) {
          const uint64_t gb = ws + j;
          if (gb < b0 || gb >= b1) continue;
          const uint32_t b = j < ph ? 16u - ph + j : j - ph;  // byte of the neighbour's run, or of the own run
          const u32x4& src = j < ph ? prev : own;
          __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(src[b >> 2] >> (8u * (b & 3u))), rs, lo + j, 0, 0);
        }
      }
    }
  }
}

// Line-owner writes of columns that keep their size (element planes from
// element columns, byte planes from byte columns): as store_split_lines16,
// with a lane's run being 16 bytes of one column (16 / U records) read
// straight from the tile's source image.
template <int U, int SL>
__device__ __forceinline__ u32x4 read_col16(const Side& s, const uint8_t* lds, uint32_t r, uint32_t c) {
  if constexpr (U == 1) {
    return u32x4{read_run4<SL>(s, lds, r, c), read_run4<SL>(s, lds, r + 4u, c), read_run4<SL>(s, lds, r + 8u, c),
                 read_run4<SL>(s, lds, r + 12u, c)};
  } else if constexpr (U == 2) {
    uint32_t e0[2], e1[2];
    read_elems4<2, SL>(s, lds, r, c, e0);
    read_elems4<2, SL>(s, lds, r + 4u, c, e1);
    return u32x4{e0[0], e0[1], e1[0], e1[1]};
  } else if constexpr (U == 4) {
    uint32_t e[4];
    read_elems4<4, SL>(s, lds, r, c, e);
    return u32x4{e[0], e[1], e[2], e[3]};
  } else {
    const u32x2 a = *(const u32x2*)(lds + src_addr<SL>(s, r, c * 8u));
    const u32x2 b = *(const u32x2*)(lds + src_addr<SL>(s, r + 1u, c * 8u));
    return u32x4{a.x, a.y, b.x, b.y};
  }
}

// 16 bytes of element column f (16 / ES records from r) merged from the ES
// byte columns of a Bytesplit source image.
template <int ES, int SL>
__device__ __forceinline__ u32x4 read_merge16(const Side& s, const uint8_t* lds, uint32_t r, uint32_t f) {
  if constexpr (ES == 2) {
    uint32_t o[4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t b0 = read_run4<SL>(s, lds, r + 4u * h, 2 * f), b1 = read_run4<SL>(s, lds, r + 4u * h, 2 * f + 1);
      o[2 * h] = __builtin_amdgcn_perm(b1, b0, 0x05010400u);
      o[2 * h + 1] = __builtin_amdgcn_perm(b1, b0, 0x07030602u);
    }
    return u32x4{o[0], o[1], o[2], o[3]};
  } else {
    // byte runs come in aligned groups of 4 records: merge the group that
    // holds records r, r + 1 (ES = 8) or r .. r + 3 (ES = 4), keep 16 bytes
    constexpr int DW = ES / 4;
    const uint32_t r4 = r & ~3u;
    uint32_t out[ES];
#pragma unroll
    for (int h = 0; h < DW; ++h) {
      uint32_t in[4], o[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) in[k] = read_run4<SL>(s, lds, r4, f * ES + 4 * h + k);
      transpose4x4(in, o);
#pragma unroll
      for (int j = 0; j < 4; ++j) out[j * DW + h] = o[j];
    }
    if constexpr (ES == 8) {
      if (r != r4) return u32x4{out[4], out[5], out[6], out[7]};
    }
    return u32x4{out[0], out[1], out[2], out[3]};
  }
}

// Line-owner writes of destination columns of U bytes (see store_lines): a
// lane's run is 16 bytes of one column (16 / U records), given by read(r, c);
// the 16-byte window starting ph bytes before it joins the left neighbour's
// last ph bytes and the run's first 16 - ph bytes, and is written when it
// lies in the bytes the tile owns.  Lane 0 of each wave only supplies its
// run; one window past the last run carries that run's last ph bytes.
template <int U, typename Read>
__device__ __forceinline__ void store_lines16(const Side& d, uint64_t i0, uint32_t nt, uint32_t nl, uint32_t C,
                                              Read&& read) {
  constexpr uint32_t R = 16u / U;  // records per run
  const uint32_t runs = (nl + R - 1u) / R;
  const uint32_t wins = runs + 1u;
  const uint32_t gpf = (wins + 62u) / 63u;
  const uint32_t w0 = wave_id(), nw = num_waves(), lane = lane_id();
  const Div dg = make_div_dev(gpf);
  const uint32_t items = C * gpf;
  const bool first = i0 == 0, last = i0 + nt >= d.n;
  const uint64_t plane = d.n * U;
  for (uint32_t it = w0; it < items; it += nw) {
    const uint32_t c = fdiv(it, dg);
    const int qi = (int)((it - c * gpf) * 63u + lane) - 1;
    const bool has = qi >= 0 && qi < (int)runs;
    const uint32_t q = qi >= 0 ? (uint32_t)qi : 0u;
    const bool writer = lane != 0u && qi >= 0 && qi < (int)wins;
    const u32x4 own = has ? read(q * R, c) : u32x4{0u, 0u, 0u, 0u};
    const uint64_t p0 = plane * c, pe = p0 + plane;
    const uint64_t t0 = p0 + i0 * U, te = t0 + (uint64_t)nt * U;
    const uint64_t b0 = first ? t0 : (t0 + 127u) & ~127ull;
    uint64_t b1 = last ? pe : (te + 127u) & ~127ull;
    if (b1 > pe) b1 = pe;
    const uint32_t ph = (uint32_t)t0 & 15u;  // wave-uniform
    const int src_lane = (int)((lane ? lane - 1u : 0u) * 4u);
    const u32x4 prev = u32x4{(uint32_t)__builtin_amdgcn_ds_bpermute(src_lane, (int)own.x),
                             (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane, (int)own.y),
                             (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane, (int)own.z),
                             (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane, (int)own.w)};
    if (!writer) continue;
    const uint64_t ws = t0 + 16ull * q - ph;
    if (ws >= b1 || ws + 16u <= b0) continue;
    const uint64_t base = ws & ~127ull;
    const auto rs = make_rsrc((const uint8_t*)d.blob[0] + base, d.blob_size - base);
    const uint32_t lo = (uint32_t)(ws - base);
    if (ws >= b0 && ws + 16u <= b1) {
      __builtin_amdgcn_raw_buffer_store_b128(ph ? funnel16(prev, own, ph) : own, rs, lo, 0, kStoreNT);
    } else {
      for (uint32_t j = 0; j < 16u; ++j) {
        const uint64_t gb = ws + j;
        if (gb < b0 || gb >= b1) continue;
        const uint32_t b = j < ph ? 16u - ph + j : j - ph;
        const u32x4& src = j < ph ? prev : own;
        __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(src[b >> 2] >> (8u * (b & 3u))), rs, lo + j, 0, 0);
      }
    }
  }
}

template <int ES, int SL, int DL>
__device__ __forceinline__ void store_merge_fused(const Side& s, const Side& d, uint64_t i0, uint32_t nt,
                                                  const uint8_t* lds) {
  const uint32_t F = d.ncols;
  const uint32_t quads = (nt + 3u) >> 2;
  const uint32_t gpf = (quads + 63u) >> 6;
  const uint32_t w0 = wave_id(), nw = num_waves(), lane = lane_id();
  const Div dg = make_div_dev(gpf);
  const uint32_t items = F * gpf;
  for (uint32_t it = w0; it < items; it += nw) {
    const uint32_t f = fdiv(it, dg);
    const uint32_t q = (it - f * gpf) * 64u + lane;
    const void* blob = (DL == LY_PLANAR && d.mb) ? d.blob[f] : d.blob[0];
    const uint64_t cb = col_base<DL>(d, i0, f);
    const uint64_t base = cb & ~15ull;
    const auto rs = make_rsrc((const uint8_t*)blob + base, d.blob_size - base);
    if (q >= quads) continue;
    const uint32_t r = q * 4u;
    uint32_t out[ES];  // the 4 elements, as ES dwords
    if constexpr (ES == 2) {
      const uint32_t b0 = read_run4<SL>(s, lds, r, 2 * f), b1 = read_run4<SL>(s, lds, r, 2 * f + 1);
      out[0] = __builtin_amdgcn_perm(b1, b0, 0x05010400u);
      out[1] = __builtin_amdgcn_perm(b1, b0, 0x07030602u);
    } else {
      constexpr int DW = ES / 4;
#pragma unroll
      for (int h = 0; h < DW; ++h) {
        uint32_t in[4], o[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) in[k] = read_run4<SL>(s, lds, r, f * ES + 4 * h + k);
        transpose4x4(in, o);
#pragma unroll
        for (int j = 0; j < 4; ++j) out[j * DW + h] = o[j];
      }
    }
    const uint32_t lo = (uint32_t)(cb - base) + col_local<DL>(d, r);
    const uint32_t nrec = nt - r < 4u ? nt - r : 4u;
    // a single-blob plane may start off the 16-byte grid (wave-uniform
    // phase): then the widest store its alignment allows
    const uint32_t ph = (uint32_t)cb & 15u;
    if (nrec == 4u) {
      if constexpr (ES == 2) {
        if ((ph & 7u) == 0u) {
          __builtin_amdgcn_raw_buffer_store_b64(u32x2{out[0], out[1]}, rs, lo, 0, kStoreNT);
        } else if ((ph & 3u) == 0u) {
          __builtin_amdgcn_raw_buffer_store_b32(out[0], rs, lo, 0, kStoreNT);
          __builtin_amdgcn_raw_buffer_store_b32(out[1], rs, lo + 4u, 0, kStoreNT);
        } else {
#pragma unroll
          for (uint32_t j = 0; j < 4u; ++j)
            __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(out[j >> 1] >> (16u * (j & 1u))), rs, lo + 2u * j, 0,
                                                  kStoreNT);
        }
      } else if (ph == 0u) {
#pragma unroll
        for (int q4 = 0; q4 < ES / 4; ++q4)
          __builtin_amdgcn_raw_buffer_store_b128(u32x4{out[4 * q4], out[4 * q4 + 1], out[4 * q4 + 2], out[4 * q4 + 3]},
                                                 rs, lo + 16u * q4, 0, kStoreNT);
      } else if ((ph & 7u) == 0u) {
#pragma unroll
        for (int q2 = 0; q2 < ES / 2; ++q2)
          __builtin_amdgcn_raw_buffer_store_b64(u32x2{out[2 * q2], out[2 * q2 + 1]}, rs, lo + 8u * q2, 0, kStoreNT);
      } else {
#pragma unroll
        for (int j = 0; j < ES; ++j) __builtin_amdgcn_raw_buffer_store_b32(out[j], rs, lo + 4u * j, 0, kStoreNT);
      }
    } else if constexpr (ES == 2) {
      for (uint32_t j = 0; j < nrec; ++j)
        __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(out[j >> 1] >> (16u * (j & 1u))), rs, lo + 2u * j, 0, 0);
    } else {
      for (uint32_t j = 0; j < nrec * (ES / 4u); ++j) __builtin_amdgcn_raw_buffer_store_b32(out[j], rs, lo + 4u * j, 0, 0);
    }
  }
}

// ---------------------------------------------------------------------------
// Element access for conversions and codecs
// ---------------------------------------------------------------------------

// Stored element of field f (ES bytes) of tile-local record r from the source
// tile in LDS; a Bytesplit source (cs = 1) is gathered byte by byte.
template <int ES, int SL>
__device__ __forceinline__ uint64_t fetch_elem(const Side& s, const uint8_t* lds, uint32_t r, uint32_t f) {
  if (s.cs == (uint32_t)ES) return lds_read<ES>(lds, src_addr<SL>(s, r, f * ES));
  uint64_t v = 0;
#pragma unroll
  for (int k = 0; k < ES; ++k) v |= (uint64_t)lds[src_addr<SL>(s, r, f * ES + k)] << (8 * k);
  return v;
}

// ChangeType conversions (Sec. 3): the hardware conversion instructions,
// with NaN made quiet and keeping its top payload bits.
__device__ __forceinline__ uint32_t cvt_f64_f32(uint64_t x) {
  const float f = (float)__builtin_bit_cast(double, x);  // v_cvt_f32_f64, round to nearest even
  const uint32_t r = __builtin_bit_cast(uint32_t, f);
  const bool nan = (x & 0x7FFFFFFFFFFFFFFFull) > 0x7FF0000000000000ull;
  const uint32_t rn = ((uint32_t)(x >> 32) & 0x80000000u) | 0x7FC00000u | (uint32_t)((x >> 29) & 0x7FFFFFu);
  return nan ? rn : r;
}

__device__ __forceinline__ uint64_t cvt_f32_f64(uint32_t x) {
  const double d = (double)__builtin_bit_cast(float, x);  // v_cvt_f64_f32, exact
  const uint64_t r = __builtin_bit_cast(uint64_t, d);
  const bool nan = (x & 0x7FFFFFFFu) > 0x7F800000u;
  const uint64_t rn = ((uint64_t)(x >> 31) << 63) | 0x7FF8000000000000ull | ((uint64_t)(x & 0x7FFFFFu) << 29);
  return nan ? rn : r;
}

// Generic ChangeType conversions between IEEE binary formats given by their
// exponent and mantissa widths (f64 11/52, f32 8/23, f16 5/10, bf16 8/7).
//
// Narrowing rounds to nearest, ties to even.  The value is the source
// significand (hidden bit at MS) scaled by its exponent; it is shifted so the
// hidden bit lands on bit MD, or lower for a target subnormal, and the
// dropped bits decide the rounding.  Adding (exponent - 1) << MD to a
// significand that still carries its hidden bit lets a rounding carry move
// into the exponent by itself.  Codes at or past the Inf code become Inf.
// A NaN keeps its sign and top MD payload bits and gets the quiet bit.
// Both work in 32-bit words when source and target fit in them (W).
template <int ES, int MS, int ED, int MD>
using ConvWord = typename std::conditional<(ES + MS < 32 && ED + MD < 32), uint32_t, uint64_t>::type;

template <int ES, int MS, int ED, int MD>
__device__ __forceinline__ uint64_t narrow_rne(uint64_t x64) {
  using W = ConvWord<ES, MS, ED, MD>;
  const W x = (W)x64;
  constexpr int emax_s = (1 << ES) - 1, emax_d = (1 << ED) - 1;
  constexpr int bias_s = (1 << (ES - 1)) - 1, bias_d = (1 << (ED - 1)) - 1;
  const W sign = (x >> (ES + MS)) & (W)1;
  const W m = x & (((W)1 << MS) - (W)1);
  const int es = (int)((x >> MS) & (W)emax_s);
  W code;
  if (es == emax_s) {
    code = ((W)emax_d << MD) | (m ? ((m >> (MS - MD)) | ((W)1 << (MD - 1))) : (W)0);
  } else {
    const W sig = es ? (m | ((W)1 << MS)) : m;
    const int ed = (es ? es : 1) - bias_s + bias_d;  // target exponent field of the hidden-bit position
    const int sh = MS - MD + (ed < 1 ? 1 - ed : 0);  // >= 1: the formats narrow
    W q = 0;
    if (sh <= MS + 1) {  // otherwise the value is below half the smallest subnormal
      q = sig >> sh;
      const W rem = sig & (((W)1 << sh) - (W)1), half = (W)1 << (sh - 1);
      q += (rem > half || (rem == half && (q & (W)1))) ? (W)1 : (W)0;
    }
    code = ed >= 1 ? ((W)(ed - 1) << MD) + q : q;
    const W inf = (W)emax_d << MD;
    code = code >= inf ? inf : code;
  }
  return code | (sign << (ED + MD));
}

// Widening is exact: a source subnormal becomes a target normal when the
// target exponent range is wider (a subnormal when it is the same); a NaN's
// payload moves up and the quiet bit is set.
template <int ES, int MS, int ED, int MD>
__device__ __forceinline__ uint64_t widen(uint64_t x64) {
  using W = ConvWord<ES, MS, ED, MD>;
  const W x = (W)x64;
  constexpr int emax_s = (1 << ES) - 1, emax_d = (1 << ED) - 1;
  constexpr int bias_s = (1 << (ES - 1)) - 1, bias_d = (1 << (ED - 1)) - 1;
  const W sign = (x >> (ES + MS)) & (W)1;
  const W m = x & (((W)1 << MS) - (W)1);
  const int es = (int)((x >> MS) & (W)emax_s);
  W code;
  if (es == emax_s) {
    code = ((W)emax_d << MD) | (m << (MD - MS)) | (m ? ((W)1 << (MD - 1)) : (W)0);
  } else if (es == 0) {
    if (m == 0) {
      code = 0;
    } else if constexpr (ED == ES) {  // same exponent range: still a subnormal
      code = m << (MD - MS);
    } else {  // m * 2^(1 - bias_s - MS), a normal of the wider range
      const int p = 63 - __builtin_clzll((uint64_t)m);
      code = ((W)(p + 1 - bias_s - MS + bias_d) << MD) | ((m ^ ((W)1 << p)) << (MD - p));
    }
  } else {
    code = ((W)(es - bias_s + bias_d) << MD) | (m << (MD - MS));
  }
  return code | (sign << (ED + MD));
}

// BitPackedFloatSoA codes (Sec. 3): [sign | E | M], bias 2^(E-1)-1,
// mantissa truncated, overflow -> Inf, gradual underflow, NaN kept quiet.
__device__ __forceinline__ uint32_t enc_f32(uint32_t x, uint32_t E, uint32_t M) {
  const uint32_t sh = 23u - M;
  const uint32_t bias = (1u << (E - 1u)) - 1u;
  const uint32_t emin = 128u - bias;  // smallest source exponent field with a target normal
  const uint32_t inf_code = ((1u << E) - 1u) << M;
  const uint32_t ax = x & 0x7FFFFFFFu;
  const uint32_t t = ax >> sh;  // (exponent field << M) | truncated mantissa
  // target normal: rebias the exponent field.  A finite value past the
  // target range lands at or above the Inf code, so the min maps it to Inf.
  const uint32_t c_norm = min(t - ((emin - 1u) << M), inf_code);
  // target subnormal: |x| in units of the smallest target subnormal,
  // 2^(1 - bias - M), truncated.  Scaling by powers of two is exact here
  // (two factors keep each one finite) and the float-to-integer conversion
  // truncates.
  const uint32_t k = bias + M - 1u;  // 0 .. 149
  const uint32_t k1 = k < 127u ? k : 127u;
  const float s1 = __builtin_bit_cast(float, (k1 + 127u) << 23), s2 = __builtin_bit_cast(float, (k - k1 + 127u) << 23);
  const float mag = __builtin_bit_cast(float, ax) * s1 * s2;
  const uint32_t c_sub = ax < (emin << 23) ? (uint32_t)mag : 0u;
  // NaN: quiet, keeping the top mantissa bits (with M = 0 it becomes Inf)
  const uint32_t quiet = M ? (1u << (M - 1u)) : 0u;
  const uint32_t c_nan = inf_code | quiet | (t & ((1u << M) - 1u));
  uint32_t c = ax >= (emin << 23) ? c_norm : c_sub;
  c = ax > 0x7F800000u ? c_nan : c;
  return c | ((x >> 31) << (E + M));
}

// Round-to-nearest-even forms (mapping flag): the dropped mantissa bits of a
// target normal round the code up (a carry moves into the exponent, past the
// largest finite code to Inf); a target subnormal is the scaled magnitude
// rounded to the nearest integer, ties to even (exact scaling, rint).  Ties
// compare the significand's last bit: the mantissa's, or the hidden bit when
// M = 0, which rounds a tie away from zero.
__device__ __forceinline__ uint32_t enc_f32_rne(uint32_t x, uint32_t E, uint32_t M) {
  const uint32_t sh = 23u - M;
  const uint32_t bias = (1u << (E - 1u)) - 1u;
  const uint32_t emin = 128u - bias;
  const uint32_t inf_code = ((1u << E) - 1u) << M;
  const uint32_t ax = x & 0x7FFFFFFFu;
  const uint32_t t = ax >> sh;
  const uint32_t rem = ax & ((1u << sh) - 1u), half = sh ? (1u << (sh - 1u)) : 0u;
  const uint32_t odd = M ? (t & 1u) : 1u;
  const uint32_t up = (sh != 0u) && (rem > half || (rem == half && odd)) ? 1u : 0u;
  const uint32_t c_norm = min(t + up - ((emin - 1u) << M), inf_code);
  const uint32_t k = bias + M - 1u;
  const uint32_t k1 = k < 127u ? k : 127u;
  const float s1 = __builtin_bit_cast(float, (k1 + 127u) << 23), s2 = __builtin_bit_cast(float, (k - k1 + 127u) << 23);
  const float mag = __builtin_bit_cast(float, ax) * s1 * s2;
  const uint32_t c_sub = ax < (emin << 23) ? (uint32_t)__builtin_rintf(mag) : 0u;
  const uint32_t quiet = M ? (1u << (M - 1u)) : 0u;
  const uint32_t c_nan = inf_code | quiet | (t & ((1u << M) - 1u));
  uint32_t c = ax >= (emin << 23) ? c_norm : c_sub;
  c = ax > 0x7F800000u ? c_nan : c;
  return c | ((x >> 31) << (E + M));
}

__device__ __forceinline__ uint32_t enc_f64_rne(uint64_t x, uint32_t E, uint32_t M) {
  const uint32_t sh = 52u - M;  // >= 21: codes have at most 32 bits
  const uint32_t bias = (1u << (E - 1u)) - 1u;
  const uint32_t emin = 1024u - bias;
  const uint64_t inf_code = (uint64_t)(((1u << E) - 1u) << M);
  const uint64_t ax = x & 0x7FFFFFFFFFFFFFFFull;
  const uint64_t t = ax >> sh;
  const uint64_t rem = ax & ((1ull << sh) - 1ull), half = 1ull << (sh - 1u);
  const uint64_t odd = M ? (t & 1ull) : 1ull;
  const uint64_t up = (rem > half || (rem == half && odd)) ? 1ull : 0ull;
  const uint64_t cn = t + up - ((uint64_t)(emin - 1u) << M);
  const uint32_t c_norm = (uint32_t)(cn < inf_code ? cn : inf_code);
  const uint32_t k = bias + M - 1u;  // 0 .. 1051
  const uint32_t k1 = k < 1023u ? k : 1023u;
  const double s1 = __builtin_bit_cast(double, (uint64_t)(k1 + 1023u) << 52);
  const double s2 = __builtin_bit_cast(double, (uint64_t)(k - k1 + 1023u) << 52);
  const double mag = __builtin_bit_cast(double, ax) * s1 * s2;
  const uint32_t c_sub = ax < ((uint64_t)emin << 52) ? (uint32_t)__builtin_rint(mag) : 0u;
  const uint32_t quiet = M ? (1u << (M - 1u)) : 0u;
  const uint32_t c_nan = (uint32_t)inf_code | quiet | (uint32_t)(t & ((1ull << M) - 1ull));
  uint32_t c = ax >= ((uint64_t)emin << 52) ? c_norm : c_sub;
  c = ax > 0x7FF0000000000000ull ? c_nan : c;
  return c | ((uint32_t)(x >> 63) << (E + M));
}

__device__ __forceinline__ uint32_t dec_f32(uint32_t c, uint32_t E, uint32_t M) {
  const uint32_t sh = 23u - M;
  const uint32_t bias = (1u << (E - 1u)) - 1u;
  const uint32_t emax = (1u << E) - 1u;
  const uint32_t cm = c & ((1u << (E + M)) - 1u);  // code without its sign
  // normal, Inf and NaN codes: exponent and mantissa fields move up as one;
  // the exponent field is then rebiased (Inf / NaN: to all ones)
  const uint32_t up = cm >= (emax << M) ? (255u - emax) << 23 : (127u - bias) << 23;
  const uint32_t r_norm = (cm << sh) + up;
  // subnormal codes (and zero): m * 2^(1 - bias - M), exact in float32
  // (an integer below 2^23 times a power of two)
  const int ex = 1 - (int)bias - (int)M;  // >= -149
  const float p2 = ex >= -126 ? __builtin_bit_cast(float, (uint32_t)(ex + 127) << 23)
                              : __builtin_bit_cast(float, 1u << (ex + 149));
  const uint32_t r_sub = __builtin_bit_cast(uint32_t, (float)cm * p2);
  const uint32_t r = cm < (1u << M) ? r_sub : r_norm;
  return r | ((c >> (E + M)) << 31);
}

__device__ __forceinline__ uint32_t enc_f64(uint64_t x, uint32_t E, uint32_t M) {
  const uint32_t sh = 52u - M;
  const uint32_t bias = (1u << (E - 1u)) - 1u;
  const uint32_t emin = 1024u - bias;
  const uint32_t emaxf = 1023u + bias;
  const uint32_t inf_code = ((1u << E) - 1u) << M;
  const uint64_t ax = x & 0x7FFFFFFFFFFFFFFFull, m = ax & 0xFFFFFFFFFFFFFull;
  const uint32_t e = (uint32_t)(ax >> 52);
  const uint32_t c_norm = ((e - emin + 1u) << M) | (uint32_t)(m >> sh);
  const uint64_t sig = e ? (m | 0x10000000000000ull) : m;
  const uint32_t dsh = emin - (e ? e : 1u) + sh;
  const uint32_t c_sub = dsh < 64u ? (uint32_t)(sig >> dsh) : 0u;
  const uint32_t quiet = M ? (1u << (M - 1u)) : 0u;
  const uint32_t c_inf = inf_code | ((ax > 0x7FF0000000000000ull && M) ? ((uint32_t)(m >> sh) | quiet) : 0u);
  const uint32_t c = e > emaxf ? c_inf : (e >= emin ? c_norm : c_sub);
  return c | ((uint32_t)(x >> 63) << (E + M));
}

__device__ __forceinline__ uint64_t dec_f64(uint32_t c, uint32_t E, uint32_t M) {
  const uint32_t sh = 52u - M;
  const uint32_t bias = (1u << (E - 1u)) - 1u;
  const uint32_t emax = (1u << E) - 1u;
  const uint32_t e = (c >> M) & emax, m = c & ((1u << M) - 1u);
  const uint64_t sign = (uint64_t)((c >> (E + M)) & 1u) << 63;
  uint64_t r;
  if (e == emax) {
    r = 0x7FF0000000000000ull | ((uint64_t)m << sh);
  } else if (e) {
    r = ((uint64_t)(e + 1023u - bias) << 52) | ((uint64_t)m << sh);
  } else if (m == 0u) {
    r = 0ull;
  } else {
    const int p = 31 - __builtin_clz(m);
    const int u = 1 - (int)bias - (int)M + p;
    r = u >= -1022 ? (((uint64_t)(u + 1023) << 52) | ((uint64_t)(m ^ (1u << p)) << (52 - p)))
                   : ((uint64_t)m << sh);
  }
  return r | sign;
}

// user element -> code (pack)
template <int CODEC>
__device__ __forceinline__ uint32_t encode(uint64_t v, const Side& d) {
  if constexpr (CODEC == CD_F32)
    return d.rne ? enc_f32_rne((uint32_t)v, d.exp_bits, d.man_bits) : enc_f32((uint32_t)v, d.exp_bits, d.man_bits);
  else if constexpr (CODEC == CD_F64)
    return d.rne ? enc_f64_rne(v, d.exp_bits, d.man_bits) : enc_f64(v, d.exp_bits, d.man_bits);
  else return (uint32_t)v & (d.bits >= 32u ? 0xFFFFFFFFu : ((1u << d.bits) - 1u));
}

// code -> user element bits (unpack)
template <int CODEC>
__device__ __forceinline__ uint64_t decode(uint32_t c, const Side& s) {
  if constexpr (CODEC == CD_F32) return dec_f32(c, s.exp_bits, s.man_bits);
  else if constexpr (CODEC == CD_F64) return dec_f64(c, s.exp_bits, s.man_bits);
  else {
    constexpr bool SGN = CODEC == CD_I8 || CODEC == CD_I16 || CODEC == CD_I32 || CODEC == CD_I64;
    if constexpr (SGN) {
      const int32_t v = s.bits >= 32u ? (int32_t)c : ((int32_t)(c << (32u - s.bits)) >> (32u - s.bits));
      return (uint64_t)(int64_t)v;
    } else {
      return (uint64_t)c;
    }
  }
}

template <int CODEC>
struct CodecInfo {
  static constexpr int ES = (CODEC == CD_U8 || CODEC == CD_I8) ? 1
                          : (CODEC == CD_U16 || CODEC == CD_I16) ? 2
                          : (CODEC == CD_U32 || CODEC == CD_I32 || CODEC == CD_F32) ? 4 : 8;
};

// code of tile-local value r from an LDS bit-stream plane (B <= 32)
__device__ __forceinline__ uint32_t stream_code(const uint8_t* plane, uint32_t r, uint32_t B) {
  const uint32_t p = r * B;
  const uint32_t* wp = (const uint32_t*)plane + (p >> 5);
  const uint32_t lo = wp[0], hi = wp[1];
  const uint32_t v = __builtin_amdgcn_alignbit(hi, lo, p & 31u);
  return B >= 32u ? v : (v & ((1u << B) - 1u));
}

// ---------------------------------------------------------------------------
// Phase B, ChangeType conversion.  Units are destination storage bytes of
// U = (destination column size); the source element is read whole.
// ---------------------------------------------------------------------------

template <int CONV>
struct ConvInfo {
  static constexpr int ES_SRC = (CONV == CV_F64_F32 || CONV == CV_F64_F16 || CONV == CV_F64_BF16) ? 8
                                : (CONV == CV_F32_F64 || CONV == CV_F32_F16 || CONV == CV_F32_BF16) ? 4
                                                                                                     : 2;
  static constexpr int ES_DST = (CONV == CV_F32_F64 || CONV == CV_F16_F64 || CONV == CV_BF16_F64) ? 8
                                : (CONV == CV_F64_F32 || CONV == CV_F16_F32 || CONV == CV_BF16_F32) ? 4
                                                                                                     : 2;
};

// f32 -> f16 and f32 -> bf16 with the hardware conversions (v_cvt_f16_f32,
// v_cvt_pk_bf16_f32): both round to nearest even under the kernel's FP mode,
// which keeps denormals, and overflow to Inf.  A NaN is rewritten with the
// ChangeType rule: sign, top payload bits, quiet bit set.
__device__ __forceinline__ uint32_t cvt_f32_f16(uint32_t x) {
  const uint32_t h = __builtin_bit_cast(uint16_t, (_Float16)__builtin_bit_cast(float, x));
  const bool nan = (x & 0x7FFFFFFFu) > 0x7F800000u;
  const uint32_t hn = ((x >> 16) & 0x8000u) | 0x7E00u | ((x >> 13) & 0x3FFu);
  return nan ? hn : h;
}

__device__ __forceinline__ uint32_t cvt_f32_bf16(uint32_t x) {
  const uint32_t h = __builtin_bit_cast(uint16_t, (__bf16)__builtin_bit_cast(float, x));
  const bool nan = (x & 0x7FFFFFFFu) > 0x7F800000u;
  return nan ? ((x >> 16) | 0x40u) : h;
}

template <int CONV>
__device__ __forceinline__ uint64_t convert(uint64_t v) {
  if constexpr (CONV == CV_F64_F32) return cvt_f64_f32(v);
  else if constexpr (CONV == CV_F32_F64) return cvt_f32_f64((uint32_t)v);
  else if constexpr (CONV == CV_F32_F16) return cvt_f32_f16((uint32_t)v);
  else if constexpr (CONV == CV_F32_BF16) return cvt_f32_bf16((uint32_t)v);
  else if constexpr (CONV == CV_F64_F16) return narrow_rne<11, 52, 5, 10>(v);
  else if constexpr (CONV == CV_F64_BF16) return narrow_rne<11, 52, 8, 7>(v);
  else if constexpr (CONV == CV_F16_F32) return widen<5, 10, 8, 23>(v);
  else if constexpr (CONV == CV_BF16_F32) return widen<8, 7, 8, 23>(v);
  else if constexpr (CONV == CV_F16_F64) return widen<5, 10, 11, 52>(v);
  else return widen<8, 7, 11, 52>(v);
}

// Element planes on both sides, runs on the 16-byte grid: a lane converts the
// 16 / ES_DST values of one destination chunk from contiguous source
// elements (wide LDS reads) and stores the chunk whole.
template <int CONV>
__device__ __forceinline__ void store_conv_planar(const Side& s, const Side& d, uint64_t i0, uint32_t nt,
                                                  const uint8_t* lds, uint32_t f) {
  constexpr int ESS = ConvInfo<CONV>::ES_SRC, ESD = ConvInfo<CONV>::ES_DST;
  constexpr int V = 16 / ESD;         // values per destination chunk
  constexpr int NB = V * ESS;         // source bytes per chunk: 4 .. 64
  const uint32_t chunks = (nt + V - 1u) / V;
  const uint64_t start = seg_start<LY_PLANAR>(d, f, i0);
  const auto rs = make_rsrc((const uint8_t*)seg_blob<LY_PLANAR>(d, f) + start, d.blob_size - start);
  const uint8_t* plane = lds + f * s.lds_stride;
  for (uint32_t c = threadIdx.x; c < chunks; c += blockDim.x) {
    const uint32_t r = c * V;
    uint32_t raw[NB / 4];
    const uint8_t* p = plane + r * ESS;
    if constexpr (NB >= 16) {
#pragma unroll
      for (int q = 0; q < NB / 16; ++q) {
        const u32x4 x = *(const u32x4*)(p + 16 * q);
        raw[4 * q] = x.x;
        raw[4 * q + 1] = x.y;
        raw[4 * q + 2] = x.z;
        raw[4 * q + 3] = x.w;
      }
    } else if constexpr (NB == 8) {
      const u32x2 x = *(const u32x2*)p;
      raw[0] = x.x;
      raw[1] = x.y;
    } else {
      raw[0] = *(const uint32_t*)p;
    }
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int k = 0; k < V; ++k) {
      uint64_t e;
      if constexpr (ESS == 8) e = (uint64_t)raw[2 * k] | ((uint64_t)raw[2 * k + 1] << 32);
      else if constexpr (ESS == 4) e = raw[k];
      else e = (raw[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
      put_unit<ESD>(w, k, convert<CONV>(e));
    }
    const uint32_t valid = nt - r >= (uint32_t)V ? (1u << V) - 1u : (1u << (nt - r)) - 1u;
    store_chunk<ESD>(rs, 16u * c, w, valid, (1u << V) - 1u);
  }
}

// Narrowing f32 -> f16 / bf16 on element planes: a lane converts the four
// values of one 16-byte source chunk (consecutive lanes read consecutive
// chunks: no LDS bank conflicts) and stores their 8 bytes whole.  (f64
// sources keep store_conv_planar and 32 KiB tiles: with this form and
// 16 KiB tiles f64 -> f32 measured 11 % slower.)
template <int CONV>
__device__ __forceinline__ void store_conv_planar_narrow(const Side& s, const Side& d, uint64_t i0, uint32_t nt,
                                                         const uint8_t* lds, uint32_t f) {
  constexpr int ESS = ConvInfo<CONV>::ES_SRC, ESD = ConvInfo<CONV>::ES_DST;
  constexpr int V = 16 / ESS;      // values per source chunk (4 or 2)
  constexpr int OB = V * ESD;      // destination bytes per chunk (8 or 4)
  const uint32_t chunks = (nt + V - 1u) / V;
  const uint64_t start = seg_start<LY_PLANAR>(d, f, i0);
  const auto rs = make_rsrc((const uint8_t*)seg_blob<LY_PLANAR>(d, f) + start, d.blob_size - start);
  const uint8_t* plane = lds + f * s.lds_stride;
  for (uint32_t c = threadIdx.x; c < chunks; c += blockDim.x) {
    const uint32_t r = c * V;
    const u32x4 x = *(const u32x4*)(plane + 16u * c);
    uint32_t w[2] = {0u, 0u};
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const uint64_t e = ESS == 8 ? ((uint64_t)x[2 * k] | ((uint64_t)x[2 * k + 1] << 32)) : (uint64_t)x[k];
      const uint64_t v = convert<CONV>(e);
      const uint32_t bit = 8u * ESD * k;  // position of the value in the chunk
      w[bit >> 5] |= (uint32_t)v << (bit & 31u);
    }
    const uint32_t off = (uint32_t)OB * c;
    if (r + V <= nt) {
      if constexpr (OB == 8) __builtin_amdgcn_raw_buffer_store_b64(u32x2{w[0], w[1]}, rs, off, 0, kStoreNT);
      else __builtin_amdgcn_raw_buffer_store_b32(w[0], rs, off, 0, kStoreNT);
    } else {
      for (uint32_t k = 0; r + k < nt; ++k) {
        const uint32_t bit = 8u * ESD * k;
        if constexpr (ESD == 2)
          __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(w[bit >> 5] >> (bit & 31u)), rs, off + ESD * k, 0, 0);
        else
          __builtin_amdgcn_raw_buffer_store_b32(w[bit >> 5], rs, off + ESD * k, 0, 0);
      }
    }
  }
}

template <int CONV, int U, int DL, int SL>
__device__ __forceinline__ void store_conv(const Side& s, const Side& d, uint64_t i0, uint32_t nt,
                                           const uint8_t* lds) {
  if constexpr (DL == LY_PLANAR && SL == LY_PLANAR && U == ConvInfo<CONV>::ES_DST) {
    constexpr uint32_t ESS = ConvInfo<CONV>::ES_SRC, ESD = ConvInfo<CONV>::ES_DST;
    if (s.cs == ESS && (s.mb || ((s.n * ESS) & 15u) == 0u) && (d.mb || ((d.n * ESD) & 15u) == 0u)) {
      for (uint32_t f = 0; f < d.ncols; ++f) {
        if constexpr (ESS == 4 && ESD == 2) store_conv_planar_narrow<CONV>(s, d, i0, nt, lds, f);
        else store_conv_planar<CONV>(s, d, i0, nt, lds, f);
      }
      return;
    }
  }
  constexpr int NU = 16 / U;
  constexpr uint32_t FULL = (1u << NU) - 1u;
  constexpr int ESS = ConvInfo<CONV>::ES_SRC, ESD = ConvInfo<CONV>::ES_DST;
  constexpr int LOG_ESD = ESD == 8 ? 3 : ESD == 4 ? 2 : 1;
  for_dst_chunks<DL>(d, i0, nt, [&](__amdgpu_buffer_rsrc_t rs, uint32_t seg, uint32_t off, int x0, uint32_t len) {
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    uint32_t valid = 0;
#pragma unroll
    for (int t = 0; t < NU; ++t) {
      const int x = x0 + t * U;
      bool ok = x >= 0 && x < (int)len;
      uint32_t r, b;
      dst_inv<DL>(d, seg, ok ? (uint32_t)x : 0u, r, b);
      ok = ok && r < nt;
      if (ok) {
        const uint64_t v = convert<CONV>(fetch_elem<ESS, SL>(s, lds, r, b >> LOG_ESD));
        const uint32_t k = b & (ESD - 1);
        put_unit<U>(w, t, U == ESD ? v : ((v >> (8u * k)) & ((1ull << (8 * U)) - 1ull)));
      }
      valid |= (uint32_t)ok << t;
    }
    store_chunk<U>(rs, off, w, valid, FULL);
  });
}

// ---------------------------------------------------------------------------
// Phase B, pack into bit streams (Sec. 3 bit-packed SoA).  Every value of the
// tile is encoded exactly once.  A lane takes four consecutive values of an
// element plane (one 16-byte LDS read) and writes their codes into an LDS
// image of the tile's stream words: with B = 8, 16 or 32 the four codes fill
// whole words of their own, which are stored plainly; otherwise the codes
// (as one group for B <= 8, two pairs for B <= 16, singly above) are ORed in
// with LDS atomics, since a word's bits may come from two lanes.  The image
// starts zeroed, so the bits past the last value stay zero, and goes out with
// 16-byte stores: a wave writes 1 KiB contiguous per store.
// ---------------------------------------------------------------------------

// Float formats that get a compile-time encoder (any other goes through the
// run-time one).
enum PackFmt : uint32_t { PF_RUNTIME = 0, PF_E8M7 = 1, PF_E5M10 = 2, PF_E8M15 = 3 };

template <int FMT> struct PackFmtInfo { static constexpr uint32_t E = 0, M = 0; };
template <> struct PackFmtInfo<PF_E8M7> { static constexpr uint32_t E = 8, M = 7; };
template <> struct PackFmtInfo<PF_E5M10> { static constexpr uint32_t E = 5, M = 10; };
template <> struct PackFmtInfo<PF_E8M15> { static constexpr uint32_t E = 8, M = 15; };

// Truncating f32 encoder for a format fixed at compile time.  With E = 8 the
// target has the source's exponent range, so normals, subnormals and Inf
// keep their exponent field and lose their low mantissa bits: one shift, and
// a NaN keeps its all-ones exponent and gets its quiet bit.  Other formats
// constant-fold the run-time encoder.
template <uint32_t E, uint32_t M>
__device__ __forceinline__ uint32_t enc_f32_fixed(uint32_t x) {
  if constexpr (E == 5 && M == 10) {
    // [sign|5|10] is the binary16 layout: the hardware conversion with
    // rounding toward zero (v_cvt_pkrtz_f16_f32) truncates the mantissa and
    // keeps gradual underflow (the kernel's FP mode keeps denormals).  It
    // saturates at the largest finite code, but values with an exponent above
    // the bias (|x| >= 2^16) must give Inf; a NaN takes the NaN rule.
    const uint32_t ax = x & 0x7FFFFFFFu;
    const auto h2 = __builtin_amdgcn_cvt_pkrtz(__builtin_bit_cast(float, x), 0.0f);
    uint32_t c = __builtin_bit_cast(uint16_t, h2[0]);
    const uint32_t sgn = (x >> 16) & 0x8000u;
    c = ax >= 0x47800000u ? (sgn | 0x7C00u) : c;
    c = ax > 0x7F800000u ? (sgn | 0x7E00u | ((ax >> 13) & 0x3FFu)) : c;
    return c;
  } else if constexpr (E == 8) {
    const uint32_t ax = x & 0x7FFFFFFFu;
    uint32_t c = ax >> (23u - M);
    if constexpr (M > 0) c |= ax > 0x7F800000u ? (1u << (M - 1u)) : 0u;
    return c | ((x >> 31) << (E + M));
  } else {
    return enc_f32(x, E, M);
  }
}

template <int CODEC, int FMT>
__device__ __forceinline__ uint32_t encode_fmt(uint64_t v, const Side& d) {
  if constexpr (CODEC == CD_F32 && FMT != PF_RUNTIME)
    return enc_f32_fixed<PackFmtInfo<FMT>::E, PackFmtInfo<FMT>::M>((uint32_t)v);
  else
    return encode<CODEC>(v, d);
}

__device__ __forceinline__ void pack_clear_words(uint32_t* words, uint32_t nwords) {
  for (uint32_t k = threadIdx.x * 4u; k < nwords; k += blockDim.x * 4u) *(u32x4*)(words + k) = u32x4{0u, 0u, 0u, 0u};
}

// ORs the W-bit group `code` into the word image at stream bit `bit` (it
// spans at most two words).
__device__ __forceinline__ void or_bits(uint32_t* wf, uint32_t bit, uint32_t code, uint32_t W) {
  const uint32_t w = bit >> 5, sh = bit & 31u;
  __hip_atomic_fetch_or(wf + w, code << sh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  if (sh + W > 32u)
    __hip_atomic_fetch_or(wf + w + 1u, code >> (32u - sh), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The NWQ = B / 8 stream words that four consecutive B-bit codes fill
// exactly (B = 8, 16, 24, 32), in stream order.
template <int NWQ>
__device__ __forceinline__ void pack_quad_words(const uint32_t (&c)[4], uint32_t (&w)[4]) {
  if constexpr (NWQ == 1) {
    w[0] = c[0] | (c[1] << 8) | (c[2] << 16) | (c[3] << 24);
  } else if constexpr (NWQ == 2) {
    w[0] = c[0] | (c[1] << 16);
    w[1] = c[2] | (c[3] << 16);
  } else if constexpr (NWQ == 3) {
    w[0] = c[0] | (c[1] << 24);
    w[1] = (c[1] >> 8) | (c[2] << 16);
    w[2] = (c[2] >> 16) | (c[3] << 8);
  } else {
    w[0] = c[0]; w[1] = c[1]; w[2] = c[2]; w[3] = c[3];
  }
}

// Codes of a plane of 4-byte values straight from registers to the stream
// (B = 8 * NWQ): a lane encodes four consecutive values from one 16-byte LDS
// read and stores their NWQ whole words, so a wave writes 64 * NWQ * 4
// contiguous bytes per store.  Full quads need no checks; the tile's last,
// partial quad is written by one lane, word by word up to the stream's end.
template <int NWQ, int CODEC, int FMT>
__device__ __forceinline__ void pack_direct(const uint8_t* plane, uint32_t nt, uint32_t nw,
                                            __amdgpu_buffer_rsrc_t rs, const Side& d) {
  const uint32_t full = nt >> 2;
#pragma unroll 2
  for (uint32_t q = threadIdx.x; q < full; q += blockDim.x) {
    const u32x4 v = *(const u32x4*)(plane + 16u * q);
    uint32_t c[4], w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = encode_fmt<CODEC, FMT>(v[k], d);
    pack_quad_words<NWQ>(c, w);
    const uint32_t off = 4u * NWQ * q;  // the quad's first word
    if constexpr (NWQ == 1) __builtin_amdgcn_raw_buffer_store_b32(w[0], rs, off, 0, kStoreNT);
    else if constexpr (NWQ == 2) __builtin_amdgcn_raw_buffer_store_b64(u32x2{w[0], w[1]}, rs, off, 0, kStoreNT);
    else if constexpr (NWQ == 3) __builtin_amdgcn_raw_buffer_store_b96(u32x3{w[0], w[1], w[2]}, rs, off, 0, kStoreNT);
    else __builtin_amdgcn_raw_buffer_store_b128(u32x4{w[0], w[1], w[2], w[3]}, rs, off, 0, kStoreNT);
  }
  if ((nt & 3u) && threadIdx.x == 0) {
    const u32x4 v = *(const u32x4*)(plane + 16u * full);
    uint32_t c[4], w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = 4u * full + k < nt ? encode_fmt<CODEC, FMT>(v[k], d) : 0u;
    pack_quad_words<NWQ>(c, w);
    for (uint32_t k = 0; k < (uint32_t)NWQ && NWQ * full + k < nw; ++k)
      __builtin_amdgcn_raw_buffer_store_b32(w[k], rs, 4u * (NWQ * full + k), 0, 0);
  }
}

// Codes of a plane of 4-byte values into the tile's stream-word image, four
// consecutive values per lane.  CLS 0: B = 8, 16 or 32 (whole words, plain
// LDS stores); CLS 1: B < 8 (the four codes as one group); CLS 2: B < 16 (two
// pairs); CLS 3: B < 32 (one by one).  Groups that may share a word with
// another lane's are ORed in with LDS atomics (a group spans at most two
// words).  Values past the tile give code 0.  (Assembling whole words in
// registers with one ds_bpermute carry per lane, so that every word has one
// plain writer, measured 7 % slower than the atomics.)
template <int CLS, int CODEC, int FMT>
__device__ __forceinline__ void pack_image(const uint8_t* plane, uint32_t nt, uint32_t B, uint32_t* wf,
                                           const Side& d) {
  const uint32_t quads = (nt + 3u) >> 2;
  for (uint32_t q = threadIdx.x; q < quads; q += blockDim.x) {
    const u32x4 v = *(const u32x4*)(plane + 16u * q);
    const uint32_t r = 4u * q;
    uint32_t c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = encode_fmt<CODEC, FMT>(v[k], d);
    if (r + 4u > nt) {
#pragma unroll
      for (int k = 1; k < 4; ++k) c[k] = r + k < nt ? c[k] : 0u;
    }
    if constexpr (CLS == 0) {
      if (B == 8u) wf[q] = c[0] | (c[1] << 8) | (c[2] << 16) | (c[3] << 24);
      else if (B == 16u) *(u32x2*)(wf + 2u * q) = u32x2{c[0] | (c[1] << 16), c[2] | (c[3] << 16)};
      else *(u32x4*)(wf + 4u * q) = u32x4{c[0], c[1], c[2], c[3]};
    } else if constexpr (CLS == 1) {
      or_bits(wf, r * B, c[0] | (c[1] << B) | (c[2] << (2u * B)) | (c[3] << (3u * B)), 4u * B);
    } else if constexpr (CLS == 2) {
      or_bits(wf, r * B, c[0] | (c[1] << B), 2u * B);
      or_bits(wf, r * B + 2u * B, c[2] | (c[3] << B), 2u * B);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) or_bits(wf, r * B + k * B, c[k], B);
    }
  }
}

template <int CODEC, int FMT, int SL>
__device__ __forceinline__ void store_pack(const Side& s, const Side& d, uint64_t i0, uint32_t nt,
                                           const uint8_t* lds, uint32_t* words, uint32_t wstride) {
  constexpr int ES = CodecInfo<CODEC>::ES;
  const uint32_t B = d.bits;
  const uint32_t F = d.ncols;
  const uint32_t nw = (nt * B + 31u) >> 5;  // stream words of this tile
  // element planes of 4-byte values on the 16-byte grid (not Bytesplit byte
  // planes) are read four values at a time; with B a multiple of 8 their
  // codes bypass the word image
  auto quad_plane = [&](uint32_t f) {
    return SL == LY_PLANAR && ES == 4 && s.cs == 4u && (planar_phase(s, f) & 15u) == 0u;
  };
  auto direct = [&](uint32_t f) { return quad_plane(f) && (B & 7u) == 0u; };
  bool imaged = false;  // some field went through the word image
  for (uint32_t f = 0; f < F; ++f) {
    uint32_t* wf = words + f * wstride;
    if constexpr (SL == LY_PLANAR && ES == 4) {
      if (direct(f)) {
        // B = 8, 16, 24, 32: the four codes of a quad are B / 8 whole words
        // starting on a word boundary, so they go from registers straight to
        // the stream (a wave writes 64 * B / 2 contiguous bytes per store, whole
        // 128-byte lines); no word image, no barrier.  Only the tile's last
        // quad may hold words past the stream, which are dropped word by word.
        const uint8_t* plane = lds + f * s.lds_stride;
        const uint64_t start = seg_start<LY_STREAM>(d, f, i0);
        const auto rs = make_rsrc((const uint8_t*)seg_blob<LY_STREAM>(d, f) + start, d.blob_size - start);
        constexpr uint32_t FB = 1u + PackFmtInfo<FMT>::E + PackFmtInfo<FMT>::M;  // a fixed format's code bits
        if constexpr (FMT != PF_RUNTIME && FB % 8u == 0u) {
          pack_direct<FB / 8u, CODEC, FMT>(plane, nt, nw, rs, d);
        } else {
          switch (B) {  // block-uniform, once per field
            case 8u: pack_direct<1, CODEC, FMT>(plane, nt, nw, rs, d); break;
            case 16u: pack_direct<2, CODEC, FMT>(plane, nt, nw, rs, d); break;
            case 24u: pack_direct<3, CODEC, FMT>(plane, nt, nw, rs, d); break;
            default: pack_direct<4, CODEC, FMT>(plane, nt, nw, rs, d); break;
          }
        }
        continue;
      }
      if (quad_plane(f)) {
        imaged = true;
        const uint8_t* plane = lds + f * s.lds_stride;
        // the code-width class is block-uniform: one loop per class, no
        // width branches inside
        if (B == 8u || B == 16u || B == 32u) pack_image<0, CODEC, FMT>(plane, nt, B, wf, d);
        else if (B < 8u) pack_image<1, CODEC, FMT>(plane, nt, B, wf, d);
        else if (B < 16u) pack_image<2, CODEC, FMT>(plane, nt, B, wf, d);
        else pack_image<3, CODEC, FMT>(plane, nt, B, wf, d);
        continue;
      }
    }
    imaged = true;
    for (uint32_t r = threadIdx.x; r < nt; r += blockDim.x)
      or_bits(wf, r * B, encode_fmt<CODEC, FMT>(fetch_elem<ES, SL>(s, lds, r, f), d), B);
  }
  if (!imaged) return;  // block-uniform: every field went out directly
  __syncthreads();
  const uint32_t nch = (nw + 3u) >> 2;
  for (uint32_t f = 0; f < F; ++f) {
    if (direct(f)) continue;
    // tiles are multiples of 128 records, so every tile's stream starts 16-byte aligned
    const uint64_t start = seg_start<LY_STREAM>(d, f, i0);
    const auto rs = make_rsrc((const uint8_t*)seg_blob<LY_STREAM>(d, f) + start, d.blob_size - start);
    const uint32_t* wf = words + f * wstride;
    for (uint32_t c = threadIdx.x; c < nch; c += blockDim.x) {
      const u32x4 v = *(const u32x4*)(wf + 4u * c);
      if (4u * c + 4u <= nw) {
        __builtin_amdgcn_raw_buffer_store_b128(v, rs, 16u * c, 0, kStoreNT);
      } else {
        __builtin_amdgcn_raw_buffer_store_b32(v[0], rs, 16u * c, 0, 0);
        if (4u * c + 1u < nw) __builtin_amdgcn_raw_buffer_store_b32(v[1], rs, 16u * c + 4u, 0, 0);
        if (4u * c + 2u < nw) __builtin_amdgcn_raw_buffer_store_b32(v[2], rs, 16u * c + 8u, 0, 0);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Phase B, unpack from bit streams into a physical layout
// ---------------------------------------------------------------------------

// Unpack into element planes of 4-byte values: a lane decodes four
// consecutive values of one field straight from the stream words and stores
// them as one 16-byte chunk (a wave writes 1 KiB contiguous).  Used when the
// plane's tile run starts on the 16-byte grid; the generic gather below
// handles every other destination.
template <int CODEC>
__device__ __forceinline__ void store_unpack_planar4(const Side& s, const Side& d, uint64_t i0, uint32_t nt,
                                                     const uint8_t* lds, uint32_t f) {
  const uint32_t B = s.bits;
  const uint32_t quads = (nt + 3u) >> 2;
  const uint64_t start = seg_start<LY_PLANAR>(d, f, i0);
  const auto rs = make_rsrc((const uint8_t*)seg_blob<LY_PLANAR>(d, f) + start, d.blob_size - start);
  const uint8_t* plane = lds + f * s.lds_stride;
  for (uint32_t q = threadIdx.x; q < quads; q += blockDim.x) {
    const uint32_t r = 4u * q;
    uint32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (uint32_t)decode<CODEC>(stream_code(plane, r + k, B), s);
    if (r + 4u <= nt) {
      __builtin_amdgcn_raw_buffer_store_b128(u32x4{v[0], v[1], v[2], v[3]}, rs, 16u * q, 0, kStoreNT);
    } else {
      for (uint32_t k = 0; r + k < nt; ++k) __builtin_amdgcn_raw_buffer_store_b32(v[k], rs, 16u * q + 4u * k, 0, 0);
    }
  }
}

template <int CODEC, int U, int DL>
__device__ __forceinline__ void store_unpack(const Side& s, const Side& d, uint64_t i0, uint32_t nt,
                                             const uint8_t* lds) {
  if constexpr (DL == LY_PLANAR && U == 4 && CodecInfo<CODEC>::ES == 4) {
    // every field's run must start on the 16-byte grid (single-blob planes
    // start at f * 4n)
    if (d.mb || (d.n & 3u) == 0u) {
      for (uint32_t f = 0; f < d.ncols; ++f) store_unpack_planar4<CODEC>(s, d, i0, nt, lds, f);
      return;
    }
  }
  constexpr int NU = 16 / U;
  constexpr uint32_t FULL = (1u << NU) - 1u;
  constexpr int ES = CodecInfo<CODEC>::ES;
  constexpr int LOG_ES = ES == 8 ? 3 : ES == 4 ? 2 : ES == 2 ? 1 : 0;
  const uint32_t B = s.bits;
  for_dst_chunks<DL>(d, i0, nt, [&](__amdgpu_buffer_rsrc_t rs, uint32_t seg, uint32_t off, int x0, uint32_t len) {
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    uint32_t valid = 0;
#pragma unroll
    for (int t = 0; t < NU; ++t) {
      const int x = x0 + t * U;
      bool ok = x >= 0 && x < (int)len;
      uint32_t r, b;
      dst_inv<DL>(d, seg, ok ? (uint32_t)x : 0u, r, b);
      ok = ok && r < nt;
      if (ok) {
        const uint32_t f = b >> LOG_ES;
        const uint64_t v = decode<CODEC>(stream_code(lds + f * s.lds_stride, r, B), s);
        const uint32_t k = b & (ES - 1);
        put_unit<U>(w, t, U == ES ? v : ((v >> (8u * k)) & ((1ull << (8 * U)) - 1ull)));
      }
      valid |= (uint32_t)ok << t;
    }
    store_chunk<U>(rs, off, w, valid, FULL);
  });
}

}  // namespace lm
