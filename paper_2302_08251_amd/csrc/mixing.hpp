// Per-leaf addressing of the mapping trees flattened by the host (MixSide):
// the device side of the per-leaf and value-level copies.
#pragma once
#include "kernels.hpp"

namespace lm {

// Where record i sits in a group: the byte offset of its block and its index
// inside the block (planar groups: the record index itself).
struct MixPos {
  uint64_t base;
  uint64_t lane;
};

__device__ __forceinline__ MixPos mix_pos(const MixGroup& g, uint64_t i) {
  if (g.L == 0) return {0, i};
  if (g.L == 1) return {i * g.block, 0};
  uint64_t q;
  if (g.log2L < 64) q = i >> g.log2L;
  else if (i <= 0xFFFFFFFFull) q = (uint32_t)i / g.L;
  else q = i / g.L;
  return {q * g.block, i - q * g.L};
}

__device__ __forceinline__ uint8_t* mix_at(const MixSide& s, const MixPos& p, uint32_t c, uint32_t size) {
  return const_cast<uint8_t*>(s.col[c]) + p.base + p.lane * size;
}

// Leaf f of record i, its bytes in memory order (little-endian value); 0 from a NULL part.
__device__ __forceinline__ uint64_t mix_load(const MixSide& s, uint64_t i, uint32_t f, uint32_t lsz) {
  const MixGroup& g = s.g[s.grp[f]];
  if (g.kind == MX_NULL) return 0;
  const uint32_t size = 1u << lsz, c = s.cidx[f];
  const MixPos p = mix_pos(g, i);
  uint64_t v = 0;
  if (g.kind == MX_BYTES) {  // Bytesplit: byte k of the leaf is byte column c + k
    for (uint32_t k = 0; k < size; ++k) v |= (uint64_t)*mix_at(s, p, c + k, 1) << (8 * k);
    return v;
  }
  const uint8_t* a = mix_at(s, p, c, size);
  if ((s.elem_ok >> f) & 1ull) {
    switch (lsz) {
      case 0: return *a;
      case 1: return *(const uint16_t*)a;
      case 2: return *(const uint32_t*)a;
      default: return *(const uint64_t*)a;
    }
  }
  for (uint32_t k = 0; k < size; ++k) v |= (uint64_t)a[k] << (8 * k);
  return v;
}

__device__ __forceinline__ void mix_store(const MixSide& s, uint64_t i, uint32_t f, uint32_t lsz, uint64_t v) {
  const MixGroup& g = s.g[s.grp[f]];
  if (g.kind == MX_NULL) return;
  const uint32_t size = 1u << lsz, c = s.cidx[f];
  const MixPos p = mix_pos(g, i);
  if (g.kind == MX_BYTES) {
    for (uint32_t k = 0; k < size; ++k) *mix_at(s, p, c + k, 1) = (uint8_t)(v >> (8 * k));
    return;
  }
  uint8_t* a = mix_at(s, p, c, size);
  if ((s.elem_ok >> f) & 1ull) {
    switch (lsz) {
      case 0: *a = (uint8_t)v; return;
      case 1: *(uint16_t*)a = (uint16_t)v; return;
      case 2: *(uint32_t*)a = (uint32_t)v; return;
      default: *(uint64_t*)a = v; return;
    }
  }
  for (uint32_t k = 0; k < size; ++k) a[k] = (uint8_t)(v >> (8 * k));
}

// The source's linear index of the destination's record i when the two are
// linearised in different orders (row-major: last extent fastest;
// column-major: first extent fastest).
__device__ __forceinline__ uint64_t mix_src_index(const Order& a, uint64_t i) {
  if (!a.reorder) return i;
  uint64_t digit[8];
  if (a.dst_col_major) {
    for (uint32_t d = 0; d < a.rank; ++d) {
      digit[d] = i % a.ext[d];
      i /= a.ext[d];
    }
  } else {
    for (uint32_t d = a.rank; d-- > 0;) {
      digit[d] = i % a.ext[d];
      i /= a.ext[d];
    }
  }
  uint64_t j = 0;
  if (a.src_col_major) {
    for (uint32_t d = a.rank; d-- > 0;) j = j * a.ext[d] + digit[d];
  } else {
    for (uint32_t d = 0; d < a.rank; ++d) j = j * a.ext[d] + digit[d];
  }
  return j;
}

}  // namespace lm
