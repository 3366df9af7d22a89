// Pack of planes of 32-bit integers into bit streams (Sec. 3 BitpackIntSoA:
// the low B bits of every value), the planar path of pack for the code widths
// it serves best (B < 24, not a multiple of 8).
//
// Every wave works alone on chunks of 2048 values of one field, with no
// workgroup barrier:
//   1. eight coalesced 16-byte loads per lane bring the chunk (8 KiB) into
//      registers, issued two chunks ahead so that a wave's next two chunks are
//      in flight while it packs the current one;
//   2. the chunk goes through the wave's LDS region once, transposed, so that
//      lane l holds values 32 l .. 32 l + 31 (the region has 16 bytes of pad
//      after every 128, which keeps the transposed 16-byte reads free of bank
//      conflicts);
//   3. 32 codes of B bits are exactly B stream words: the lane assembles them
//      in registers with compile-time shifts (no atomics, no word image to
//      clear) and writes them to the region;
//   4. the chunk's 64 B words leave as 16-byte non-temporal stores, each wave
//      instruction writing whole 128-byte lines.
// Buffer range checks work per dword: values past the plane's end load as 0
// (whose code is 0) and words past the stream's end are not stored, so the
// last chunk of a plane takes no other path.  Loads stream (read once, no L1).
#include "kernels.hpp"

namespace lm {

namespace {

constexpr uint32_t kWaves = kThreads / 64u;
constexpr uint32_t kChunk = 2048;        // values per wave and chunk: 32 per lane
constexpr uint32_t kRegionWords = 2304;  // 8 KiB of values plus 16 bytes after every 128

// Orders the wave's LDS accesses around an exchange between its lanes (the
// LDS executes one wave's instructions in order; this keeps the compiler
// from moving accesses across the exchange).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <uint32_t B>
__device__ __forceinline__ uint32_t code_of(uint32_t v) {
  return B >= 32u ? v : (v & ((1u << B) - 1u));
}

// The B stream words that 32 consecutive B-bit codes fill exactly.
template <uint32_t B>
__device__ __forceinline__ void words_of_32(const uint32_t (&c)[32], uint32_t (&w)[B]) {
#pragma unroll
  for (uint32_t j = 0; j < B; ++j) w[j] = 0u;
#pragma unroll
  for (uint32_t k = 0; k < 32u; ++k) {
    const uint32_t bit = k * B, j = bit >> 5, sh = bit & 31u;
    w[j] |= c[k] << sh;
    if (sh + B > 32u) w[j + 1u] |= c[k] >> (32u - sh);
  }
}

// A lane's B words at word B * lane of the region, in the widest stores
// their alignment allows (B odd: 32-bit stores, lanes B words apart, which
// are conflict-free for odd B).
template <uint32_t B>
__device__ __forceinline__ void put_words(uint32_t* r, const uint32_t (&w)[B]) {
  if constexpr (B % 4u == 0u) {
#pragma unroll
    for (uint32_t j = 0; j < B; j += 4u) *(u32x4*)(r + j) = u32x4{w[j], w[j + 1u], w[j + 2u], w[j + 3u]};
  } else if constexpr (B % 2u == 0u) {
#pragma unroll
    for (uint32_t j = 0; j < B; j += 2u) *(u32x2*)(r + j) = u32x2{w[j], w[j + 1u]};
  } else {
#pragma unroll
    for (uint32_t j = 0; j < B; ++j) r[j] = w[j];
  }
}

// A chunk: field f, chunk c of that field's plane (wave-uniform).
struct ChunkPos {
  uint32_t f;
  uint64_t c;
};

// The chunk W chunks after p, fields in order (no division: W / cpf rounds at most).
__device__ __forceinline__ ChunkPos advance(ChunkPos p, uint64_t W, uint64_t cpf) {
  p.c += W;
  while (p.c >= cpf) {
    p.c -= cpf;
    ++p.f;
  }
  return p;
}

// The chunk's values into registers: lane l gets its 16-byte quads l, l + 64,
// ..., l + 448.  Past the last field the loads still issue, through an empty
// range (they return 0): every path through the loop then has the same
// memory operations in flight, so the waits before each chunk count only
// that chunk's own loads.
__device__ __forceinline__ void load_chunk(const PlanarPackArgs& a, ChunkPos p, uint32_t lane, u32x4 (&q)[8]) {
  const bool live = p.f < a.nf;
  const uint64_t v0 = live ? p.c * kChunk : 0u;
  const auto rs = make_rsrc(a.src[live ? p.f : 0u] + 4u * v0, live ? 4u * (a.n - v0) : 0u);
#pragma unroll
  for (uint32_t k = 0; k < 8u; ++k) q[k] = __builtin_amdgcn_raw_buffer_load_b128(rs, 16u * (lane + 64u * k), 0, kLoadStream);
}

// One chunk: its values (q, already loaded) through the region into codes and
// words, and out to the stream; q is reloaded with chunk `ahead` meanwhile.
template <uint32_t B>
__device__ __forceinline__ void pack_chunk(const PlanarPackArgs& a, uint32_t* r, uint32_t lane, uint64_t nw,
                                           ChunkPos p, ChunkPos ahead, u32x4 (&q)[8]) {
#pragma unroll
  for (uint32_t k = 0; k < 8u; ++k) {
    const uint32_t j = lane + 64u * k;  // the chunk's quad j, at word 4 j plus its pad
    *(u32x4*)(r + 4u * j + 4u * (j >> 3)) = q[k];
  }
  load_chunk(a, ahead, lane, q);  // in flight while this chunk is packed
  wave_lds_sync();
  uint32_t c[32];
#pragma unroll
  for (uint32_t k = 0; k < 8u; ++k) {
    const u32x4 v = *(const u32x4*)(r + 36u * lane + 4u * k);  // quad 8 lane + k
#pragma unroll
    for (uint32_t e = 0; e < 4u; ++e) c[4u * k + e] = code_of<B>(v[e]);
  }
  uint32_t w[B];
  words_of_32<B>(c, w);
  wave_lds_sync();  // every lane has its values before the words overwrite them
  put_words<B>(r + B * lane, w);
  wave_lds_sync();
  // the chunk's 64 B words: 16 B quads, 16 B / 64 per lane rounded up; the
  // store range ends at the chunk's last word (or the stream's), so the
  // lanes of the last round past it store nothing
  // (a chunk past the last field stores nothing: an empty range)
  constexpr uint32_t kQuads = 16u * B, kPer = (kQuads + 63u) / 64u;
  const bool live = p.f < a.nf;
  const uint64_t w0 = live ? p.c * 64u * B : 0u;  // the chunk's first stream word
  const uint64_t left = live ? 4u * (nw - w0) : 0u;
  const auto rs = make_rsrc(a.dst[live ? p.f : 0u] + 4u * w0, left < 16u * kQuads ? left : 16u * kQuads);
  u32x4 o[kPer];
#pragma unroll
  for (uint32_t m = 0; m < kPer; ++m) o[m] = *(const u32x4*)(r + 4u * (lane + 64u * m));
#pragma unroll
  for (uint32_t m = 0; m < kPer; ++m) __builtin_amdgcn_raw_buffer_store_b128(o[m], rs, 16u * (lane + 64u * m), 0, kStoreNT);
  wave_lds_sync();  // the words are read before the next chunk's values overwrite them
}

template <uint32_t B>
__global__ __launch_bounds__(kThreads) void k_pack_planar(PlanarPackArgs a) {
  __shared__ __attribute__((aligned(16))) uint32_t region[kWaves][kRegionWords];
  uint32_t* r = region[wave_id()];
  const uint32_t lane = lane_id();
  const uint64_t cpf = (a.n + kChunk - 1u) / kChunk;  // chunks per field
  const uint64_t nw = (a.n * B + 31u) >> 5;          // stream words per field
  const uint64_t W = (uint64_t)gridDim.x * kWaves;
  // a wave's chunks are W apart; two are in flight ahead of the one it packs,
  // in two register sets used in turn.  The loop runs a fixed count of chunk
  // pairs with no other branch (a pair's second chunk may lie past the end),
  // so that every chunk waits only for its own loads.
  const uint64_t g0 = (uint64_t)blockIdx.x * kWaves + wave_id(), total = cpf * a.nf;
  if (g0 >= total) return;
  const uint64_t pairs = ((total - g0 + W - 1u) / W + 1u) / 2u;
  ChunkPos pa = advance(ChunkPos{0u, 0u}, g0, cpf);
  ChunkPos pb = advance(pa, W, cpf);
  u32x4 qa[8], qb[8];
  load_chunk(a, pa, lane, qa);
  __builtin_amdgcn_sched_barrier(0);  // qa's loads issue first, as in the loop
  load_chunk(a, pb, lane, qb);
  for (uint64_t it = 0; it < pairs; ++it) {
    const ChunkPos pc = advance(pb, W, cpf);
    pack_chunk<B>(a, r, lane, nw, pa, pc, qa);
    const ChunkPos pd = advance(pc, W, cpf);
    pack_chunk<B>(a, r, lane, nw, pb, pd, qb);
    pa = pc;
    pb = pd;
  }
}

template <uint32_t B>
hipError_t launch_one(const PlanarPackArgs& a, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL((k_pack_planar<B>), dim3(grid), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

template <uint32_t... Bs>
hipError_t launch_b(const PlanarPackArgs& a, uint32_t grid, hipStream_t st, std::integer_sequence<uint32_t, Bs...>) {
  hipError_t e = hipErrorInvalidValue;
  ((a.bits == Bs + 1u ? (void)(e = launch_one<Bs + 1u>(a, grid, st)) : (void)0), ...);
  return e;
}

}  // namespace

hipError_t launch_pack_planar(const PlanarPackArgs& a, uint32_t grid, hipStream_t st) {
  return launch_b(a, grid, st, std::make_integer_sequence<uint32_t, 32>{});
}

}  // namespace lm
