// Pack of planes of 32-bit integers into bit streams (Sec. 3 BitpackIntSoA:
// the low B bits of every value), the planar path of pack for the code widths
// it serves best (B <= 27, not a multiple of 8).
//
// One workgroup takes a tile of four chunks of 2048 values (8 KiB each), one
// per wave; a wave works on its chunk alone, with no workgroup barrier:
//   1. eight direct buffer -> LDS loads (1 KiB per wave instruction, the
//      streaming cache policy) bring the chunk into the wave's LDS region;
//      load k goes to byte 1040 k, so that the transposed reads below meet at
//      most 4-way bank conflicts;
//   2. lane l reads values 32 l .. 32 l + 31 from the region;
//   3. 32 codes of B bits are exactly B stream words: the lane assembles them
//      in registers with compile-time shifts (no atomics, no word image to
//      clear) and writes them back to the region;
//   4. the chunk's 64 B words leave as 16-byte non-temporal stores, each wave
//      instruction writing whole 128-byte lines.
// Buffer range checks work per dword: values past the plane's end load as 0
// (whose code is 0) and words past the stream's end are not stored, so the
// last chunk of a plane takes no other path.  (A persistent form, each wave
// streaming its chunks through registers two ahead, measured 7 % slower.)
#include "kernels.hpp"

namespace lm {

namespace {

constexpr uint32_t kWaves = kThreads / 64u;
constexpr uint32_t kChunk = 2048;          // values per wave and tile: 32 per lane
constexpr uint32_t kLoadStride = 1040;     // LDS bytes between a chunk's eight 1 KiB loads
constexpr uint32_t kRegionBytes = 8320;    // 8 * kLoadStride

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

template <uint32_t B>
__global__ __launch_bounds__(kThreads) void k_pack_planar(PlanarPackArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t region[kWaves][kRegionBytes];
  uint8_t* r8 = region[wave_id()];
  uint32_t* r = (uint32_t*)r8;
  const uint32_t lane = lane_id();
  const uint64_t cpf = (a.n + kChunk - 1u) / kChunk;  // chunks per field
  const uint64_t total = cpf * a.nf;
  const uint64_t nw = (a.n * B + 31u) >> 5;          // stream words per field
  for (uint64_t t = blockIdx.x; t * kWaves < total; t += gridDim.x) {
    // this wave's chunk: field f, chunk c of its plane (past the last one:
    // empty ranges, the loads return 0 and nothing is stored)
    const uint64_t g = t * kWaves + wave_id();
    const bool live = g < total;
    const uint32_t f = live ? (uint32_t)(g / cpf) : 0u;
    const uint64_t c = live ? g - (uint64_t)f * cpf : 0u;
    const uint64_t v0 = c * kChunk;
    const auto rs = make_rsrc(a.src[f] + 4u * v0, live ? 4u * (a.n - v0) : 0u);
#pragma unroll
    for (uint32_t k = 0; k < 8u; ++k)  // quads 64 k + lane of the chunk at byte kLoadStride k + 16 lane
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void*)(r8 + kLoadStride * k), 16, 16u * (lane + 64u * k), 0, 0,
                                               kLoadStream);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    wave_lds_sync();
    uint32_t cv[32];
#pragma unroll
    for (uint32_t k = 0; k < 8u; ++k) {  // quad 8 lane + k: load lane >> 3, its lane 8 (lane & 7) + k
      const u32x4 v = *(const u32x4*)(r8 + kLoadStride * (lane >> 3) + 128u * (lane & 7u) + 16u * k);
#pragma unroll
      for (uint32_t e = 0; e < 4u; ++e) cv[4u * k + e] = code_of<B>(v[e]);
    }
    uint32_t w[B];
    words_of_32<B>(cv, w);
    wave_lds_sync();  // every lane has its values before the words overwrite them
    put_words<B>(r + B * lane, w);
    wave_lds_sync();
    // the chunk's 64 B words: 16 B quads, 16 B / 64 per lane rounded up; the
    // store range ends at the chunk's last word (or the stream's), so the
    // lanes of the last pass past it store nothing
    constexpr uint32_t kQuads = 16u * B, kPer = (kQuads + 63u) / 64u;
    const uint64_t w0 = c * 64u * B;  // the chunk's first stream word
    const uint64_t left = live ? 4u * (nw - w0) : 0u;
    const auto rd = make_rsrc(a.dst[f] + 4u * w0, left < 16u * kQuads ? left : 16u * kQuads);
    u32x4 o[kPer];
#pragma unroll
    for (uint32_t m = 0; m < kPer; ++m) o[m] = *(const u32x4*)(r + 4u * (lane + 64u * m));
#pragma unroll
    for (uint32_t m = 0; m < kPer; ++m) __builtin_amdgcn_raw_buffer_store_b128(o[m], rd, 16u * (lane + 64u * m), 0, kStoreNT);
    wave_lds_sync();  // the words are read before a next tile's loads overwrite them
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
