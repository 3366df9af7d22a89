// All-pairs n-body consumer reading and writing particles through a mapping
// (LLAMA, arXiv 2302.08251, Sec. 5: the update loads every particle, lets it
// interact with all others and stores only the velocity; the move phase then
// advances positions).  Interaction: softened gravity with G = 1,
//   a_i = sum_j m_j (x_j - x_i) (|x_j - x_i|^2 + eps2)^(-3/2).
// Record: {pos.x, pos.y, pos.z, vel.x, vel.y, vel.z, mass}.
// Storage forms: F32 leaves in any physical mapping (Bytesplit included),
// ChangeType(F64 -> F32, physical), BitPackedFloatSoA with E <= 8, M <= 23
// (codes decode exactly to float32).  Compute and accumulation are FP32;
// only the energy check runs in FP64.
#include <mutex>

#include "host.hpp"
#include "static_view.hpp"
#include "tile_engine.hpp"

namespace lm {

constexpr uint32_t NB_T = 256;  // threads per workgroup, i-particles per block, j-tile size

// The j-tile cache of the update is itself a view in LDS (Sec. 2: static
// extents make the view a trivial value type that can live in shared memory;
// Sec. 3: Split and Null select the fields it keeps): 256 particles with
// fully static extents and a 16-bit index type, whose Split sends
// {pos.x, pos.y, pos.z, mass} (leaves 0, 1, 2, 6) to a 16-byte AoS record and
// the velocities to Null.  It stores nothing but those bytes, and every offset
// is a compile-time constant plus 16 * particle.
using JTileExt = sv::Extents<uint16_t, NB_T>;
using JTileMap = sv::Split<0x47ull, sv::AoS<JTileExt, 4, float>, sv::Null<JTileExt, 3, float>>;
using JTile = sv::View<JTileMap>;
static_assert(sizeof(JTile) == NB_T * 4 * sizeof(float), "the j-tile view holds exactly its mapped bytes");

// Byte offset of column `col` of record i within its blob (physical sides).
__device__ __forceinline__ uint32_t nb_off(const Side& s, uint32_t i, uint32_t col) {
  switch (s.layout) {
    case LY_AOS: return i * s.rec_bytes + col * s.cs;
    case LY_PLANAR: return (s.mb ? 0u : (uint32_t)s.n * s.cs * col) + i * s.cs;
    default: {
      const uint32_t blk = fdiv(i, s.div_L);
      return blk * s.lanes * s.rec_bytes + col * s.lanes * s.cs + (i - blk * s.lanes) * s.cs;
    }
  }
}

__device__ __forceinline__ const void* nb_blob(const Side& s, uint32_t col) {
  return (s.layout == LY_STREAM || (s.layout == LY_PLANAR && s.mb)) ? s.blob[col] : s.blob[0];
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t nb_rsrc(const Side& s, uint32_t col) {
  return make_rsrc(nb_blob(s, col), s.blob_size);
}

// float32 value of field f of particle i, decoded through the mapping
__device__ __forceinline__ float nb_load(const Side& s, uint32_t i, uint32_t f) {
  uint32_t bits;
  if (s.layout == LY_STREAM) {
    const auto rs = nb_rsrc(s, f);
    const uint32_t p = i * s.bits;
    const uint32_t lo = __builtin_amdgcn_raw_buffer_load_b32(rs, (p >> 5) * 4u, 0, 0);
    const uint32_t hi = __builtin_amdgcn_raw_buffer_load_b32(rs, (p >> 5) * 4u + 4u, 0, 0);
    uint32_t c = __builtin_amdgcn_alignbit(hi, lo, p & 31u);
    c = s.bits >= 32u ? c : (c & ((1u << s.bits) - 1u));
    bits = dec_f32(c, s.exp_bits, s.man_bits);
  } else if (s.cs == 4u) {
    bits = __builtin_amdgcn_raw_buffer_load_b32(nb_rsrc(s, f), nb_off(s, i, f), 0, 0);
  } else {  // Bytesplit: four byte columns
    bits = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k)
      bits |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(nb_rsrc(s, 4 * f + k), nb_off(s, i, 4 * f + k), 0, 0)
              << (8 * k);
  }
  return __builtin_bit_cast(float, bits);
}

// physical sides only
__device__ __forceinline__ void nb_store(const Side& s, uint32_t i, uint32_t f, float v) {
  const uint32_t bits = __builtin_bit_cast(uint32_t, v);
  if (s.cs == 4u) {
    __builtin_amdgcn_raw_buffer_store_b32(bits, nb_rsrc(s, f), nb_off(s, i, f), 0, 0);
  } else {
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k)
      __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(bits >> (8 * k)), nb_rsrc(s, 4 * f + k),
                                           nb_off(s, i, 4 * f + k), 0, 0);
  }
}

// ---------------------------------------------------------------------------
// Instrumentation of the consumer (Sec. 4): every load and store the kernels
// make through an instrumented particle view adds one to its counters.
// FieldAccessCount: counter 2f counts the loads of leaf f, 2f + 1 its
// stores.  Heatmap: one counter per G bytes of each data blob; an access adds
// one to every counter whose bytes it touches.  Counts are aggregated per
// wave (and per workgroup where the same counter repeats) before the global
// atomic add, so they are the per-access counts with far fewer atomics.
// ---------------------------------------------------------------------------

struct NbCount {
  uint64_t* fac;        // FieldAccessCount counters (14), or null
  uint64_t* heat[7];    // Heatmap: counter blob of the data blob holding leaf f, or null
  uint32_t heat_shift;  // log2 of the bytes per Heatmap counter
  uint32_t pad;
};

__device__ __forceinline__ uint64_t wave_ballot(bool b) { return __builtin_amdgcn_ballot_w64(b); }

// FieldAccessCount: adds the wave's sum of `v` (one lane's accesses) to
// counter k (lane 0 of the wave adds).
__device__ __forceinline__ void nb_fac_add(const NbCount& c, uint32_t k, uint32_t v) {
  if (!c.fac) return;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane_id() == 0 && v) atomicAdd((unsigned long long*)(c.fac + k), (unsigned long long)v);
}

// Heatmap: one access of the 4-byte element of leaf f at byte `off` of its
// blob, by the lanes with `valid`; lanes that hit the same counter add once.
__device__ __forceinline__ void nb_heat(const NbCount& c, uint32_t f, uint32_t off, bool valid) {
  uint64_t* ctr = c.heat[f];
  if (!ctr) return;
  const uint32_t sh = c.heat_shift;
  const uint32_t first = off >> sh, last = (off + 3u) >> sh;
  for (uint32_t k = 0; k <= (3u >> (sh < 2u ? sh : 2u)); ++k) {  // counters an element can touch
    const uint32_t q = first + k;
    bool act = valid && q <= last;
    uint64_t pending = wave_ballot(act);
    while (pending) {
      const uint32_t leader = (uint32_t)__builtin_ctzll(pending);
      const uint32_t lq = (uint32_t)__builtin_amdgcn_readlane((int)q, (int)leader);
      const uint64_t same = wave_ballot(act && q == lq);
      if (lane_id() == leader) atomicAdd((unsigned long long*)(ctr + lq), (unsigned long long)__builtin_popcountll(same));
      act = act && q != lq;
      pending &= ~same;
    }
  }
}

// one access (load: which = 0, store: 1) of leaf f of particle i by the
// lanes with `valid`
__device__ __forceinline__ void nb_count(const NbCount& c, const Side& s, uint32_t f, uint32_t which, uint32_t i,
                                         bool valid) {
  nb_fac_add(c, 2u * f + which, valid ? 1u : 0u);
  if (c.heat[f]) nb_heat(c, f, valid ? nb_off(s, i, f) : 0u, valid);
}

// ---------------------------------------------------------------------------
// Update: partial accelerations of i-block blockIdx.x over j-slice blockIdx.y
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(NB_T) void k_nb_update(const Side s, uint32_t n, float eps2, uint32_t per_slice,
                                                   float* __restrict__ part, const NbCount cnt) {
  __shared__ JTile tile;
  const uint32_t i = blockIdx.x * NB_T + threadIdx.x;
  const uint32_t j0 = blockIdx.y * per_slice;
  uint32_t j1 = j0 + per_slice;
  if (j1 > n) j1 = n;
  float xi = 0.f, yi = 0.f, zi = 0.f;
  if (i < n) {
    xi = nb_load(s, i, 0);
    yi = nb_load(s, i, 1);
    zi = nb_load(s, i, 2);
  }
  // counted once per particle: in the first slice of each i-block
  const bool counting = cnt.fac || cnt.heat[0];
  if (counting && blockIdx.y == 0)
    for (uint32_t f = 0; f < 3; ++f) nb_count(cnt, s, f, 0, i, i < n);
  uint32_t jloads = 0;  // j-tile loads of this thread (each of leaves 0, 1, 2, 6)
  // running sums with compensation (Kahan) across j-tiles
  float ax = 0.f, ay = 0.f, az = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
  for (uint32_t jt = j0; jt < j1; jt += NB_T) {
    const uint32_t j = jt + threadIdx.x;
    const uint16_t me = (uint16_t)threadIdx.x;  // this thread's particle in the j-tile
    float px = 0.f, py = 0.f, pz = 0.f, pm = 0.f;  // mass 0 outside the slice: no contribution
    if (j < j1) {
      px = nb_load(s, j, 0);
      py = nb_load(s, j, 1);
      pz = nb_load(s, j, 2);
      pm = nb_load(s, j, 6);
      ++jloads;
    }
    if (counting && cnt.heat[0]) {
      nb_heat(cnt, 0, j < j1 ? nb_off(s, j, 0) : 0u, j < j1);
      nb_heat(cnt, 1, j < j1 ? nb_off(s, j, 1) : 0u, j < j1);
      nb_heat(cnt, 2, j < j1 ? nb_off(s, j, 2) : 0u, j < j1);
      nb_heat(cnt, 6, j < j1 ? nb_off(s, j, 6) : 0u, j < j1);
    }
    tile.store<0>(me, px);
    tile.store<1>(me, py);
    tile.store<2>(me, pz);
    tile.store<6>(me, pm);
    __syncthreads();
    float tx = 0.f, ty = 0.f, tz = 0.f;
#pragma unroll 8
    for (uint32_t k = 0; k < NB_T; ++k) {
      const uint16_t kk = (uint16_t)k;
      const float qx = tile.load<0>(kk), qy = tile.load<1>(kk), qz = tile.load<2>(kk), qm = tile.load<6>(kk);
      const float dx = qx - xi, dy = qy - yi, dz = qz - zi;
      const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2)));
      const float inv = __builtin_amdgcn_rsqf(r2);
      const float w = qm * inv * inv * inv;
      tx = __builtin_fmaf(dx, w, tx);
      ty = __builtin_fmaf(dy, w, ty);
      tz = __builtin_fmaf(dz, w, tz);
    }
    float y, t;
    y = tx - cx; t = ax + y; cx = (t - ax) - y; ax = t;
    y = ty - cy; t = ay + y; cy = (t - ay) - y; ay = t;
    y = tz - cz; t = az + y; cz = (t - az) - y; az = t;
    __syncthreads();
  }
  if (i < n) {
    float* p = part + (size_t)blockIdx.y * 3u * n;
    p[i] = ax;
    p[n + i] = ay;
    p[2u * n + i] = az;
  }
  if (cnt.fac) {
    nb_fac_add(cnt, 0, jloads);
    nb_fac_add(cnt, 2, jloads);
    nb_fac_add(cnt, 4, jloads);
    nb_fac_add(cnt, 12, jloads);
  }
}

__device__ __forceinline__ void nb_accel(const float* __restrict__ part, uint32_t n, uint32_t slices, uint32_t i,
                                         float& ax, float& ay, float& az) {
  ax = ay = az = 0.f;
  for (uint32_t sl = 0; sl < slices; ++sl) {  // fixed order: deterministic
    const float* p = part + (size_t)sl * 3u * n;
    ax += p[i];
    ay += p[n + i];
    az += p[2u * n + i];
  }
}

// Kick (v += dt a) then drift (x += dt v as stored), physical storage.
__global__ __launch_bounds__(NB_T) void k_nb_kick_drift(const Side s, uint32_t n, float dt, uint32_t slices,
                                                       const float* __restrict__ part, const NbCount cnt) {
  const uint32_t i = blockIdx.x * NB_T + threadIdx.x;
  if (cnt.fac || cnt.heat[0]) {  // vel loaded and stored, then pos loaded and stored
    for (uint32_t c = 0; c < 3; ++c) {
      nb_count(cnt, s, 3 + c, 0, i, i < n);
      nb_count(cnt, s, 3 + c, 1, i, i < n);
      nb_count(cnt, s, c, 0, i, i < n);
      nb_count(cnt, s, c, 1, i, i < n);
    }
  }
  if (i >= n) return;
  float a[3];
  nb_accel(part, n, slices, i, a[0], a[1], a[2]);
#pragma unroll
  for (uint32_t c = 0; c < 3; ++c) {
    const float v = __builtin_fmaf(dt, a[c], nb_load(s, i, 3 + c));
    nb_store(s, i, 3 + c, v);
    const float x = __builtin_fmaf(dt, v, nb_load(s, i, c));
    nb_store(s, i, c, x);
  }
}

// Kick and drift for bit-packed streams: codes of a 256-particle tile are
// staged in LDS and the stream words (a tile is a whole number of words)
// are assembled and stored by one lane each.
__global__ __launch_bounds__(NB_T) void k_nb_kick_drift_stream(const Side s, uint32_t n, float dt,
                                                              uint32_t slices, const float* __restrict__ part,
                                                              const NbCount cnt) {
  __shared__ uint32_t codes[6][NB_T];
  const uint32_t i0 = blockIdx.x * NB_T;
  const uint32_t i = i0 + threadIdx.x;
  if (cnt.fac)
    for (uint32_t f = 0; f < 6; ++f) {  // every position and velocity code loaded once and stored once
      nb_fac_add(cnt, 2u * f, i < n ? 1u : 0u);
      nb_fac_add(cnt, 2u * f + 1u, i < n ? 1u : 0u);
    }
  const uint32_t nt = n - i0 < NB_T ? n - i0 : NB_T;
  const uint32_t E = s.exp_bits, M = s.man_bits, B = s.bits;
  if (i < n) {
    float a[3];
    nb_accel(part, n, slices, i, a[0], a[1], a[2]);
#pragma unroll
    for (uint32_t c = 0; c < 3; ++c) {
      const float v = __builtin_fmaf(dt, a[c], nb_load(s, i, 3 + c));
      const uint32_t cv = enc_f32(__builtin_bit_cast(uint32_t, v), E, M);
      const float vs = __builtin_bit_cast(float, dec_f32(cv, E, M));  // velocity as stored
      const float x = __builtin_fmaf(dt, vs, nb_load(s, i, c));
      codes[3 + c][threadIdx.x] = cv;
      codes[c][threadIdx.x] = enc_f32(__builtin_bit_cast(uint32_t, x), E, M);
    }
  }
  __syncthreads();
  const uint32_t words = (nt * B + 31u) >> 5;
  const uint32_t wbase = (i0 * B) >> 5;  // i0 * B is a multiple of 32
  const uint32_t mask = B >= 32u ? 0xFFFFFFFFu : ((1u << B) - 1u);
  for (uint32_t q = threadIdx.x; q < 6u * words; q += NB_T) {
    const uint32_t f = q / words, w = q - f * words;
    const uint32_t bit0 = w * 32u;
    uint32_t r = bit0 / B;
    const uint32_t first = bit0 - r * B;
    uint32_t acc = (codes[f][r] & mask) >> first;
    uint32_t nb = B - first;
    for (++r; nb < 32u && r < nt; ++r, nb += B) acc |= (codes[f][r] & mask) << nb;
    __builtin_amdgcn_raw_buffer_store_b32(acc, nb_rsrc(s, f), (wbase + w) * 4u, 0, 0);
  }
}

// ---------------------------------------------------------------------------
// Energy in FP64 (deterministic fixed-order reductions)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(NB_T) void k_nb_decode64(const Side s, uint32_t n, double* __restrict__ d,
                                                     const NbCount cnt) {
  const uint32_t i = blockIdx.x * NB_T + threadIdx.x;
  if (cnt.fac || cnt.heat[0])
    for (uint32_t f = 0; f < 7; ++f) nb_count(cnt, s, f, 0, i, i < n);
  if (i >= n) return;
  for (uint32_t f = 0; f < 7; ++f) d[(size_t)f * n + i] = (double)nb_load(s, i, f);
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (uint32_t w = NB_T / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// block (bi, bj), bj >= bi: sum over i in block bi, j in block bj, j > i of
// m_i m_j / sqrt(|x_i - x_j|^2 + eps2); blocks with bj < bi write 0.
__global__ __launch_bounds__(NB_T) void k_nb_potential(const double* __restrict__ d, uint32_t n, double eps2,
                                                      double* __restrict__ partial) {
  __shared__ double red[NB_T];
  __shared__ double4 tj[NB_T];
  const uint32_t bi = blockIdx.x, bj = blockIdx.y;
  double acc = 0.0;
  if (bj >= bi) {
    const uint32_t j = bj * NB_T + threadIdx.x;
    tj[threadIdx.x] = j < n ? double4{d[j], d[n + j], d[2u * n + j], d[6u * n + j]} : double4{0, 0, 0, 0};
    __syncthreads();
    const uint32_t i = bi * NB_T + threadIdx.x;
    if (i < n) {
      const double xi = d[i], yi = d[n + i], zi = d[2u * n + i], mi = d[6u * n + i];
      for (uint32_t k = 0; k < NB_T; ++k) {
        const uint32_t jj = bj * NB_T + k;
        if (jj <= i || jj >= n) continue;
        const double4 q = tj[k];
        const double dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
        acc += q.w / sqrt(dx * dx + dy * dy + dz * dz + eps2);
      }
      acc *= mi;
    }
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) partial[(size_t)bi * gridDim.y + bj] = t;
}

__global__ __launch_bounds__(NB_T) void k_nb_kinetic(const double* __restrict__ d, uint32_t n,
                                                    double* __restrict__ partial) {
  __shared__ double red[NB_T];
  const uint32_t i = blockIdx.x * NB_T + threadIdx.x;
  double k = 0.0;
  if (i < n) {
    const double vx = d[3u * n + i], vy = d[4u * n + i], vz = d[5u * n + i];
    k = 0.5 * d[6u * n + i] * (vx * vx + vy * vy + vz * vz);
  }
  const double t = block_sum(k, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// result = sum(kin[0..nk)) - sum(pot[0..np)), summed by one workgroup in fixed order
__global__ __launch_bounds__(NB_T) void k_nb_final(const double* __restrict__ kin, uint32_t nk,
                                                  const double* __restrict__ pot, uint32_t np,
                                                  double* __restrict__ out) {
  __shared__ double red[NB_T];
  double k = 0.0, p = 0.0;
  for (uint32_t q = threadIdx.x; q < nk; q += NB_T) k += kin[q];
  for (uint32_t q = threadIdx.x; q < np; q += NB_T) p += pot[q];
  const double ks = block_sum(k, red);
  const double ps = block_sum(p, red);
  if (threadIdx.x == 0) out[0] = ks - ps;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

namespace {

struct Scratch {
  std::mutex mu;
  void* ptr = nullptr;
  size_t bytes = 0;
  double* host = nullptr;  // pinned result slot
};

Scratch g_scratch[64];

// Scratch of the allocation-free step (nbody_step_noalloc): the per-slice
// partial accelerations live in this file-scope device array instead of a
// library allocation.  Each GPU holds its own copy at its own address, which
// hipGetSymbolAddress returns once per device with that device current; the
// host code only ever passes that address to kernels, never the array's name.
constexpr size_t kStaticScratchBytes = 16u << 20;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

struct StaticScratch {
  std::once_flag once;
  hipError_t err = hipSuccess;
  void* ptr = nullptr;
};

StaticScratch g_static[64];

llama_status static_scratch_get(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(LLAMA_ERR_HIP, "hipGetDevice failed");
  StaticScratch& sc = g_static[dev];
  std::call_once(sc.once, [&sc]() { sc.err = hipGetSymbolAddress(&sc.ptr, HIP_SYMBOL(scratch)); });
  if (sc.err != hipSuccess || !sc.ptr)
    return fail(LLAMA_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(sc.err));
  *out = sc.ptr;
  return LLAMA_OK;
}

llama_status scratch_get(size_t bytes, hipStream_t st, void** out, double** host) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(LLAMA_ERR_HIP, "hipGetDevice failed");
  Scratch& sc = g_scratch[dev];
  std::lock_guard<std::mutex> lock(sc.mu);
  if (sc.bytes < bytes) {
    if (sc.ptr) {
      (void)hipStreamSynchronize(st);
      (void)hipDeviceSynchronize();
      (void)hipFree(sc.ptr);
      sc.ptr = nullptr;
      sc.bytes = 0;
    }
    if (hipMalloc(&sc.ptr, bytes) != hipSuccess) return fail(LLAMA_ERR_NO_MEMORY, "scratch allocation failed");
    sc.bytes = bytes;
  }
  if (!sc.host && hipHostMalloc((void**)&sc.host, sizeof(double), hipHostMallocDefault) != hipSuccess)
    return fail(LLAMA_ERR_NO_MEMORY, "pinned allocation failed");
  *out = sc.ptr;
  if (host) *host = sc.host;
  return LLAMA_OK;
}

// The data side of a particle view and, for FIELD_ACCESS_COUNT and HEATMAP
// views, the counters every access adds to (Sec. 4).
llama_status nb_side(const llama_view* vin, Side& s, NbCount& cnt) {
  if (!vin) return fail(LLAMA_ERR_INVALID_ARG, "view is NULL");
  if (vin->rec.size() != 7) return fail(LLAMA_ERR_INVALID_ARG, "n-body needs the 7-field particle record");
  for (auto t : vin->rec)
    if (t != vin->rec[0] || (t != LLAMA_F32 && t != LLAMA_F64))
      return fail(LLAMA_ERR_INVALID_ARG, "n-body needs 7 F32 or 7 F64 leaves");
  cnt = NbCount{};
  llama_view inner;
  const llama_view* v = vin;
  if (instrumented(vin)) {
    inner_view(vin, inner);
    v = &inner;
    const size_t c = inner.blobs.size();  // the counter blobs follow the data blobs
    if (vin->map.kind == LLAMA_MAP_FIELD_ACCESS_COUNT) {
      cnt.fac = (uint64_t*)vin->blobs[c];
    } else {
      uint32_t sh = 0;
      while ((1u << sh) < vin->map.lanes) ++sh;
      cnt.heat_shift = sh;
      const bool per_field = inner.map.kind == LLAMA_MAP_SOA_MB;
      for (uint32_t f = 0; f < 7; ++f) cnt.heat[f] = (uint64_t*)vin->blobs[c + (per_field ? f : 0u)];
    }
  }
  llama_scalar ut, st;
  llama_status r = make_side(v, s, ut, st);
  if (r != LLAMA_OK) return r;
  const bool f32_storage = (s.vkind == VK_RAW && ut == LLAMA_F32) || (s.vkind == VK_CONV && st == LLAMA_F32);
  const bool stream = s.vkind == VK_FLOAT && s.exp_bits <= 8 && s.man_bits <= 23;
  if (!(f32_storage && s.layout != LY_STREAM) && !stream)
    return fail(LLAMA_ERR_UNSUPPORTED,
                "n-body supports F32 storage (physical or ChangeType F64->F32) and BitPackedFloat with E<=8, M<=23");
  if (v->n > (1u << 24)) return fail(LLAMA_ERR_UNSUPPORTED, "n-body supports at most 2^24 particles");
  for (auto b : v->blob_bytes)
    if (b > 0xFFFFFFFFull) return fail(LLAMA_ERR_UNSUPPORTED, "n-body blobs must be < 4 GiB");
  return LLAMA_OK;
}

uint32_t nb_slices(uint32_t n) {
  // enough workgroups to fill 256 CUs several times over
  const uint32_t iblocks = (n + NB_T - 1) / NB_T;
  uint32_t sl = 1;
  while (iblocks * sl < 2048 && sl * NB_T * 2 <= n) sl *= 2;
  return sl;
}

// Bytes of per-slice partial accelerations for n particles.
size_t nb_scratch_bytes(uint32_t n) { return (size_t)nb_slices(n) * 3u * n * sizeof(float); }

// Largest particle count whose partial accelerations fit the static scratch
// (for n >= 2^19 one slice, 12 bytes per particle).
constexpr uint32_t kNoallocMaxParticles = (uint32_t)(kStaticScratchBytes / 12u);

// The launches of `steps` update + move steps, partial sums in `part`
// (nb_scratch_bytes(n) bytes; every element read is written first).
llama_status nb_launch_steps(const Side& s, const NbCount& cnt, uint32_t n, uint32_t steps, float dt, float eps2,
                             float* part, hipStream_t st) {
  const uint32_t slices = nb_slices(n);
  uint32_t per = (n + slices - 1) / slices;
  per = (per + NB_T - 1) / NB_T * NB_T;
  const uint32_t iblocks = (n + NB_T - 1) / NB_T;
  const uint32_t used = (n + per - 1) / per;
  for (uint32_t k = 0; k < steps; ++k) {
    hipLaunchKernelGGL(k_nb_update, dim3(iblocks, used), dim3(NB_T), 0, st, s, n, eps2, per, part, cnt);
    if (s.layout == LY_STREAM)
      hipLaunchKernelGGL(k_nb_kick_drift_stream, dim3(iblocks), dim3(NB_T), 0, st, s, n, dt, used, part, cnt);
    else
      hipLaunchKernelGGL(k_nb_kick_drift, dim3(iblocks), dim3(NB_T), 0, st, s, n, dt, used, part, cnt);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LLAMA_ERR_HIP, std::string("n-body launch: ") + hipGetErrorString(e));
  return LLAMA_OK;
}

}  // namespace
}  // namespace lm

using namespace lm;

extern "C" {

llama_status nbody_step(llama_view* view, uint32_t steps, float dt, float eps2, void* stream) {
  clear_error();
  Side s;
  NbCount cnt;
  llama_status r = nb_side(view, s, cnt);
  if (r != LLAMA_OK) return r;
  if (!(eps2 > 0.f)) return fail(LLAMA_ERR_INVALID_ARG, "eps2 must be > 0");
  const uint32_t n = (uint32_t)view->n;
  if (n == 0 || steps == 0) return LLAMA_OK;
  hipStream_t st = (hipStream_t)stream;
  void* buf;
  if ((r = scratch_get(nb_scratch_bytes(n), st, &buf, nullptr)) != LLAMA_OK) return r;
  return nb_launch_steps(s, cnt, n, steps, dt, eps2, (float*)buf, st);
}

llama_status nbody_step_noalloc(llama_view* view, uint32_t steps, float dt, float eps2, void* stream) {
  clear_error();
  Side s;
  NbCount cnt;
  llama_status r = nb_side(view, s, cnt);
  if (r != LLAMA_OK) return r;
  if (!(eps2 > 0.f)) return fail(LLAMA_ERR_INVALID_ARG, "eps2 must be > 0");
  const uint32_t n = (uint32_t)view->n;
  const size_t need = nb_scratch_bytes(n);
  if (need > kStaticScratchBytes)
    return fail(LLAMA_ERR_NO_MEMORY, "nbody_step_noalloc: " + std::to_string(n) + " particles need " +
                                         std::to_string(need) + " bytes of scratch, the static maximum is " +
                                         std::to_string(kStaticScratchBytes) + " (at most " +
                                         std::to_string(kNoallocMaxParticles) + " particles)");
  if (n == 0 || steps == 0) return LLAMA_OK;
  void* buf;
  if ((r = static_scratch_get(&buf)) != LLAMA_OK) return r;
  return nb_launch_steps(s, cnt, n, steps, dt, eps2, (float*)buf, (hipStream_t)stream);
}

llama_status nbody_energy(const llama_view* view, float eps2, double* energy, void* stream) {
  clear_error();
  if (!energy) return fail(LLAMA_ERR_INVALID_ARG, "energy is NULL");
  Side s;
  NbCount cnt;
  llama_status r = nb_side(view, s, cnt);
  if (r != LLAMA_OK) return r;
  const uint32_t n = (uint32_t)view->n;
  hipStream_t st = (hipStream_t)stream;
  const uint32_t nb = (n + NB_T - 1) / NB_T;
  const size_t dbytes = (size_t)7 * n * sizeof(double);
  const size_t pbytes = (size_t)nb * nb * sizeof(double);
  const size_t kbytes = (size_t)nb * sizeof(double);
  void* buf;
  double* host;
  if ((r = scratch_get(dbytes + pbytes + kbytes + 64, st, &buf, &host)) != LLAMA_OK) return r;
  if (n == 0) {
    *energy = 0.0;
    return LLAMA_OK;
  }
  double* d = (double*)buf;
  double* pot = d + (size_t)7 * n;
  double* kin = pot + (size_t)nb * nb;
  double* out = kin + nb;
  hipLaunchKernelGGL(k_nb_decode64, dim3(nb), dim3(NB_T), 0, st, s, n, d, cnt);
  hipLaunchKernelGGL(k_nb_potential, dim3(nb, nb), dim3(NB_T), 0, st, (const double*)d, n, (double)eps2, pot);
  hipLaunchKernelGGL(k_nb_kinetic, dim3(nb), dim3(NB_T), 0, st, (const double*)d, n, kin);
  hipLaunchKernelGGL(k_nb_final, dim3(1), dim3(NB_T), 0, st, (const double*)kin, nb, (const double*)pot, nb * nb, out);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(host, out, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(LLAMA_ERR_HIP, std::string("n-body energy: ") + hipGetErrorString(e));
  *energy = *host;
  return LLAMA_OK;
}

}  // extern "C"
