// Access counters of the instrumentation mappings (Sec. 4): FieldAccessCount
// and Heatmap.
//
// The paper counts with one atomic increment per access, made by the code
// that accesses the view.  Here the copy kernels move whole tiles, so the
// counters of a copy are added after it on the same stream, aggregated
// instead of one per access.  A copy loads every field of every record of
// the source once and stores it once into the destination.
//  - FieldAccessCount: one atomic add of n per field counter.
//  - Heatmap: each counter (G bytes of an inner blob) belongs to one thread.
//    The thread counts the accesses that touch those bytes from the inner
//    layout's geometry and adds them with a plain read-modify-write,
//    skipping zeros.  Each counter is then touched once per copy, so the
//    kernel is bound by HBM: 8 bytes read and 8 written per counter.
#include "host.hpp"

namespace lm {

__global__ __launch_bounds__(64) void k_field_count(unsigned long long* counts, uint32_t nf, uint32_t which,
                                                    unsigned long long n) {
  const uint32_t f = threadIdx.x + blockIdx.x * blockDim.x;
  if (f < nf) atomicAdd(counts + 2u * f + which, n);
}

// Accessed elements of one period k of the inner layout that meet the bytes
// [lo, hi) of that period (0 <= lo < hi <= period).  T = uint32_t when the
// period fits 32 bits.
template <typename T>
__device__ inline uint64_t period_hits(const HeatGeo& g, uint64_t k, T lo, T hi) {
  const uint64_t left = g.n - k * g.recs;
  const T rk = (T)(left < g.recs ? left : g.recs);  // records in this period
  T c = 0;
  for (uint32_t f = 0; f < g.nruns; ++f) {
    const T o = (T)g.run_off[f];
    const T end = o + (rk << g.run_lsz[f]);
    if (hi <= o || lo >= end) continue;
    const T e0 = ((lo > o ? lo : o) - o) >> g.run_lsz[f];
    const T e1 = ((hi < end ? hi : end) - 1 - o) >> g.run_lsz[f];
    c += e1 - e0 + 1;
  }
  return c;
}

// floor(a / p) for a < 2^53 and p >= 1: the double quotient is within one of
// the true one, and one step of integer correction makes it exact.
__device__ inline uint64_t div_floor(uint64_t a, uint64_t p, double inv_p) {
  uint64_t k = (uint64_t)((double)a * inv_p);
  if (k * p > a) --k;
  else if ((k + 1) * p <= a) ++k;
  return k;
}

template <typename Hits>
__device__ inline uint64_t granule_hits(const HeatGeo& g, uint64_t q, uint64_t used, double inv_p, Hits hits) {
  const uint64_t a = q << g.shift;
  uint64_t b = a + (1ull << g.shift);
  if (b > used) b = used;
  if (a >= b) return 0;
  const uint64_t k0 = div_floor(a, g.period, inv_p), k1 = div_floor(b - 1, g.period, inv_p);
  if (k0 == k1) return hits(k0, a - k0 * g.period, b - k0 * g.period);
  // the periods strictly between k0 and k1 are full
  return hits(k0, a - k0 * g.period, g.period) + hits(k1, 0, b - k1 * g.period) +
         (k1 - k0 - 1) * g.recs * g.nruns;
}

// Periods of at most kHeatTable bytes get two per-byte tables in LDS, built
// by each block: A[x] = elements of a full period that start before byte x,
// B[x] = elements that end at or before x.  The elements meeting [lo, hi)
// are then A[hi] - B[lo]; the last, partial period keeps the loop.
constexpr uint32_t kHeatTable = 2048;

// Counter pairs (16 bytes) per thread, read and written as one 16-byte
// access, with consecutive lanes on consecutive pairs so that every wave
// store writes 1 KiB of whole lines; a block covers kHeatRounds * 256 pairs
// per grid-stride step.  When a counter is no wider than a period, the
// pair's period and offset come from one division and the second counter
// advances by G; a counter that straddles a period boundary (or is wider
// than a period) takes the general path.  Every counter belongs to one
// thread of the launch, so a plain read-modify-write is exact; launches
// that overlap in time on the same counter blob race, as overlapping writes
// to any blob do.
constexpr uint32_t kHeatRounds = 2;

template <typename T>
__global__ __launch_bounds__(256) void k_heatmap(unsigned long long* ctr, uint64_t ncounters, const HeatGeo g) {
  const uint64_t nper = (g.n + g.recs - 1) / g.recs;  // periods holding records
  const uint64_t used = nper * g.period;              // bytes of those periods
  const double inv_p = 1.0 / (double)g.period;
  const uint64_t G = 1ull << g.shift;
  const uint64_t npairs = ncounters / 2;
  const uint64_t step = (uint64_t)gridDim.x * blockDim.x * kHeatRounds;
  ulonglong2* c2 = reinterpret_cast<ulonglong2*>(ctr);
  __shared__ uint32_t tA[kHeatTable + 1], tB[kHeatTable + 1];
  // a block builds its tables at (period + 1) * runs steps: bounded so that
  // wide records with long periods keep the loop instead
  const bool table = g.period <= kHeatTable && (g.period + 1) * g.nruns <= 16384;
  const uint64_t nfull = g.n / g.recs;  // periods holding g.recs records
  if (table) {
    const uint32_t P = (uint32_t)g.period, R = (uint32_t)g.recs;
    for (uint32_t x = threadIdx.x; x <= P; x += blockDim.x) {
      uint32_t ca = 0, cb = 0;
      for (uint32_t f = 0; f < g.nruns; ++f) {
        const uint32_t o = (uint32_t)g.run_off[f], l = g.run_lsz[f];
        if (x <= o) continue;
        const uint32_t d = x - o;
        const uint32_t sa = (d + (1u << l) - 1u) >> l, sb = d >> l;
        ca += sa < R ? sa : R;
        cb += sb < R ? sb : R;
      }
      tA[x] = ca;
      tB[x] = cb;
    }
    __syncthreads();
  }
  auto hits = [&](uint64_t k, uint64_t lo, uint64_t hi) -> uint64_t {
    if (table && k < nfull) return (uint64_t)(tA[hi] - tB[lo]);
    return period_hits<T>(g, k, (T)lo, (T)hi);
  };
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x * kHeatRounds; base < npairs; base += step) {
#pragma unroll
    for (uint32_t r = 0; r < kHeatRounds; ++r) {
      const uint64_t p = base + r * blockDim.x + threadIdx.x;
      if (p >= npairs) break;
      const uint64_t q0 = 2 * p, a = q0 << g.shift;
      uint64_t h0, h1;
      if (G > g.period || a >= used) {
        h0 = granule_hits(g, q0, used, inv_p, hits);
        h1 = granule_hits(g, q0 + 1, used, inv_p, hits);
      } else {
        uint64_t k = div_floor(a, g.period, inv_p), lo = a - k * g.period;
        h0 = lo + G > g.period ? granule_hits(g, q0, used, inv_p, hits) : hits(k, lo, lo + G);
        lo += G;
        if (lo >= g.period) {
          lo -= g.period;
          ++k;
        }
        if (k >= nper) h1 = 0;
        else if (lo + G > g.period) h1 = granule_hits(g, q0 + 1, used, inv_p, hits);
        else h1 = hits(k, lo, lo + G);
      }
      if (h0 | h1) {
        ulonglong2 v = c2[p];
        v.x += h0;
        v.y += h1;
        c2[p] = v;
      }
    }
  }
  if ((ncounters & 1) && blockIdx.x == 0 && threadIdx.x == 0)
    ctr[ncounters - 1] += granule_hits(g, ncounters - 1, used, inv_p, hits);
}

void launch_field_count(void* counts, uint32_t nf, uint32_t which, uint64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_field_count, dim3(1), dim3(64), 0, st, (unsigned long long*)counts, nf, which,
                     (unsigned long long)n);
}

void launch_heatmap(void* ctr, uint64_t ncounters, const HeatGeo& g, int num_cus, hipStream_t st) {
  const uint64_t want = (ncounters / 2 + 256 * kHeatRounds - 1) / (256 * kHeatRounds), cap = (uint64_t)num_cus * 32;
  const uint32_t grid = (uint32_t)(want < 1 ? 1 : want < cap ? want : cap);
  // a period of at most 2^32 - 1 bytes keeps the in-period arithmetic in 32 bits
  if (g.period <= 0xFFFFFFFFull)
    hipLaunchKernelGGL(k_heatmap<uint32_t>, dim3(grid), dim3(256), 0, st, (unsigned long long*)ctr, ncounters, g);
  else
    hipLaunchKernelGGL(k_heatmap<uint64_t>, dim3(grid), dim3(256), 0, st, (unsigned long long*)ctr, ncounters, g);
}

}  // namespace lm
