// Copies between views linearised in different orders (Sec. 2 array
// extents: row-major or column-major).  dst(a) = src(a) for every multi-index
// a: a batched 2-D transpose of records through LDS.  A workgroup takes one
// tile of T x T records: for each of T positions p along the destination's
// fastest axis P it loads T records that are consecutive in the source (along
// Q), and for each of the T positions q along Q it stores T records that are
// consecutive in the destination.  Each lane moves one unit (U bytes) of one
// record per step; consecutive lanes take consecutive records of one column
// (planar, AoSoA) or consecutive units of one record (AoS), so every wave
// access is one contiguous run.  The LDS image is [unit][q][p] with rows of
// T + 1 units, which keeps the column writes free of bank conflicts.
#include "kernels.hpp"

namespace lm {

// 64-bit quotient x / L by multiply-high with m = ceil(2^64 / L) (exact for
// x * L < 2^64), or a shift when L is a power of two (m = 0).
__device__ __forceinline__ uint64_t xp_div(uint64_t x, uint64_t m, const Div& d) {
  return m ? __umul64hi(x, m) : (x >> d.sh);
}

// Address of unit u of record i of a physical side.
template <int U>
__device__ __forceinline__ uint8_t* xp_addr(const Side& s, uint64_t lmag, uint64_t i, uint32_t u) {
  const uint32_t byte = u * U;
  const uint32_t c = byte >> s.log2cs, bo = byte & (s.cs - 1u);
  switch (s.layout) {
    case LY_AOS:
      return (uint8_t*)s.blob[0] + i * s.rec_bytes + byte;
    case LY_PLANAR:
      return (uint8_t*)(s.mb ? s.blob[c] : s.blob[0]) + (s.mb ? 0ull : (uint64_t)c * s.n * s.cs) + i * s.cs + bo;
    default: {  // AoSoA: block, column, lane
      const uint64_t blk = xp_div(i, lmag, s.div_L);
      const uint64_t lane = i - blk * s.lanes;
      return (uint8_t*)s.blob[0] + blk * s.lanes * s.rec_bytes + (uint64_t)c * s.lanes * s.cs + lane * s.cs + bo;
    }
  }
}

template <int U>
struct Unit;
template <> struct Unit<1> { typedef uint8_t T; };
template <> struct Unit<2> { typedef uint16_t T; };
template <> struct Unit<4> { typedef uint32_t T; };
template <> struct Unit<8> { typedef uint64_t T; };

template <int U>
__global__ __launch_bounds__(kThreads) void k_xpose(const XposeArgs a) {
  typedef typename Unit<U>::T W;
  extern __shared__ __attribute__((aligned(16))) uint8_t lds_raw[];
  W* img = (W*)lds_raw;
  const uint32_t T = a.T, lt = a.log2T, row = T + 1u, nu = a.nunits;
  const uint32_t per_tile = (T * T) * nu;
  for (uint64_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    // tile -> (middle index, tile along P, tile along Q)
    const uint64_t qt = t % a.nQt, rest = t / a.nQt;
    const uint64_t pt = rest % a.nPt;
    uint64_t m = rest / a.nPt, sbase = 0, dbase = 0;
    for (uint32_t k = 0; k < a.nmid; ++k) {  // last middle axis varies fastest
      const uint32_t j = a.nmid - 1u - k;
      const uint64_t x = m % a.mext[j];
      m /= a.mext[j];
      sbase += x * a.msrc[j];
      dbase += x * a.mdst[j];
    }
    const uint64_t p0 = pt << lt, q0 = qt << lt;
    const uint32_t np = (uint32_t)(a.eP - p0 < T ? a.eP - p0 : T);
    const uint32_t nq = (uint32_t)(a.eQ - q0 < T ? a.eQ - q0 : T);
    sbase += p0 * a.sP + q0;  // source record of (p, q) = sbase + p sP + q
    dbase += q0 * a.dQ + p0;  // destination record of (p, q) = dbase + q dQ + p
    for (uint32_t idx = threadIdx.x; idx < per_tile; idx += blockDim.x) {
      uint32_t p, q, u;
      if (a.src_rec_major) {
        const uint32_t r = fdiv(idx, a.div_units);
        u = idx - r * nu;
        q = r & (T - 1u);
        p = r >> lt;
      } else {
        q = idx & (T - 1u);
        const uint32_t r = idx >> lt;
        p = fdiv(r, a.div_units);
        u = r - p * nu;
      }
      if (p < np && q < nq)
        img[(u * T + q) * row + p] = *(const W*)xp_addr<U>(a.src, a.src_lmag, sbase + (uint64_t)p * a.sP + q, u);
    }
    __syncthreads();
    for (uint32_t idx = threadIdx.x; idx < per_tile; idx += blockDim.x) {
      uint32_t p, q, u;
      if (a.dst_rec_major) {
        const uint32_t r = fdiv(idx, a.div_units);
        u = idx - r * nu;
        p = r & (T - 1u);
        q = r >> lt;
      } else {
        p = idx & (T - 1u);
        const uint32_t r = idx >> lt;
        q = fdiv(r, a.div_units);
        u = r - q * nu;
      }
      if (p < np && q < nq)
        *(W*)xp_addr<U>(a.dst, a.dst_lmag, dbase + (uint64_t)q * a.dQ + p, u) = img[(u * T + q) * row + p];
    }
    __syncthreads();
  }
}

hipError_t launch_xpose(const XposeArgs& a, uint32_t unit, uint32_t grid, uint32_t lds, hipStream_t st) {
  switch (unit) {
    case 1: hipLaunchKernelGGL(k_xpose<1>, dim3(grid), dim3(kThreads), lds, st, a); break;
    case 2: hipLaunchKernelGGL(k_xpose<2>, dim3(grid), dim3(kThreads), lds, st, a); break;
    case 4: hipLaunchKernelGGL(k_xpose<4>, dim3(grid), dim3(kThreads), lds, st, a); break;
    case 8: hipLaunchKernelGGL(k_xpose<8>, dim3(grid), dim3(kThreads), lds, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lm
