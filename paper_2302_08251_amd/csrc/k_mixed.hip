// Copies of records whose leaves differ in size (Sec. 1 record dimension: a
// record is any tree of leaf types; e.g. the C struct {u8; f64; i16; f32}),
// and of SPLIT views (Sec. 3) against a partner that is not divided at the
// same leaf.  The tile engine moves records as columns of one element size
// and one mapping; here each thread takes one record and moves its leaves one
// by one, each through the mapping of its own SPLIT part: a leaf is one
// naturally aligned load and store where both sides keep it whole and aligned
// (AoS with C alignment, SoA, AoSoA with aligned blocks), otherwise its bytes
// move one at a time (packed AoS, Bytesplit byte columns).  The leaf loop is
// uniform across the wave, so every branch on a leaf's size or form is a
// scalar branch.  Consecutive lanes take consecutive records, so planar
// accesses coalesce and record-major ones stay within the wave's own lines.
#include "mixing.hpp"

namespace lm {

__global__ __launch_bounds__(kThreads) void k_mixed(MixArgs a) {
  const uint64_t stride = (uint64_t)gridDim.x * kThreads;
  for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < a.n; i += stride) {
    const uint64_t is = mix_src_index(a.order, i);
    for (uint32_t f = 0; f < a.nf; ++f) {
      const uint32_t lsz = a.lsz[f];
      mix_store(a.dst, i, f, lsz, mix_load(a.src, is, f, lsz));
    }
  }
}

hipError_t launch_mixed(const MixArgs& a, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(k_mixed, dim3(grid), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace lm
