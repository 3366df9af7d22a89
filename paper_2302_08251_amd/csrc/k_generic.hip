// Value-level copies: dst(i).f = src(i).f with each value loaded through the
// source mapping and stored through the destination mapping (Sec. 1 copy;
// Sec. 3 computed mappings), for the pairs the tile kernels do not move:
// two computed views (bit-packed to bit-packed, ChangeType to ChangeType with
// conversions on both sides), integer ChangeType, bit-packed codes of 33 to
// 64 bits, bit-packed floats of f16 / bf16 leaves, SPLIT trees with computed
// parts against a partner of another form.  One thread takes 32
// consecutive records (of the destination's order) and moves them field by
// field: 32 codes of B bits are exactly B whole stream words, so a bit-packed
// destination is written without atomics, one word at a time as the codes
// fill it.  The value codecs here are written for this kernel from the IEEE
// binary formats: narrowing (truncating or round to nearest even) and exact
// widening between any two float formats, integer narrowing and extension.
#include "mixing.hpp"

namespace lm {

__device__ __forceinline__ uint64_t low_mask64(uint32_t b) { return b >= 64u ? ~0ull : ((1ull << b) - 1ull); }

// Float bits of format (Es, Ms) -> format (E, M) with E <= Es, M <= Ms:
// truncation toward zero or round to nearest even (ties compare the last bit
// of the significand: the mantissa's, or a normal's hidden bit when M = 0); a
// value past the largest finite code gives Inf; gradual underflow; a NaN
// keeps its sign and top M payload bits and gets its quiet bit (M = 0: Inf).
__device__ uint64_t gen_narrow(uint64_t x, uint32_t Es, uint32_t Ms, uint32_t E, uint32_t M, bool rne) {
  const uint64_t sign = (x >> (Es + Ms)) & 1ull;
  const uint32_t emaxS = (1u << Es) - 1u, emaxT = (1u << E) - 1u;
  const uint32_t ex = (uint32_t)((x >> Ms) & emaxS);
  const uint64_t mx = x & low_mask64(Ms);
  const int biasS = (1 << (Es - 1)) - 1, biasT = (1 << (E - 1)) - 1;
  uint64_t code;
  if (ex == emaxS) {  // Inf, NaN
    code = (uint64_t)emaxT << M;
    if (mx && M) code |= (1ull << (M - 1u)) | (mx >> (Ms - M));
  } else {
    const uint64_t sig = ex ? (mx | (1ull << Ms)) : mx;
    const int eu = ex ? (int)ex - biasS - (int)Ms : 1 - biasS - (int)Ms;  // value = sig * 2^eu
    if (sig == 0ull) {
      code = 0ull;
    } else {
      const int p = 63 - __builtin_clzll(sig) + eu;  // value in [2^p, 2^(p+1))
      int shift;
      uint64_t base;
      const bool normal = p >= 1 - biasT;
      if (normal) {  // target normal: quantum 2^(p - M)
        shift = p - (int)M - eu;
        base = (uint64_t)(p + biasT - 1) << M;  // plus the significand with its hidden bit
      } else {  // target subnormal: quantum 2^(1 - biasT - M)
        shift = 1 - biasT - (int)M - eu;
        base = 0ull;
      }
      uint64_t kept, rem = 0ull, half = 0ull;
      if (shift >= 64) {
        kept = 0ull;
        rem = sig;
        half = ~0ull;  // below half a quantum: never rounds up
      } else {
        kept = sig >> shift;
        rem = sig & low_mask64((uint32_t)shift);
        half = shift ? (1ull << (shift - 1)) : 0ull;
      }
      code = base + kept;
      if (rne && shift > 0) {
        // the significand's last bit: a normal's hidden bit when M = 0
        const uint64_t odd = (normal && M == 0u) ? 1ull : (code & 1ull);
        if (rem > half || (rem == half && odd && half != ~0ull)) code += 1ull;
      }
      if (code >= ((uint64_t)emaxT << M)) code = (uint64_t)emaxT << M;  // overflow: Inf
    }
  }
  return code | (sign << (E + M));
}

// Float bits of format (E, M) -> format (Et, Mt) with Et >= E, Mt >= M,
// exactly; with `quiet` a NaN also gets its quiet bit.
__device__ uint64_t gen_widen(uint64_t c, uint32_t E, uint32_t M, uint32_t Et, uint32_t Mt, bool quiet) {
  const uint64_t sign = (c >> (E + M)) & 1ull;
  const uint32_t emax = (1u << E) - 1u, emaxT = (1u << Et) - 1u;
  const uint32_t e = (uint32_t)((c >> M) & emax);
  const uint64_t m = c & low_mask64(M);
  const int bias = (1 << (E - 1)) - 1, biasT = (1 << (Et - 1)) - 1;
  uint64_t r;
  if (e == emax) {
    r = ((uint64_t)emaxT << Mt) | (m << (Mt - M));
    if (quiet && m) r |= 1ull << (Mt - 1u);
  } else if (e) {
    r = ((uint64_t)(e - bias + biasT) << Mt) | (m << (Mt - M));
  } else if (m == 0ull) {
    r = 0ull;
  } else {
    const int p = 63 - __builtin_clzll(m);
    const int u = 1 - bias - (int)M + p;  // unbiased exponent of the value
    if (u >= 1 - biasT) r = ((uint64_t)(u + biasT) << Mt) | ((m ^ (1ull << p)) << (Mt - p));
    else r = m << (Mt - M + (uint32_t)(biasT - bias));
  }
  return r | (sign << (Et + Mt));
}

__device__ __forceinline__ void gen_float_fmt(uint32_t t, uint32_t& E, uint32_t& M) {
  switch (t) {
    case LLAMA_F16: E = 5; M = 10; return;
    case LLAMA_BF16: E = 8; M = 7; return;
    case LLAMA_F32: E = 8; M = 23; return;
    default: E = 11; M = 52; return;
  }
}

__device__ __forceinline__ bool gen_is_float(uint32_t t) {
  return t == LLAMA_F32 || t == LLAMA_F64 || t == LLAMA_F16 || t == LLAMA_BF16;
}

__device__ __forceinline__ uint32_t gen_bytes(uint32_t t) {
  switch (t) {
    case LLAMA_I8: case LLAMA_U8: return 1;
    case LLAMA_I16: case LLAMA_U16: case LLAMA_F16: case LLAMA_BF16: return 2;
    case LLAMA_F32: case LLAMA_I32: case LLAMA_U32: return 4;
    default: return 8;
  }
}

__device__ __forceinline__ bool gen_signed(uint32_t t) {
  return t == LLAMA_I8 || t == LLAMA_I16 || t == LLAMA_I32 || t == LLAMA_I64;
}

// ChangeType conversion of one value (the conversions a ChangeType mapping
// applies on load and on store): floats narrow by round to nearest even and
// widen exactly, NaNs quiet; integers keep the low bits or extend by the
// source's signedness.
__device__ uint64_t gen_convert(uint64_t v, uint32_t from, uint32_t to) {
  if (from == to) return v;
  if (gen_is_float(from)) {
    uint32_t Es, Ms, Ed, Md;
    gen_float_fmt(from, Es, Ms);
    gen_float_fmt(to, Ed, Md);
    if (Ed >= Es && Md >= Ms) return gen_widen(v, Es, Ms, Ed, Md, true);
    return gen_narrow(v, Es, Ms, Ed, Md, true);
  }
  const uint32_t wf = 8u * gen_bytes(from), wt = 8u * gen_bytes(to);
  uint64_t x = v & low_mask64(wf);
  if (wt > wf && gen_signed(from) && ((x >> (wf - 1u)) & 1ull)) x |= ~low_mask64(wf);
  return x & low_mask64(wt);
}

// B bits at stream bit `bit` (B <= 64: at most three words)
__device__ __forceinline__ uint64_t gen_read_bits(const uint8_t* stream, uint64_t bit, uint32_t B) {
  const uint32_t* w = (const uint32_t*)stream + (bit >> 5);
  const uint32_t sh = (uint32_t)(bit & 31u);
  const uint32_t nw = (sh + B + 31u) >> 5;
  unsigned __int128 acc = 0;
  for (uint32_t k = 0; k < nw; ++k) acc |= (unsigned __int128)w[k] << (32u * k);
  return (uint64_t)(acc >> sh) & low_mask64(B);
}

__device__ __forceinline__ uint64_t gen_load(const GenSide& s, const GenArgs& a, uint64_t i, uint32_t f) {
  const uint32_t ut = a.user_t[f];
  switch (s.kind[f]) {
    case GK_NULL: return 0ull;
    case GK_PHYS: return mix_load(s.m, i, f, (uint32_t)__builtin_ctz(gen_bytes(ut)));
    case GK_CONV: {
      const uint32_t st = s.stored_t[f];
      return gen_convert(mix_load(s.m, i, f, (uint32_t)__builtin_ctz(gen_bytes(st))), st, ut);
    }
    case GK_BITS_INT: {
      const uint32_t B = s.bits[f];
      const uint64_t c = gen_read_bits(s.m.col[s.m.cidx[f]], i * B, B);
      uint64_t v = c;
      if (gen_signed(ut) && B < 64u && ((c >> (B - 1u)) & 1ull)) v |= ~low_mask64(B);
      return v & low_mask64(8u * gen_bytes(ut));
    }
    default: {  // GK_BITS_FLOAT
      const uint32_t B = s.bits[f];
      const uint64_t c = gen_read_bits(s.m.col[s.m.cidx[f]], i * B, B);
      uint32_t Et, Mt;
      gen_float_fmt(ut, Et, Mt);
      return gen_widen(c, s.E[f], s.M[f], Et, Mt, false);
    }
  }
}

__device__ __forceinline__ uint64_t gen_encode(const GenSide& d, const GenArgs& a, uint64_t v, uint32_t f) {
  if (d.kind[f] == GK_BITS_INT) return v & low_mask64(d.bits[f]);
  uint32_t Et, Mt;
  gen_float_fmt(a.user_t[f], Et, Mt);
  return gen_narrow(v, Et, Mt, d.E[f], d.M[f], d.rne[f] != 0u);
}

__device__ __forceinline__ void gen_store(const GenSide& d, const GenArgs& a, uint64_t i, uint32_t f, uint64_t v) {
  const uint32_t ut = a.user_t[f];
  if (d.kind[f] == GK_PHYS) {
    mix_store(d.m, i, f, (uint32_t)__builtin_ctz(gen_bytes(ut)), v);
  } else {  // GK_CONV
    const uint32_t st = d.stored_t[f];
    mix_store(d.m, i, f, (uint32_t)__builtin_ctz(gen_bytes(st)), gen_convert(v, ut, st));
  }
}

__global__ __launch_bounds__(kThreads) void k_generic(GenArgs a) {
  const uint64_t groups = (a.n + 31u) >> 5;
  const uint64_t stride = (uint64_t)gridDim.x * kThreads;
  for (uint64_t g = (uint64_t)blockIdx.x * kThreads + threadIdx.x; g < groups; g += stride) {
    const uint64_t i0 = g * 32u;
    for (uint32_t f = 0; f < a.nf; ++f) {
      const uint32_t dk = a.dst.kind[f];
      if (dk == GK_NULL) continue;  // a NULL part of a SPLIT destination drops the values
      if (dk != GK_BITS_INT && dk != GK_BITS_FLOAT) {
        for (uint32_t k = 0; k < 32u && i0 + k < a.n; ++k) {
          const uint64_t i = i0 + k;
          gen_store(a.dst, a, i, f, gen_load(a.src, a, mix_src_index(a.order, i), f));
        }
        continue;
      }
      // 32 codes of B bits: the B words from word g * B on, written as they fill
      const uint32_t B = a.dst.bits[f];
      const uint64_t nw_stream = (a.n * B + 31u) >> 5;
      uint32_t* out = (uint32_t*)a.dst.m.col[a.dst.m.cidx[f]] + g * B;
      unsigned __int128 acc = 0;
      uint32_t have = 0, w = 0;
      for (uint32_t k = 0; k < 32u; ++k) {
        const uint64_t i = i0 + k;
        const uint64_t c = i < a.n ? gen_encode(a.dst, a, gen_load(a.src, a, mix_src_index(a.order, i), f), f) : 0ull;
        acc |= (unsigned __int128)c << have;
        have += B;
        while (have >= 32u) {
          if (g * B + w < nw_stream) out[w] = (uint32_t)acc;
          acc >>= 32;
          have -= 32u;
          ++w;
        }
      }
    }
  }
}

hipError_t launch_generic(const GenArgs& a, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(k_generic, dim3(grid), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace lm
