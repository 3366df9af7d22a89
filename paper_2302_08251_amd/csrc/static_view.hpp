// Views with compile-time array extents and stateless mappings for use inside
// kernels (LLAMA, arXiv 2302.08251, Sec. 2: array extents given partly or
// fully at compile time with a chosen index type; a view whose extents and
// mapping are all static stores nothing but its mapped bytes, so it is a
// trivial value type that can be placed in GPU shared memory; Sec. 3 Split
// and Null meta-mappings).
//
//   Extents<I, E...>   the extents (0 = dyn, a run-time extent stored in the
//                      object), index arithmetic in I (e.g. uint16_t)
//   AoS<Ext, F, T>     F leaves of type T, records back to back
//   SoA<Ext, F, T>     F planes of Ext::count leaves of type T
//   Null<Ext, F, T>    no bytes: loads give 0, stores are dropped
//   Split<MASK, A, B>  the leaves whose bit is set in MASK go through A (in
//                      record order), the others through B; A's bytes first
//   View<M>            exactly M::bytes bytes (static extents), loads and
//                      stores of leaf f of record i at compile-time offsets
#pragma once
#include <stdint.h>

#include <type_traits>

namespace lm {
namespace sv {

constexpr uint32_t dyn = 0;

template <typename I, uint32_t... E>
struct Extents {
  using index_type = I;
  static constexpr uint32_t rank = sizeof...(E);
  static constexpr bool all_static = ((E != 0) && ...);
  static constexpr uint32_t ext[rank] = {E...};
  // the run-time extents (only those given as dyn take a slot)
  static constexpr uint32_t ndyn = ((E == 0 ? 1u : 0u) + ...);
  I dyn_ext[ndyn > 0 ? ndyn : 1];

  __device__ __host__ constexpr I extent(uint32_t k) const {
    if (ext[k] != 0) return (I)ext[k];
    uint32_t slot = 0;
    for (uint32_t m = 0; m < k; ++m) slot += ext[m] == 0 ? 1u : 0u;
    return dyn_ext[slot];
  }
  // number of records (a compile-time constant when all extents are static)
  static constexpr I static_count() {
    I c = 1;
    for (uint32_t k = 0; k < rank; ++k) c = (I)(c * (I)ext[k]);
    return c;
  }
  __device__ __host__ constexpr I count() const {
    I c = 1;
    for (uint32_t k = 0; k < rank; ++k) c = (I)(c * extent(k));
    return c;
  }
  // row-major linear index of a multi-index, in the index type
  template <typename... A>
  __device__ __host__ constexpr I linear(A... a) const {
    static_assert(sizeof...(A) == rank, "one index per extent");
    const I idx[rank] = {(I)a...};
    I lin = 0;
    for (uint32_t k = 0; k < rank; ++k) lin = (I)(lin * extent(k) + idx[k]);
    return lin;
  }
};

template <typename Ext, uint32_t F, typename T>
struct AoS {
  using extents = Ext;
  using type = T;
  static constexpr uint32_t fields = F;
  static constexpr uint32_t bytes = (uint32_t)Ext::static_count() * F * sizeof(T);
  template <uint32_t f>
  __device__ __host__ static constexpr uint32_t offset(typename Ext::index_type i) {
    return ((uint32_t)i * F + f) * (uint32_t)sizeof(T);
  }
};

template <typename Ext, uint32_t F, typename T>
struct SoA {
  using extents = Ext;
  using type = T;
  static constexpr uint32_t fields = F;
  static constexpr uint32_t bytes = (uint32_t)Ext::static_count() * F * sizeof(T);
  template <uint32_t f>
  __device__ __host__ static constexpr uint32_t offset(typename Ext::index_type i) {
    return (f * (uint32_t)Ext::static_count() + (uint32_t)i) * (uint32_t)sizeof(T);
  }
};

template <typename Ext, uint32_t F, typename T>
struct Null {
  using extents = Ext;
  using type = T;
  static constexpr uint32_t fields = F;
  static constexpr uint32_t bytes = 0;
};

template <typename M> struct is_null : std::false_type {};
template <typename Ext, uint32_t F, typename T> struct is_null<Null<Ext, F, T>> : std::true_type {};

// number of set bits of m below bit f: the index of leaf f inside its part
constexpr uint32_t rank_below(uint64_t m, uint32_t f) {
  uint32_t r = 0;
  for (uint32_t k = 0; k < f; ++k) r += (m >> k) & 1u;
  return r;
}

template <uint64_t MASK, typename A, typename B>
struct Split {
  using extents = typename A::extents;
  using type = typename A::type;
  static constexpr uint32_t fields = A::fields + B::fields;
  static constexpr uint32_t bytes = A::bytes + B::bytes;
};

// Location of leaf f of a mapping: which stateless leaf mapping holds it, at
// which leaf index, after how many bytes of the view.
template <typename M, uint32_t f, uint32_t BASE = 0>
struct Locate {
  using leaf = M;
  static constexpr uint32_t index = f, base = BASE;
};
template <uint64_t MASK, typename A, typename B, uint32_t f, uint32_t BASE>
struct Locate<Split<MASK, A, B>, f, BASE> {
  static constexpr bool in_a = (MASK >> f) & 1u;
  using part = std::conditional_t<in_a, Locate<A, rank_below(MASK, f), BASE>,
                                  Locate<B, f - rank_below(MASK, f), BASE + A::bytes>>;
  using leaf = typename part::leaf;
  static constexpr uint32_t index = part::index, base = part::base;
};

// A view with static extents over its own storage: sizeof == M::bytes.
template <typename M>
struct View {
  using T = typename M::type;
  using I = typename M::extents::index_type;
  static_assert(M::extents::all_static, "an LDS-resident view needs static extents");
  static constexpr uint32_t count = (uint32_t)M::extents::static_count();
  alignas(16) uint8_t blob[M::bytes > 0 ? M::bytes : 1];

  template <uint32_t f>
  __device__ T load(I i) const {
    using L = Locate<M, f>;
    if constexpr (is_null<typename L::leaf>::value) return T(0);
    else return *(const T*)(blob + L::base + L::leaf::template offset<L::index>(i));
  }
  template <uint32_t f>
  __device__ void store(I i, T v) {
    using L = Locate<M, f>;
    if constexpr (!is_null<typename L::leaf>::value) *(T*)(blob + L::base + L::leaf::template offset<L::index>(i)) = v;
  }
};

}  // namespace sv
}  // namespace lm
