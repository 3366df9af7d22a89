// Host runtime: descriptor validation, blob sizing, views, copy planning
// and dispatch of the tile kernels.
#include "host.hpp"

#include <algorithm>
#include <cstdarg>
#include <cstring>

#include "kernels.hpp"

namespace lm {

static thread_local std::string g_error;

llama_status fail(llama_status s, const std::string& msg) {
  g_error = msg;
  return s;
}

void clear_error() { g_error.clear(); }

bool scalar_valid(int t) { return t >= LLAMA_F32 && t <= LLAMA_BF16; }

uint32_t scalar_size(llama_scalar t) {
  switch (t) {
    case LLAMA_I8: case LLAMA_U8: return 1;
    case LLAMA_I16: case LLAMA_U16: case LLAMA_F16: case LLAMA_BF16: return 2;
    case LLAMA_F32: case LLAMA_I32: case LLAMA_U32: return 4;
    case LLAMA_F64: case LLAMA_I64: case LLAMA_U64: return 8;
  }
  return 0;
}

bool scalar_is_float(llama_scalar t) {
  return t == LLAMA_F32 || t == LLAMA_F64 || t == LLAMA_F16 || t == LLAMA_BF16;
}

bool scalar_is_signed(llama_scalar t) {
  return t == LLAMA_I8 || t == LLAMA_I16 || t == LLAMA_I32 || t == LLAMA_I64;
}

static void float_bits(llama_scalar t, uint32_t& E, uint32_t& M) {
  switch (t) {
    case LLAMA_F16: E = 5; M = 10; return;
    case LLAMA_BF16: E = 8; M = 7; return;
    case LLAMA_F32: E = 8; M = 23; return;
    case LLAMA_F64: E = 11; M = 52; return;
    default: E = M = 0;
  }
}

static bool is_physical(llama_map_kind k) {
  return k == LLAMA_MAP_AOS || k == LLAMA_MAP_SOA_SB || k == LLAMA_MAP_SOA_MB || k == LLAMA_MAP_AOSOA;
}

static uint64_t packed_size(const Rec& r) {
  uint64_t s = 0;
  for (auto t : r) s += scalar_size(t);
  return s;
}

static uint64_t aligned_size(const Rec& r) {
  uint64_t o = 0, maxs = 1;
  for (auto t : r) {
    uint64_t s = scalar_size(t);
    o = (o + s - 1) / s * s + s;
    if (s > maxs) maxs = s;
  }
  return (o + maxs - 1) / maxs * maxs;
}

static Rec byte_record(const Rec& r) { return Rec(packed_size(r), LLAMA_U8); }

static const char* kind_name(int k) {
  static const char* names[] = {"AOS", "SOA_SB", "SOA_MB", "AOSOA", "BYTESPLIT", "CHANGETYPE",
                                "BITPACK_INT_SOA", "BITPACK_FLOAT_SOA", "NULL", "SPLIT",
                                "FIELD_ACCESS_COUNT", "HEATMAP"};
  return (k >= 0 && k < 12) ? names[k] : "?";
}

llama_status copy_mapping(const Rec& rec, const llama_mapping* map, MapDesc& out, int depth) {
  if (!map) return fail(LLAMA_ERR_INVALID_ARG, "mapping descriptor is NULL");
  if (depth > 8) return fail(LLAMA_ERR_INVALID_ARG, "mappings nested more than 8 deep");
  if ((int)map->kind < 0 || (int)map->kind > 11)
    return fail(LLAMA_ERR_INVALID_ARG, "unknown mapping kind " + std::to_string((int)map->kind));
  out.kind = map->kind;
  out.lanes = map->lanes;
  out.bits = map->bits;
  out.exp_bits = map->exp_bits;
  out.man_bits = map->man_bits;
  out.flags = map->flags;
  if (map->flags & ~(LLAMA_FLAG_AOS_PACKED | LLAMA_FLAG_ROUND_RNE | LLAMA_FLAG_COL_MAJOR))
    return fail(LLAMA_ERR_INVALID_ARG, "unknown mapping flags");
  if ((map->flags & LLAMA_FLAG_COL_MAJOR) && depth > 0)
    return fail(LLAMA_ERR_INVALID_ARG, "LLAMA_FLAG_COL_MAJOR applies to the outermost mapping of a view");
  if ((map->flags & LLAMA_FLAG_ROUND_RNE) && map->kind != LLAMA_MAP_BITPACK_FLOAT_SOA)
    return fail(LLAMA_ERR_INVALID_ARG, "LLAMA_FLAG_ROUND_RNE applies to BITPACK_FLOAT_SOA only");
  switch (map->kind) {
    case LLAMA_MAP_AOS:
    case LLAMA_MAP_SOA_SB:
    case LLAMA_MAP_SOA_MB:
      return LLAMA_OK;
    case LLAMA_MAP_AOSOA:
      if (map->lanes == 0) return fail(LLAMA_ERR_INVALID_ARG, "AOSOA needs lanes >= 1");
      return LLAMA_OK;
    case LLAMA_MAP_BYTESPLIT: {
      if (!map->inner) return fail(LLAMA_ERR_INVALID_ARG, "BYTESPLIT needs an inner mapping");
      if (!is_physical(map->inner->kind))
        return fail(LLAMA_ERR_INVALID_ARG, std::string("BYTESPLIT inner mapping must be AOS, SOA_SB, SOA_MB or AOSOA, got ") +
                                               kind_name(map->inner->kind));
      out.inner.reset(new MapDesc);
      return copy_mapping(byte_record(rec), map->inner, *out.inner, depth + 1);
    }
    case LLAMA_MAP_CHANGETYPE: {
      if (!map->stored_types) return fail(LLAMA_ERR_INVALID_ARG, "CHANGETYPE needs stored_types");
      if (!map->inner) return fail(LLAMA_ERR_INVALID_ARG, "CHANGETYPE needs an inner mapping");
      if (!is_physical(map->inner->kind) && map->inner->kind != LLAMA_MAP_BYTESPLIT)
        return fail(LLAMA_ERR_INVALID_ARG, "CHANGETYPE inner mapping must be physical or BYTESPLIT");
      out.stored.assign(map->stored_types, map->stored_types + rec.size());
      for (size_t f = 0; f < rec.size(); ++f) {
        if (!scalar_valid(out.stored[f])) return fail(LLAMA_ERR_INVALID_ARG, "invalid stored type");
        llama_scalar a = rec[f], b = out.stored[f];
        if (a == b) continue;
        if (scalar_is_float(a) != scalar_is_float(b))
          return fail(LLAMA_ERR_INVALID_ARG, "CHANGETYPE converts float to float or integer to integer only");
        if (scalar_is_float(a)) {
          uint32_t Ea, Ma, Eb, Mb;
          float_bits(a, Ea, Ma);
          float_bits(b, Eb, Mb);
          if (!((Eb >= Ea && Mb >= Ma) || (Eb <= Ea && Mb <= Ma)))
            return fail(LLAMA_ERR_INVALID_ARG, "CHANGETYPE between these float formats is neither widening nor narrowing");
        }
      }
      out.inner.reset(new MapDesc);
      return copy_mapping(out.stored, map->inner, *out.inner, depth + 1);
    }
    case LLAMA_MAP_BITPACK_INT_SOA:
      for (auto t : rec) {
        if (scalar_is_float(t)) return fail(LLAMA_ERR_INVALID_ARG, "BITPACK_INT_SOA needs integer fields");
        if (map->bits < 1 || map->bits > 8 * scalar_size(t))
          return fail(LLAMA_ERR_INVALID_ARG, "BITPACK_INT_SOA bits must be in [1, bit width of every field]");
      }
      return LLAMA_OK;
    case LLAMA_MAP_NULL:
      return LLAMA_OK;
    case LLAMA_MAP_SPLIT: {
      if (!map->inner) return fail(LLAMA_ERR_INVALID_ARG, "SPLIT needs inner: an array of two mappings");
      if (map->lanes < 1 || map->lanes >= rec.size())
        return fail(LLAMA_ERR_INVALID_ARG, "SPLIT needs 1 <= lanes < the number of fields");
      const Rec r0(rec.begin(), rec.begin() + map->lanes), r1(rec.begin() + map->lanes, rec.end());
      out.inner.reset(new MapDesc);
      out.inner2.reset(new MapDesc);
      llama_status st = copy_mapping(r0, &map->inner[0], *out.inner, depth + 1);
      if (st != LLAMA_OK) return st;
      return copy_mapping(r1, &map->inner[1], *out.inner2, depth + 1);
    }
    case LLAMA_MAP_FIELD_ACCESS_COUNT:
    case LLAMA_MAP_HEATMAP: {
      if (!map->inner) return fail(LLAMA_ERR_INVALID_ARG, std::string(kind_name(map->kind)) + " needs an inner mapping");
      const int ik = (int)map->inner->kind;
      if (map->kind == LLAMA_MAP_FIELD_ACCESS_COUNT && (ik < 0 || ik > (int)LLAMA_MAP_BITPACK_FLOAT_SOA))
        return fail(LLAMA_ERR_INVALID_ARG, "FIELD_ACCESS_COUNT instruments mappings of kinds 0-7");
      if (map->kind == LLAMA_MAP_HEATMAP) {
        if (!is_physical(map->inner->kind))
          return fail(LLAMA_ERR_INVALID_ARG, "HEATMAP instruments AOS, SOA_SB, SOA_MB or AOSOA");
        if (map->lanes < 1 || map->lanes > (1u << 20) || (map->lanes & (map->lanes - 1)))
          return fail(LLAMA_ERR_INVALID_ARG, "HEATMAP needs lanes = bytes per counter, a power of two in [1, 2^20]");
      }
      out.inner.reset(new MapDesc);
      return copy_mapping(rec, map->inner, *out.inner, depth + 1);
    }
    case LLAMA_MAP_BITPACK_FLOAT_SOA:
      for (auto t : rec) {
        if (!scalar_is_float(t)) return fail(LLAMA_ERR_INVALID_ARG, "BITPACK_FLOAT_SOA needs float fields");
        uint32_t E, M;
        float_bits(t, E, M);
        if (map->exp_bits < 2 || map->exp_bits > E || map->man_bits > M)
          return fail(LLAMA_ERR_INVALID_ARG,
                      "BITPACK_FLOAT_SOA needs 2 <= exp_bits <= E and man_bits <= M of every field type");
      }
      return LLAMA_OK;
  }
  return fail(LLAMA_ERR_INVALID_ARG, "unknown mapping kind");
}

static uint32_t code_bits(const MapDesc& m) {
  return m.kind == LLAMA_MAP_BITPACK_INT_SOA ? m.bits : 1 + m.exp_bits + m.man_bits;
}

uint32_t blob_count(const Rec& rec, const MapDesc& m) {
  switch (m.kind) {
    case LLAMA_MAP_AOS: case LLAMA_MAP_SOA_SB: case LLAMA_MAP_AOSOA: return 1;
    case LLAMA_MAP_SOA_MB: case LLAMA_MAP_BITPACK_INT_SOA: case LLAMA_MAP_BITPACK_FLOAT_SOA:
      return (uint32_t)rec.size();
    case LLAMA_MAP_BYTESPLIT: return blob_count(byte_record(rec), *m.inner);
    case LLAMA_MAP_CHANGETYPE: return blob_count(m.stored, *m.inner);
    case LLAMA_MAP_NULL: return 0;
    case LLAMA_MAP_SPLIT: {
      const Rec r0(rec.begin(), rec.begin() + m.lanes), r1(rec.begin() + m.lanes, rec.end());
      return blob_count(r0, *m.inner) + blob_count(r1, *m.inner2);
    }
    case LLAMA_MAP_FIELD_ACCESS_COUNT: return blob_count(rec, *m.inner) + 1;
    case LLAMA_MAP_HEATMAP: return 2 * blob_count(rec, *m.inner);
  }
  return 0;
}

uint64_t blob_size(const Rec& rec, const MapDesc& m, uint64_t n, uint32_t b) {
  switch (m.kind) {
    case LLAMA_MAP_AOS: return n * ((m.flags & LLAMA_FLAG_AOS_PACKED) ? packed_size(rec) : aligned_size(rec));
    case LLAMA_MAP_SOA_SB: return n * packed_size(rec);
    case LLAMA_MAP_SOA_MB: return n * scalar_size(rec[b]);
    case LLAMA_MAP_AOSOA: return (n + m.lanes - 1) / m.lanes * m.lanes * packed_size(rec);
    case LLAMA_MAP_BYTESPLIT: return blob_size(byte_record(rec), *m.inner, n, b);
    case LLAMA_MAP_CHANGETYPE: return blob_size(m.stored, *m.inner, n, b);
    case LLAMA_MAP_BITPACK_INT_SOA:
    case LLAMA_MAP_BITPACK_FLOAT_SOA: return 4 * ((n * code_bits(m) + 31) / 32);
    case LLAMA_MAP_NULL: return 0;
    case LLAMA_MAP_SPLIT: {
      const Rec r0(rec.begin(), rec.begin() + m.lanes), r1(rec.begin() + m.lanes, rec.end());
      const uint32_t c0 = blob_count(r0, *m.inner);
      return b < c0 ? blob_size(r0, *m.inner, n, b) : blob_size(r1, *m.inner2, n, b - c0);
    }
    case LLAMA_MAP_FIELD_ACCESS_COUNT: {
      const uint32_t c = blob_count(rec, *m.inner);
      return b < c ? blob_size(rec, *m.inner, n, b) : 16ull * rec.size();
    }
    case LLAMA_MAP_HEATMAP: {
      const uint32_t c = blob_count(rec, *m.inner);
      return b < c ? blob_size(rec, *m.inner, n, b) : 8 * ((blob_size(rec, *m.inner, n, b - c) + m.lanes - 1) / m.lanes);
    }
  }
  return 0;
}

uint64_t mapped_bytes(const Rec& rec, const MapDesc& m, uint64_t n) {
  switch (m.kind) {
    case LLAMA_MAP_AOS: case LLAMA_MAP_SOA_SB: case LLAMA_MAP_SOA_MB: case LLAMA_MAP_AOSOA:
      return n * packed_size(rec);
    case LLAMA_MAP_BYTESPLIT: return n * packed_size(rec);
    case LLAMA_MAP_CHANGETYPE: return n * packed_size(m.stored);
    case LLAMA_MAP_BITPACK_INT_SOA:
    case LLAMA_MAP_BITPACK_FLOAT_SOA: return rec.size() * ((n * code_bits(m) + 7) / 8);
    case LLAMA_MAP_NULL: return 0;
    case LLAMA_MAP_SPLIT: {
      const Rec r0(rec.begin(), rec.begin() + m.lanes), r1(rec.begin() + m.lanes, rec.end());
      return mapped_bytes(r0, *m.inner, n) + mapped_bytes(r1, *m.inner2, n);
    }
    case LLAMA_MAP_FIELD_ACCESS_COUNT:
    case LLAMA_MAP_HEATMAP: return mapped_bytes(rec, *m.inner, n);
  }
  return 0;
}

static llama_status read_record(const llama_record* r, Rec& out) {
  if (!r) return fail(LLAMA_ERR_INVALID_ARG, "record is NULL");
  if (r->n_fields < 1 || r->n_fields > kMaxFields)
    return fail(LLAMA_ERR_INVALID_ARG, "record needs 1..64 leaf fields");
  if (!r->types) return fail(LLAMA_ERR_INVALID_ARG, "record types are NULL");
  out.assign(r->types, r->types + r->n_fields);
  for (auto t : out)
    if (!scalar_valid(t)) return fail(LLAMA_ERR_INVALID_ARG, "invalid leaf type " + std::to_string((int)t));
  return LLAMA_OK;
}

static llama_status read_extents(uint32_t rank, const uint64_t* ext, uint64_t& n) {
  if (rank < 1 || rank > 8) return fail(LLAMA_ERR_INVALID_ARG, "rank must be 1..8");
  if (!ext) return fail(LLAMA_ERR_INVALID_ARG, "extents are NULL");
  n = 1;
  for (uint32_t d = 0; d < rank; ++d) {
    if (ext[d] != 0 && n > UINT64_MAX / ext[d])
      return fail(LLAMA_ERR_INDEX_OVERFLOW, "extents overflow 64 bits");
    n *= ext[d];
  }
  // keep byte sizes representable: n * (up to 512 bytes per record)
  if (n > (UINT64_MAX >> 10)) return fail(LLAMA_ERR_INDEX_OVERFLOW, "too many records");
  return LLAMA_OK;
}

static uint64_t index_max(llama_index_type t) {
  switch (t) {
    case LLAMA_IDX_I16: return 0x7FFFull;
    case LLAMA_IDX_U16: return 0xFFFFull;
    case LLAMA_IDX_I32: return 0x7FFFFFFFull;
    case LLAMA_IDX_U32: return 0xFFFFFFFFull;
    case LLAMA_IDX_I64: return 0x7FFFFFFFFFFFFFFFull;
    case LLAMA_IDX_U64: return UINT64_MAX;
  }
  return 0;
}

Div make_div(uint32_t d) {
  Div r{};
  r.d = d ? d : 1;
  if ((r.d & (r.d - 1)) == 0) {
    r.pow2 = 1;
    r.sh = (uint32_t)__builtin_ctz(r.d);
    r.m = 0;
  } else {
    r.pow2 = 0;
    r.sh = 0;
    r.m = (uint32_t)(((1ull << 32) + r.d - 1) / r.d);
  }
  return r;
}

static uint32_t log2u(uint32_t x) { return (uint32_t)__builtin_ctz(x); }

// Structural description of a physical mapping (possibly a Bytesplit)
// over a storage record of uniform element size `es`.
static llama_status physical_side(const MapDesc& m, uint32_t nf, uint32_t es, Side& s) {
  const MapDesc* p = &m;
  uint32_t cs = es, ncols = nf;
  if (m.kind == LLAMA_MAP_BYTESPLIT) {
    p = m.inner.get();
    // Bytesplit over AoS places byte k of field f at i*S + p_f + k: the
    // packed AoS byte image itself, so it is moved as an AoS of elements
    if (p->kind != LLAMA_MAP_AOS) {
      cs = 1;
      ncols = nf * es;
    }
  }
  s.cs = cs;
  s.log2cs = log2u(cs);
  s.ncols = ncols;
  s.rec_bytes = ncols * cs;
  s.mb = 0;
  s.lanes = 1;
  switch (p->kind) {
    case LLAMA_MAP_AOS: s.layout = LY_AOS; break;
    case LLAMA_MAP_SOA_SB: s.layout = LY_PLANAR; break;
    case LLAMA_MAP_SOA_MB:
      s.layout = LY_PLANAR;
      s.mb = 1;
      if (ncols > kMaxCols) return fail(LLAMA_ERR_UNSUPPORTED, "more than 64 blobs in one view");
      break;
    case LLAMA_MAP_AOSOA:
      s.layout = LY_AOSOA;
      s.lanes = p->lanes;
      break;
    default: return fail(LLAMA_ERR_UNSUPPORTED, "unsupported inner mapping");
  }
  return LLAMA_OK;
}

static llama_status uniform_type(const Rec& r, llama_scalar& t, bool same_type, const char* what) {
  t = r[0];
  for (auto x : r) {
    if (scalar_size(x) != scalar_size(t))
      return fail(LLAMA_ERR_UNSUPPORTED, std::string("the GPU tile engine needs leaves of equal size (") + what + ")");
    if (same_type && x != t)
      return fail(LLAMA_ERR_UNSUPPORTED, std::string("the GPU path needs leaves of one type (") + what + ")");
  }
  return LLAMA_OK;
}

llama_status make_side(const llama_view* v, Side& s, llama_scalar& user_t, llama_scalar& stored_t) {
  std::memset(&s, 0, sizeof(s));
  const MapDesc& m = v->map;
  const uint32_t nf = (uint32_t)v->rec.size();
  llama_status st;
  const bool need_same = m.kind == LLAMA_MAP_CHANGETYPE || m.kind == LLAMA_MAP_BITPACK_INT_SOA ||
                         m.kind == LLAMA_MAP_BITPACK_FLOAT_SOA;
  if ((st = uniform_type(v->rec, user_t, need_same, "record")) != LLAMA_OK) return st;
  stored_t = user_t;
  s.vkind = VK_RAW;
  s.n = v->n;
  s.n_mod16 = (uint32_t)(v->n & 15u);
  switch (m.kind) {
    case LLAMA_MAP_AOS: case LLAMA_MAP_SOA_SB: case LLAMA_MAP_SOA_MB: case LLAMA_MAP_AOSOA:
    case LLAMA_MAP_BYTESPLIT:
      if ((st = physical_side(m, nf, scalar_size(user_t), s)) != LLAMA_OK) return st;
      s.es = scalar_size(user_t);
      break;
    case LLAMA_MAP_CHANGETYPE:
      if ((st = uniform_type(m.stored, stored_t, true, "stored types")) != LLAMA_OK) return st;
      if ((st = physical_side(*m.inner, nf, scalar_size(stored_t), s)) != LLAMA_OK) return st;
      s.es = scalar_size(stored_t);
      s.vkind = stored_t == user_t ? VK_RAW : VK_CONV;
      break;
    case LLAMA_MAP_BITPACK_INT_SOA:
    case LLAMA_MAP_BITPACK_FLOAT_SOA:
      if (m.kind == LLAMA_MAP_BITPACK_FLOAT_SOA && user_t != LLAMA_F32 && user_t != LLAMA_F64)
        return fail(LLAMA_ERR_UNSUPPORTED, "the tile kernels pack f32 and f64 floats only");
      s.layout = LY_STREAM;
      s.vkind = m.kind == LLAMA_MAP_BITPACK_INT_SOA ? VK_INT : VK_FLOAT;
      s.bits = code_bits(m);
      s.exp_bits = m.exp_bits;
      s.man_bits = m.man_bits;
      s.rne = (m.flags & LLAMA_FLAG_ROUND_RNE) ? 1u : 0u;
      s.is_signed = scalar_is_signed(user_t);
      s.ncols = nf;
      s.cs = 4;
      s.log2cs = 2;
      s.es = scalar_size(user_t);
      if (s.bits > 32) return fail(LLAMA_ERR_UNSUPPORTED, "the GPU path packs codes of at most 32 bits");
      if (nf > kMaxCols) return fail(LLAMA_ERR_UNSUPPORTED, "more than 64 blobs in one view");
      break;
    default:  // NULL and SPLIT are resolved before a copy reaches the tile engine
      return fail(LLAMA_ERR_UNSUPPORTED, std::string("no tile-engine side for a ") + kind_name(m.kind) + " view");
  }
  s.blob_size = v->blob_bytes.empty() ? 0 : v->blob_bytes[0];
  for (size_t b = 0; b < v->blobs.size() && b < kMaxCols; ++b) s.blob[b] = v->blobs[b];
  s.div_S = make_div(s.rec_bytes);
  s.div_L = make_div(s.lanes);
  s.div_LS = make_div(s.lanes * s.rec_bytes);
  s.div_Lcs = make_div(s.lanes * s.cs);
  s.div_B = make_div(s.bits ? s.bits : 1);
  return LLAMA_OK;
}

static uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

static uint64_t lcm64(uint64_t a, uint64_t b) { return a / gcd64(a, b) * b; }

uint64_t tile_granule(const Side& s, const Side& d) {
  uint64_t g = 128;
  if (s.layout == LY_AOSOA) g = lcm64(g, s.lanes);
  if (d.layout == LY_AOSOA) g = lcm64(g, d.lanes);
  return g;
}

uint32_t tile_lds_bytes(const Side& s, uint32_t tile) {
  switch (s.layout) {
    case LY_AOS: case LY_AOSOA: return tile * s.rec_bytes;
    case LY_PLANAR: return s.ncols * (tile * s.cs + 16u);
    default: return s.ncols * (tile * s.bits / 8u + 16u);
  }
}

static uint32_t lds_stride(const Side& s, uint32_t tile) {
  if (s.layout == LY_PLANAR) return tile * s.cs + 16u;
  if (s.layout == LY_STREAM) return tile * s.bits / 8u + 16u;
  return 0;
}

static Codec codec_of(llama_scalar t) {
  switch (t) {
    case LLAMA_U8: return CD_U8;
    case LLAMA_I8: return CD_I8;
    case LLAMA_U16: return CD_U16;
    case LLAMA_I16: return CD_I16;
    case LLAMA_U32: return CD_U32;
    case LLAMA_I32: return CD_I32;
    case LLAMA_U64: return CD_U64;
    case LLAMA_I64: return CD_I64;
    case LLAMA_F32: return CD_F32;
    default: return CD_F64;
  }
}

// The planar path of pack: planes of 32-bit integers (SoA single- or
// multi-blob, or AoS / AoSoA of one field) into BitPackedIntSoA streams of
// the code widths it serves better than the tile kernels (measured on 256 Mi
// values: B <= 27 and not a multiple of 8, 5.7-6.1 TB/s against 4.6-5.7 for
// the tile kernels' word image with LDS atomics; from B = 28 the word image
// is 2-4 % ahead).  False: the tile kernels pack.
static bool plan_pack_planar(const llama_view* src, const llama_view* dst, Plan& plan) {
  const MapDesc& sm = src->map;
  const MapDesc& dm = dst->map;
  const uint32_t F = (uint32_t)src->rec.size();
  const llama_scalar t = src->rec[0];
  if (dm.kind != LLAMA_MAP_BITPACK_INT_SOA || (t != LLAMA_I32 && t != LLAMA_U32) || F > kMaxCols) return false;
  for (llama_scalar x : src->rec)
    if (x != t) return false;
  const uint32_t B = code_bits(dm);
  if (B % 8 == 0 || B > 27) return false;
  PlanarPackArgs& a = plan.pp;
  a = PlanarPackArgs{};
  const uint64_t n = src->n;
  for (uint32_t f = 0; f < F; ++f) {
    const uint8_t* b0 = (const uint8_t*)src->blobs[0];
    switch (sm.kind) {
      case LLAMA_MAP_SOA_MB: a.src[f] = (const uint8_t*)src->blobs[f]; break;
      case LLAMA_MAP_SOA_SB:
        if (n % 4u) return false;  // planes on the 16-byte grid
        a.src[f] = b0 + 4u * n * f;
        break;
      case LLAMA_MAP_AOS: case LLAMA_MAP_AOSOA:
        if (F != 1) return false;
        a.src[f] = b0;
        break;
      default: return false;
    }
    a.dst[f] = (uint8_t*)dst->blobs[f];
  }
  a.n = n;
  a.nf = F;
  a.bits = B;
  plan.kind = PK_PACK_PLANAR;
  plan.unit = 4;
  // one wave per chunk of 2048 values, one workgroup per four chunks
  const uint64_t chunks = (n + 2047u) / 2048u * F;
  plan.ntiles = chunks;
  plan.grid = (uint32_t)std::min<uint64_t>((chunks + 3u) / 4u, 1u << 30);
  plan.alg_bytes = mapped_bytes(src->rec, src->map, src->n) + mapped_bytes(dst->rec, dst->map, dst->n);
  return true;
}

llama_status plan_copy(const llama_view* src, const llama_view* dst, const llama_launch_params* p,
                       Plan& plan, uint32_t lds_cap, bool fill) {
  if (!src || !dst) return fail(LLAMA_ERR_INVALID_ARG, "view is NULL");
  if (src->rec != dst->rec) return fail(LLAMA_ERR_RECORD_MISMATCH, "source and destination records differ");
  if (src->n != dst->n) return fail(LLAMA_ERR_RECORD_MISMATCH, "source and destination record counts differ");
  plan = Plan{};
  llama_status st;
  llama_scalar su, ss, du, ds;
  Side& S = plan.args.src;
  Side& D = plan.args.dst;
  if ((st = make_side(src, S, su, ss)) != LLAMA_OK) return st;
  if ((st = make_side(dst, D, du, ds)) != LLAMA_OK) return st;
  const bool sstream = S.layout == LY_STREAM, dstream = D.layout == LY_STREAM;
  if (sstream && dstream) return fail(LLAMA_ERR_UNSUPPORTED, "copy between two bit-packed views");
  if (dstream) {
    if (S.vkind != VK_RAW) return fail(LLAMA_ERR_UNSUPPORTED, "pack needs a physical source");
    // explicit launch parameters address the tile kernels
    if ((!p || (p->tile_records == 0 && p->grid == 0)) && plan_pack_planar(src, dst, plan)) return LLAMA_OK;
    plan.kind = PK_PACK;
    plan.unit = 4;
    plan.args.codec = codec_of(su);
  } else if (sstream) {
    if (D.vkind != VK_RAW) return fail(LLAMA_ERR_UNSUPPORTED, "unpack needs a physical destination");
    plan.kind = PK_UNPACK;
    plan.unit = D.cs;
    plan.args.codec = codec_of(su);
  } else if (S.vkind == VK_RAW && D.vkind == VK_RAW) {
    plan.kind = PK_RAW;
    plan.unit = S.es;  // leaf bytes
    plan.args.mode = S.cs == D.cs ? RM_DIRECT : (S.cs == 1 ? RM_MERGE : RM_SPLIT);
    // fused relayout: the destination keeps runs of 4 records per column.
    // Planar destinations always qualify (the kernels adapt to a plane
    // start off the dword / 16-byte grid); AoSoA needs runs that stay
    // aligned to the store width in every block.
    if (plan.args.mode == RM_SPLIT) {
      const bool ok = D.layout == LY_PLANAR || (D.layout == LY_AOSOA && D.lanes % 4 == 0);
      if (ok) plan.args.mode = RM_SPLIT_FUSED;
    } else if (plan.args.mode == RM_MERGE) {
      const uint64_t A = D.es >= 4 ? 16 : 4 * D.es;  // store width of 4 elements (up to 16 bytes)
      const bool ok = D.layout == LY_PLANAR ||
                      (D.layout == LY_AOSOA && D.lanes % 4 == 0 && ((uint64_t)D.lanes * D.rec_bytes) % A == 0 &&
                       ((uint64_t)D.lanes * D.es) % A == 0);
      if (ok) plan.args.mode = RM_MERGE_FUSED;
    }
  } else if (S.vkind == VK_CONV && D.vkind == VK_CONV) {
    return fail(LLAMA_ERR_UNSUPPORTED, "copy between two ChangeType views with conversions");
  } else {
    const llama_scalar from = S.vkind == VK_CONV ? ss : su;
    const llama_scalar to = D.vkind == VK_CONV ? ds : du;
    plan.kind = PK_CONV;
    plan.unit = D.cs;
    struct Pair { llama_scalar from, to; Conv cv; };
    static const Pair pairs[] = {
        {LLAMA_F64, LLAMA_F32, CV_F64_F32},   {LLAMA_F32, LLAMA_F64, CV_F32_F64},
        {LLAMA_F32, LLAMA_F16, CV_F32_F16},   {LLAMA_F32, LLAMA_BF16, CV_F32_BF16},
        {LLAMA_F64, LLAMA_F16, CV_F64_F16},   {LLAMA_F64, LLAMA_BF16, CV_F64_BF16},
        {LLAMA_F16, LLAMA_F32, CV_F16_F32},   {LLAMA_BF16, LLAMA_F32, CV_BF16_F32},
        {LLAMA_F16, LLAMA_F64, CV_F16_F64},   {LLAMA_BF16, LLAMA_F64, CV_BF16_F64},
    };
    plan.args.conv = CV_NONE;
    for (const Pair& q : pairs)
      if (q.from == from && q.to == to) plan.args.conv = q.cv;
    if (plan.args.conv == CV_NONE)
      return fail(LLAMA_ERR_UNSUPPORTED, "the GPU path converts between the float types f64, f32, f16 and bf16 only");
  }
  // Single-blob destination planes off the 128-byte line grid: line-owner
  // writes (every line written whole by one tile), with a halo of the
  // records that fill the tile's last line of each plane
  if (plan.kind == PK_RAW && D.layout == LY_PLANAR && !D.mb && D.ncols > 1 && ((D.n * D.cs) & 127u) != 0)
    plan.args.mode = RM_LINE;
  const uint32_t mode = plan.kind == PK_RAW ? plan.args.mode : RM_DIRECT;
  const bool line = mode == RM_LINE;
  const uint64_t halo = line ? 128u / D.cs : 0u;
  // records of LDS past the tile: the halo, in whole source AoSoA blocks and
  // in multiples of 16 records (so that every LDS plane stays 16-byte aligned)
  const uint64_t hq = S.layout == LY_AOSOA ? lcm64(16, S.lanes) : 16u;
  const uint64_t halo_lds = line ? (halo + hq - 1u) / hq * hq : 0u;
  const bool canonical = mode == RM_MERGE || mode == RM_SPLIT;
  // canonical planar image of a relayout: element planes (MERGE) or byte planes (SPLIT)
  const uint32_t F = (uint32_t)src->rec.size(), ES = S.es;
  auto can_bytes = [&](uint64_t t) -> uint64_t {
    if (mode == RM_MERGE) return (uint64_t)F * (t * ES + 16u);
    if (mode == RM_SPLIT) return (uint64_t)F * ES * (t + 16u);
    return 0;
  };
  // A Bytesplit source merged into an AoS destination is merged in place over
  // the source image when every thread can hold its (quad, field) items in
  // registers: one LDS image instead of two.
  const bool merge_aos = canonical && mode == RM_MERGE && D.layout == LY_AOS;
  auto in_place = [&](uint64_t t) {
    return merge_aos && (t / 4u) * F <= (uint64_t)merge_in_place_items(ES) * kThreads;
  };
  // pack: the tile's stream-word image (t * B / 8 bytes per field), unless
  // every field's codes go from registers straight to the stream (planes of
  // 4-byte values whose tile runs start on the 16-byte grid, B a multiple of 8)
  const bool pack = plan.kind == PK_PACK;
  const bool pack_direct = pack && S.layout == LY_PLANAR && S.cs == 4 && S.es == 4 && (S.mb || (S.n & 3u) == 0) &&
                           (D.bits & 7u) == 0;
  auto lds_total = [&](uint64_t t) -> uint64_t {
    // line-owner copies build the destination's runs in registers from the
    // tile's source image (and halo), the only LDS image (+16: a misaligned
    // byte-column read fetches the dword after the last plane)
    if (line) return tile_lds_bytes(S, (uint32_t)(t + halo_lds)) + 16u;
    const uint64_t a = tile_lds_bytes(S, (uint32_t)t);
    if (pack_direct) return a;
    if (pack) return ((a + 15u) & ~15ull) + (uint64_t)D.ncols * (t * D.bits / 8u);
    if (in_place(t)) return a;
    return canonical ? ((a + 15u) & ~15ull) + can_bytes(t) : a;
  };
  const uint64_t gran = tile_granule(S, D);
  // bytes of one destination tile segment set: the destination inverse
  // divides offsets below tile * S by up to L * S, exact while that product
  // stays below 2^32, i.e. tile * S <= 65536
  const uint64_t dst_bytes = D.layout == LY_STREAM ? 0 : (uint64_t)D.rec_bytes;
  uint64_t tile = p && p->tile_records ? p->tile_records : 0;
  if (tile) {
    if (tile % gran) return fail(LLAMA_ERR_INVALID_ARG, "tile_records must be a multiple of " + std::to_string(gran));
  } else {
    // about 16 KiB per tile image on the larger side (32 KiB with two images).
    // Byte planes (a planar Bytesplit side) need longer tiles to fill whole
    // 1 KiB wave groups: about 30 KiB with one such side, 24 KiB with two.
    // Pack holds the source tile and its stream-word image in LDS: about
    // 24 KiB in all.  Unpack writes its (larger) output from registers:
    // about 8 KiB of stream words, up to a 16 KiB output tile.
    const bool bs = S.layout == LY_PLANAR && S.cs == 1, bd = D.layout == LY_PLANAR && D.cs == 1;
    // AoS to AoS (a straight 16-byte copy through LDS) is fastest with short
    // tiles: about 7 KiB.
    const bool aos2aos = plan.kind == PK_RAW && mode == RM_DIRECT && S.layout == LY_AOS && D.layout == LY_AOS;
    const bool unpack = plan.kind == PK_UNPACK;
    // direct packs: 16 KiB, 24 KiB for 8-bit codes (measured on 256 Mi
    // values: 4096 beat 6144 by 2-6 % at B = 16, 24, 32; 6144 beat 4096 by
    // 20 % at B = 8).  Word-image packs: about 32 KiB with the image, see below.
    const uint64_t target = pack_direct ? (D.bits == 8 ? 24576 : 16384) : pack ? 32768
                            : line ? (D.cs == 1 && S.cs > 1 ? 32768 : 24576)  // the tile and its halo
                            : unpack ? 8192
                            // ChangeType: 32 KiB on the wider side; f32 -> f16 / bf16
                            // 16 KiB (measured on planes: 4096 values beat 8192 by 5-8 %)
                            : plan.kind == PK_CONV ? (S.es == 4 && D.es == 2 ? 16384 : 32768)
                            : aos2aos ? 7168
                            : merge_aos ? 16384  // one image, merged in place
                            : canonical ? 32768
                            : (bs && bd) ? 24576
                            : (bs || bd) ? 30720
                                         : 16384;
    uint64_t per = plan.kind == PK_UNPACK ? lds_total(gran) : std::max<uint64_t>(lds_total(gran), gran * dst_bytes);
    uint64_t k = per ? (target / per) : 1;
    if (k < 1) k = 1;
    const uint64_t dst_cap = unpack ? 16384 : 65536;
    while (k > 1 && (gran * k > 65536 || gran * k * dst_bytes > dst_cap)) --k;
    // a word-image pack above 32000 bytes of LDS runs one workgroup fewer per
    // CU: three quarters of the tile then (measured at B = 31 on one plane:
    // 3072 values 5.8 TB/s, 4096 values 5.2)
    if (pack && !pack_direct && k > 1 && lds_total(gran * k) > 32000) k = k * 3u / 4u;
    if (line) {
      // A wave writes 63 windows of 16 bytes of one destination column per
      // step (16 / cs records each; the tile and its halo, plus one window).
      // Take the tile within the LDS target whose windows fill their wave
      // steps best, weighed by the share of the loads the halo adds
      // (measured for the split: 768 records, 57 windows, beat 512 by
      // 15-20 % and 1024, whose second step is nearly empty, by 50 %).
      const uint64_t R = 16u / D.cs;
      double best = -1.0;
      uint64_t bk = 1;
      for (uint64_t kk = 1; gran * kk <= 4096; ++kk) {
        const uint64_t t = gran * kk;
        if ((kk > 1 && lds_total(t) > target) || lds_total(t) > kMaxTileLds || t * dst_bytes > 65536) break;
        const uint64_t wins = (t + halo + R - 1u) / R + 1u;
        const uint64_t steps = (wins + 62u) / 63u;
        const double score = (double)wins / (63.0 * (double)steps) * (double)t / (double)(t + halo);
        if (score > best + 1e-9) {
          best = score;
          bk = kk;
        }
      }
      k = bk;
    }
    while (lds_cap && k > 1 && lds_total(gran * k) > lds_cap) --k;
    if (fill && lds_cap && !line) {  // grow the tile to the largest one within the cap (line tiles keep their size)
      while (gran * (k + 1) <= 65536 && lds_total(gran * (k + 1)) <= lds_cap &&
             gran * (k + 1) * dst_bytes <= 65536)
        ++k;
    }
    // Byte planes (a planar Bytesplit side) move in whole 1 KiB wave groups
    // when a tile has 1024 or 512 records.  Measured best: 1024 when both
    // sides are byte planes, for the in-place merge into AoS, for the merge
    // into one blob per element plane (SoA-MB: +4-6 % over 512) and for the
    // fused split from planar and AoSoA sources (+2.5-3.3 % timed alone; in a
    // sequence of copies +1.5-2 % from AoSoA, level from planes); 512 for the
    // fused split from AoS (level), the merge into AoSoA (level) and into
    // single-blob planes (1024 measured from -3 % to +4.5 %).
    if (plan.kind == PK_RAW && !lds_cap && (bs || bd) && !line) {
      const bool split_multi = plan.args.mode == RM_SPLIT_FUSED && S.layout != LY_AOS;
      const uint64_t want =
          ((bs && bd) || merge_aos || (bs && D.layout == LY_PLANAR && D.mb) || split_multi) ? 1024 : 512;
      uint64_t kp = std::max<uint64_t>(1, want / gran);
      while (kp > 1 && (lds_total(gran * kp) > kMaxTileLds || (merge_aos && !in_place(gran * kp)) ||
                        gran * kp * dst_bytes > 65536))
        --kp;
      if (!merge_aos || in_place(gran * kp)) k = kp;
    }
    tile = gran * k;
  }
  if (tile > 65536) return fail(LLAMA_ERR_INVALID_ARG, "tile_records must be <= 65536");
  const uint64_t lds = lds_total(tile);
  if (lds > kMaxTileLds)
    return fail(tile == gran ? LLAMA_ERR_UNSUPPORTED : LLAMA_ERR_INVALID_ARG,
                "a tile of " + std::to_string(tile) + " records needs " + std::to_string(lds) +
                    " bytes of LDS (limit 65536); reduce the tile or the AoSoA lane count");
  if (tile * dst_bytes > 65536)
    return fail(tile == gran ? LLAMA_ERR_UNSUPPORTED : LLAMA_ERR_INVALID_ARG,
                "a destination tile of " + std::to_string(tile) + " records spans more than 65536 bytes");
  S.lds_stride = lds_stride(S, (uint32_t)(tile + halo_lds));
  D.lds_stride = lds_stride(D, (uint32_t)tile);
  plan.args.halo = (uint32_t)halo;
  if (plan.kind == PK_RAW) {
    // destination chunks are 16-byte runs of one column when the mapping
    // keeps consecutive records of a column together
    auto runs = [](const Side& x) {
      return x.layout == LY_PLANAR || (x.layout == LY_AOSOA && (x.lanes * x.cs) % 16u == 0u);
    };
    Geo& g = plan.args.can;
    std::memset(&g, 0, sizeof(g));
    if (mode == RM_DIRECT) {
      plan.args.colrun = (runs(D) && runs(S)) || (D.layout == LY_AOS && S.layout == LY_AOS);
    } else if (canonical && mode == RM_MERGE && D.layout == LY_AOS) {
      // merged straight into the destination's AoS record image
      plan.args.colrun = 1;
      g.layout = LY_AOS;
      g.cs = ES;
      g.log2cs = log2u(ES);
      g.ncols = F;
      g.rec_bytes = F * ES;
      g.lanes = 1;
      g.div_L = make_div(F);  // the relayout's (quad, field) split
      // offset 0: merged in place over the source image
      plan.args.can_off = in_place(tile) ? 0u : (uint32_t)((tile_lds_bytes(S, (uint32_t)tile) + 15u) & ~15u);
    } else if (canonical) {
      plan.args.colrun = runs(D);
      g.layout = LY_PLANAR;
      g.cs = mode == RM_MERGE ? ES : 1u;
      g.log2cs = log2u(g.cs);
      g.ncols = mode == RM_MERGE ? F : F * ES;
      g.rec_bytes = F * ES;
      g.lanes = 1;
      // the canonical planes take the destination planes' start phase
      // (mod 16), so that Phase B moves aligned 16-byte chunks
      g.mb = D.layout == LY_PLANAR ? D.mb : 1u;
      g.n_mod16 = D.n_mod16;
      g.lds_stride = (uint32_t)(tile * g.cs + 16u);
      g.div_L = make_div(1);
      plan.args.can_off = (uint32_t)((tile_lds_bytes(S, (uint32_t)tile) + 15u) & ~15u);
    }
  }
  // can_off 0: no word image (every field stored directly)
  if (pack && !pack_direct) plan.args.can_off = (uint32_t)((tile_lds_bytes(S, (uint32_t)tile) + 15u) & ~15u);
  plan.args.tile = (uint32_t)tile;
  plan.ntiles = (src->n + tile - 1) / tile;
  if (plan.ntiles > 0xFFFFFFFFull) return fail(LLAMA_ERR_INDEX_OVERFLOW, "too many tiles");
  plan.args.ntiles_lo = (uint32_t)plan.ntiles;
  plan.grid = (p && p->grid) ? (uint32_t)(p->grid < plan.ntiles ? p->grid : plan.ntiles) : (uint32_t)plan.ntiles;
  plan.lds = (uint32_t)((lds + 15u) & ~15ull);  // whole 16-byte units: funnel-shift reads may touch the last one
  plan.alg_bytes = mapped_bytes(src->rec, src->map, src->n) + mapped_bytes(dst->rec, dst->map, dst->n);
  return LLAMA_OK;
}

llama_status plan_zero(const llama_view* dst, Plan& plan) {
  plan = Plan{};
  Side& D = plan.args.dst;
  llama_scalar du, ds;
  llama_status st = make_side(dst, D, du, ds);
  if (st != LLAMA_OK) return st;
  plan.kind = PK_ZERO;
  plan.unit = D.layout == LY_STREAM ? 4u : D.cs;
  plan.args.src = D;  // record count only
  const uint64_t gran = tile_granule(D, D);
  const uint64_t per = D.layout == LY_STREAM ? 0 : gran * D.rec_bytes;
  uint64_t k = per ? 16384 / per : 32;
  if (k < 1) k = 1;
  while (k > 1 && gran * k * (D.layout == LY_STREAM ? 0 : D.rec_bytes) > 65536) --k;
  const uint64_t tile = gran * k;
  plan.args.tile = (uint32_t)tile;
  plan.ntiles = (dst->n + tile - 1) / tile;
  if (plan.ntiles > 0xFFFFFFFFull) return fail(LLAMA_ERR_INDEX_OVERFLOW, "too many tiles");
  plan.args.ntiles_lo = (uint32_t)plan.ntiles;
  plan.grid = (uint32_t)plan.ntiles;
  plan.lds = 0;
  plan.alg_bytes = mapped_bytes(dst->rec, dst->map, dst->n);
  return LLAMA_OK;
}

bool orders_differ(const llama_view* a, const llama_view* b) {
  if (a->col_major == b->col_major) return false;
  uint32_t big = 0;  // extents above 1: with at most one, both orders coincide
  for (uint32_t d = 0; d < a->rank; ++d) big += a->extents[d] > 1 ? 1u : 0u;
  return big > 1;
}

llama_status plan_xpose(const llama_view* src, const llama_view* dst, Plan& plan) {
  plan = Plan{};
  Side& S = plan.xa.src;
  Side& D = plan.xa.dst;
  llama_scalar su, ss, du, ds;
  llama_status st;
  if ((st = make_side(src, S, su, ss)) != LLAMA_OK) return st;
  if ((st = make_side(dst, D, du, ds)) != LLAMA_OK) return st;
  if (S.vkind != VK_RAW || D.vkind != VK_RAW)
    return fail(LLAMA_ERR_UNSUPPORTED,
                "a copy between views of different linearisation orders moves physical mappings only");
  if (S.rec_bytes != D.rec_bytes) return fail(LLAMA_ERR_RECORD_MISMATCH, "stored record sizes differ");
  // unit extents do not change either linearisation: drop them
  uint64_t e[8];
  uint32_t r = 0;
  for (uint32_t d = 0; d < src->rank; ++d)
    if (src->extents[d] > 1) e[r++] = src->extents[d];
  // strides of every axis in each order (records)
  auto strides = [&](bool col, uint64_t* out) {
    uint64_t acc = 1;
    if (col) {
      for (uint32_t k = 0; k < r; ++k) { out[k] = acc; acc *= e[k]; }
    } else {
      for (int k = (int)r - 1; k >= 0; --k) { out[k] = acc; acc *= e[k]; }
    }
  };
  uint64_t ss_[8], ds_[8];
  strides(src->col_major, ss_);
  strides(dst->col_major, ds_);
  const uint32_t P = dst->col_major ? 0u : r - 1u;  // the destination's fastest axis
  const uint32_t Q = src->col_major ? 0u : r - 1u;  // the source's fastest axis
  XposeArgs& a = plan.xa;
  a.eP = e[P];
  a.eQ = e[Q];
  a.sP = ss_[P];
  a.dQ = ds_[Q];
  a.nmid = 0;
  for (uint32_t k = 0; k < r; ++k) {
    if (k == P || k == Q) continue;
    a.mext[a.nmid] = e[k];
    a.msrc[a.nmid] = ss_[k];
    a.mdst[a.nmid] = ds_[k];
    ++a.nmid;
  }
  const uint32_t U = std::min(S.cs, D.cs);
  a.nunits = S.rec_bytes / U;
  a.div_units = make_div(a.nunits);
  // T x T records of the LDS image ([unit][q][p], rows of T + 1 units)
  a.T = 32;
  while (a.T > 4 && (uint64_t)S.rec_bytes * a.T * (a.T + 1) > kMaxTileLds) a.T >>= 1;
  a.log2T = log2u(a.T);
  a.src_rec_major = S.layout == LY_AOS ? 1u : 0u;
  a.dst_rec_major = D.layout == LY_AOS ? 1u : 0u;
  auto lmag = [](const Side& x) -> uint64_t {
    if (x.layout != LY_AOSOA || (x.lanes & (x.lanes - 1)) == 0) return 0;
    return ~0ull / x.lanes + 1ull;  // ceil(2^64 / L) for L not a power of two
  };
  a.src_lmag = lmag(S);
  a.dst_lmag = lmag(D);
  a.nPt = (a.eP + a.T - 1) / a.T;
  a.nQt = (a.eQ + a.T - 1) / a.T;
  uint64_t M = 1;
  for (uint32_t k = 0; k < a.nmid; ++k) M *= a.mext[k];
  a.ntiles = M * a.nPt * a.nQt;
  plan.kind = PK_XPOSE;
  plan.unit = U;
  plan.ntiles = a.ntiles;
  plan.grid = (uint32_t)std::min<uint64_t>(a.ntiles, 1u << 20);
  plan.lds = (uint32_t)(((uint64_t)S.rec_bytes * a.T * (a.T + 1) + 15u) & ~15ull);
  plan.alg_bytes = mapped_bytes(src->rec, src->map, src->n) + mapped_bytes(dst->rec, dst->map, dst->n);
  return LLAMA_OK;
}

// ---------------------------------------------------------------- per-leaf copies

bool mixed_record(const Rec& r) {
  for (auto t : r)
    if (scalar_size(t) != scalar_size(r[0])) return true;
  return false;
}

// Adds the groups of mapping `m` over leaves [f0, f0 + rec.size()) whose blobs
// are blobs[0 ..): a SPLIT adds one per part, an instrumented mapping its
// inner mapping's, a physical mapping or NULL one group.
static llama_status mix_flatten(const Rec& rec, const MapDesc& m, uint64_t n, void* const* blobs, uint32_t f0,
                                MixSide& s, uint32_t& ng, uint32_t& ncol) {
  const uint32_t nf = (uint32_t)rec.size();
  switch (m.kind) {
    case LLAMA_MAP_SPLIT: {
      const Rec r0(rec.begin(), rec.begin() + m.lanes), r1(rec.begin() + m.lanes, rec.end());
      llama_status st = mix_flatten(r0, *m.inner, n, blobs, f0, s, ng, ncol);
      if (st != LLAMA_OK) return st;
      return mix_flatten(r1, *m.inner2, n, blobs + blob_count(r0, *m.inner), f0 + m.lanes, s, ng, ncol);
    }
    case LLAMA_MAP_FIELD_ACCESS_COUNT:
    case LLAMA_MAP_HEATMAP:
      return mix_flatten(rec, *m.inner, n, blobs, f0, s, ng, ncol);
    default:
      break;
  }
  if (ng >= kMaxGroups) return fail(LLAMA_ERR_UNSUPPORTED, "more than 8 mappings in one SPLIT tree");
  MixGroup& g = s.g[ng];
  g = MixGroup{};
  g.log2L = 64;
  const MapDesc* p = &m;
  bool bytes = false;
  if (m.kind == LLAMA_MAP_BYTESPLIT) {
    p = m.inner.get();
    // over AoS the byte record's image is the packed AoS image of the leaves
    bytes = p->kind != LLAMA_MAP_AOS;
    if (!is_physical(p->kind)) return fail(LLAMA_ERR_UNSUPPORTED, "BYTESPLIT over a computed mapping");
  }
  if (m.kind == LLAMA_MAP_NULL) {
    g.kind = MX_NULL;
  } else if (!is_physical(p->kind)) {
    return fail(LLAMA_ERR_UNSUPPORTED, std::string("no per-leaf copy of a ") + kind_name(m.kind) + " view");
  } else {
    g.kind = bytes ? MX_BYTES : MX_ELEM;
  }
  const bool packed = m.kind == LLAMA_MAP_BYTESPLIT || (m.flags & LLAMA_FLAG_AOS_PACKED);
  const uint64_t P = packed_size(rec), S = (p->kind == LLAMA_MAP_AOS && !packed) ? aligned_size(rec) : P;
  switch (p->kind) {
    case LLAMA_MAP_AOS: g.L = 1; g.block = S; break;
    case LLAMA_MAP_AOSOA:
      g.L = p->lanes;
      g.block = (uint64_t)p->lanes * P;
      if ((p->lanes & (p->lanes - 1)) == 0) g.log2L = (uint32_t)__builtin_ctz(p->lanes);
      break;
    default: g.L = 0; break;  // SOA_SB, SOA_MB
  }
  uint64_t q = 0, po = 0;  // aligned and packed offsets of the leaf in the record
  for (uint32_t j = 0; j < nf; ++j) {
    const uint32_t f = f0 + j;
    const uint64_t sz = scalar_size(rec[j]);
    q = packed ? po : (q + sz - 1) / sz * sz;
    s.grp[f] = (uint8_t)ng;
    s.cidx[f] = (uint8_t)ncol;
    if (g.kind != MX_NULL) {
      const uint32_t cols = g.kind == MX_BYTES ? (uint32_t)sz : 1u;
      if (ncol + cols > kMaxCols) return fail(LLAMA_ERR_UNSUPPORTED, "more than 64 storage columns in one view");
      for (uint32_t k = 0; k < cols; ++k) {
        const uint8_t* b = (const uint8_t*)blobs[0];
        const uint64_t byte = po + k;  // byte column of a Bytesplit
        switch (p->kind) {
          case LLAMA_MAP_AOS: b += g.kind == MX_BYTES ? byte : q; break;
          case LLAMA_MAP_SOA_SB: b += n * (g.kind == MX_BYTES ? byte : po); break;
          case LLAMA_MAP_SOA_MB: b = (const uint8_t*)blobs[g.kind == MX_BYTES ? byte : j]; break;
          case LLAMA_MAP_AOSOA: b += (uint64_t)g.L * (g.kind == MX_BYTES ? byte : po); break;
          default: break;
        }
        s.col[ncol + k] = b;
      }
      if (g.kind == MX_ELEM && (uintptr_t)s.col[ncol] % sz == 0 && (g.L == 0 || g.block % sz == 0))
        s.elem_ok |= 1ull << f;
      ncol += cols;
    }
    q += sz;
    po += sz;
  }
  ++ng;
  return LLAMA_OK;
}

static void set_order(const llama_view* src, const llama_view* dst, Order& o) {
  o = Order{};
  if (!orders_differ(src, dst)) return;
  o.reorder = 1;
  o.rank = dst->rank;
  for (uint32_t d = 0; d < dst->rank; ++d) o.ext[d] = dst->extents[d];
  o.src_col_major = src->col_major ? 1u : 0u;
  o.dst_col_major = dst->col_major ? 1u : 0u;
}

static llama_status mix_side(const llama_view* v, MixSide& s) {
  std::memset(&s, 0, sizeof(s));
  uint32_t ng = 0, ncol = 0;
  return mix_flatten(v->rec, v->map, v->n, v->blobs.data(), 0, s, ng, ncol);
}

llama_status plan_mixed(const llama_view* src, const llama_view* dst, Plan& plan) {
  plan = Plan{};
  MixArgs& a = plan.ma;
  llama_status st;
  if ((st = mix_side(src, a.src)) != LLAMA_OK || (st = mix_side(dst, a.dst)) != LLAMA_OK) return st;
  const uint32_t nf = (uint32_t)dst->rec.size();
  a.n = dst->n;
  a.nf = nf;
  for (uint32_t f = 0; f < nf; ++f) a.lsz[f] = (uint8_t)__builtin_ctz(scalar_size(dst->rec[f]));
  set_order(src, dst, a.order);
  plan.kind = PK_MIXED;
  plan.ntiles = (dst->n + kThreads - 1) / kThreads;
  plan.grid = (uint32_t)std::min<uint64_t>(plan.ntiles, 1u << 16);
  plan.alg_bytes = mapped_bytes(src->rec, src->map, src->n) + mapped_bytes(dst->rec, dst->map, dst->n);
  return LLAMA_OK;
}

// ---------------------------------------------------------------- value-level copies

// Float pairs a ChangeType converts (widening or narrowing in both fields),
// or any two integer types.
static bool conversion_ok(llama_scalar a, llama_scalar b) {
  if (a == b) return true;
  if (scalar_is_float(a) != scalar_is_float(b)) return false;
  if (!scalar_is_float(a)) return true;
  uint32_t Ea, Ma, Eb, Mb;
  float_bits(a, Ea, Ma);
  float_bits(b, Eb, Mb);
  return (Eb >= Ea && Mb >= Ma) || (Eb <= Ea && Mb <= Ma);
}

// One side of a value-level copy: the kind of every leaf over the mapping
// tree (SPLIT parts, the mapping an instrumentation forwards to), physical
// parts flattened as for the per-leaf copy, one stream per bit-packed leaf.
static llama_status gen_flatten(const Rec& rec, const MapDesc& m, uint64_t n, void* const* blobs, uint32_t f0,
                                GenSide& s, uint32_t& ng, uint32_t& ncol) {
  const uint32_t nf = (uint32_t)rec.size();
  switch (m.kind) {
    case LLAMA_MAP_SPLIT: {
      const Rec r0(rec.begin(), rec.begin() + m.lanes), r1(rec.begin() + m.lanes, rec.end());
      llama_status st = gen_flatten(r0, *m.inner, n, blobs, f0, s, ng, ncol);
      if (st != LLAMA_OK) return st;
      return gen_flatten(r1, *m.inner2, n, blobs + blob_count(r0, *m.inner), f0 + m.lanes, s, ng, ncol);
    }
    case LLAMA_MAP_FIELD_ACCESS_COUNT:
    case LLAMA_MAP_HEATMAP:
      return gen_flatten(rec, *m.inner, n, blobs, f0, s, ng, ncol);
    case LLAMA_MAP_CHANGETYPE:
      for (uint32_t j = 0; j < nf; ++j) {
        if (!conversion_ok(rec[j], m.stored[j]))
          return fail(LLAMA_ERR_UNSUPPORTED, "ChangeType between these leaf types is not a conversion");
        s.kind[f0 + j] = GK_CONV;
        s.stored_t[f0 + j] = (uint8_t)m.stored[j];
      }
      return mix_flatten(m.stored, *m.inner, n, blobs, f0, s.m, ng, ncol);
    case LLAMA_MAP_BITPACK_INT_SOA:
    case LLAMA_MAP_BITPACK_FLOAT_SOA:
      if (ncol + nf > kMaxCols) return fail(LLAMA_ERR_UNSUPPORTED, "more than 64 storage columns in one view");
      for (uint32_t j = 0; j < nf; ++j) {
        const uint32_t f = f0 + j;
        s.kind[f] = m.kind == LLAMA_MAP_BITPACK_INT_SOA ? GK_BITS_INT : GK_BITS_FLOAT;
        s.bits[f] = (uint8_t)code_bits(m);  // at most the leaf's 64 bits
        s.E[f] = (uint8_t)m.exp_bits;
        s.M[f] = (uint8_t)m.man_bits;
        s.rne[f] = (m.flags & LLAMA_FLAG_ROUND_RNE) ? 1u : 0u;
        s.m.cidx[f] = (uint8_t)ncol;
        s.m.col[ncol++] = (const uint8_t*)blobs[j];
      }
      return LLAMA_OK;
    case LLAMA_MAP_NULL:
      for (uint32_t j = 0; j < nf; ++j) s.kind[f0 + j] = GK_NULL;
      return LLAMA_OK;
    default:  // physical, Bytesplit
      for (uint32_t j = 0; j < nf; ++j) s.kind[f0 + j] = GK_PHYS;
      return mix_flatten(rec, m, n, blobs, f0, s.m, ng, ncol);
  }
}

llama_status plan_generic(const llama_view* src, const llama_view* dst, Plan& plan) {
  plan = Plan{};
  GenArgs& a = plan.ga;
  llama_status st;
  uint32_t ng = 0, ncol = 0;
  if ((st = gen_flatten(src->rec, src->map, src->n, src->blobs.data(), 0, a.src, ng, ncol)) != LLAMA_OK) return st;
  ng = ncol = 0;
  if ((st = gen_flatten(dst->rec, dst->map, dst->n, dst->blobs.data(), 0, a.dst, ng, ncol)) != LLAMA_OK) return st;
  const uint32_t nf = (uint32_t)dst->rec.size();
  a.n = dst->n;
  a.nf = nf;
  for (uint32_t f = 0; f < nf; ++f) a.user_t[f] = (uint8_t)dst->rec[f];
  set_order(src, dst, a.order);
  plan.kind = PK_GENERIC;
  // one thread per 32 records
  plan.ntiles = ((dst->n + 31u) / 32u + kThreads - 1) / kThreads;
  plan.grid = (uint32_t)std::min<uint64_t>(plan.ntiles, 1u << 16);
  plan.alg_bytes = mapped_bytes(src->rec, src->map, src->n) + mapped_bytes(dst->rec, dst->map, dst->n);
  return LLAMA_OK;
}

llama_status launch_plan(const Plan& plan, hipStream_t st) {
  if (plan.ntiles == 0) return LLAMA_OK;
  hipError_t e = hipSuccess;
  switch (plan.kind) {
    case PK_RAW: e = launch_raw(plan.args, plan.unit, raw_variant(plan.args, plan.unit), plan.grid, plan.lds, st); break;
    case PK_CONV: e = launch_conv(plan.args, plan.unit, plan.grid, plan.lds, st); break;
    case PK_PACK: e = launch_pack(plan.args, plan.grid, plan.lds, st); break;
    case PK_ZERO: e = launch_zero(plan.args, plan.unit, plan.grid, st); break;
    case PK_UNPACK: e = launch_unpack(plan.args, plan.unit, plan.grid, plan.lds, st); break;
    case PK_XPOSE: e = launch_xpose(plan.xa, plan.unit, plan.grid, plan.lds, st); break;
    case PK_MIXED: e = launch_mixed(plan.ma, plan.grid, st); break;
    case PK_GENERIC: e = launch_generic(plan.ga, plan.grid, st); break;
    case PK_PACK_PLANAR: e = launch_pack_planar(plan.pp, plan.grid, st); break;
  }
  if (e != hipSuccess) return fail(LLAMA_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return LLAMA_OK;
}

static void clone_map(const MapDesc& a, MapDesc& b) {
  b.kind = a.kind;
  b.lanes = a.lanes;
  b.bits = a.bits;
  b.exp_bits = a.exp_bits;
  b.man_bits = a.man_bits;
  b.flags = a.flags;
  b.stored = a.stored;
  b.inner.reset();
  b.inner2.reset();
  if (a.inner) {
    b.inner.reset(new MapDesc);
    clone_map(*a.inner, *b.inner);
  }
  if (a.inner2) {
    b.inner2.reset(new MapDesc);
    clone_map(*a.inner2, *b.inner2);
  }
}

bool instrumented(const llama_view* v) {
  return v->map.kind == LLAMA_MAP_FIELD_ACCESS_COUNT || v->map.kind == LLAMA_MAP_HEATMAP;
}

// The view an instrumentation mapping forwards to: its inner mapping over the
// leading blobs.
void inner_view(const llama_view* v, llama_view& out) {
  out.rec = v->rec;
  clone_map(*v->map.inner, out.map);
  out.rank = v->rank;
  for (int d = 0; d < 8; ++d) out.extents[d] = v->extents[d];
  out.n = v->n;
  out.index_type = v->index_type;
  out.col_major = v->col_major;
  const size_t c = blob_count(v->rec, *v->map.inner);
  out.blobs.assign(v->blobs.begin(), v->blobs.begin() + c);
  out.blob_bytes.assign(v->blob_bytes.begin(), v->blob_bytes.begin() + c);
}

}  // namespace lm

using namespace lm;

extern "C" {

const char* llama_last_error(void) { return g_error.c_str(); }

const char* llama_version(void) { return "llama-mi 0.1 (gfx950)"; }

llama_status llama_mapping_blob_count(const llama_record* rec, const llama_mapping* map, uint32_t* n) {
  clear_error();
  Rec r;
  MapDesc m;
  llama_status st;
  if ((st = read_record(rec, r)) != LLAMA_OK) return st;
  if ((st = copy_mapping(r, map, m)) != LLAMA_OK) return st;
  if (!n) return fail(LLAMA_ERR_INVALID_ARG, "output pointer is NULL");
  *n = blob_count(r, m);
  return LLAMA_OK;
}

llama_status llama_mapping_blob_size(const llama_record* rec, const llama_mapping* map, uint32_t rank,
                                     const uint64_t* extents, uint32_t blob, uint64_t* bytes) {
  clear_error();
  Rec r;
  MapDesc m;
  uint64_t n;
  llama_status st;
  if ((st = read_record(rec, r)) != LLAMA_OK) return st;
  if ((st = copy_mapping(r, map, m)) != LLAMA_OK) return st;
  if ((st = read_extents(rank, extents, n)) != LLAMA_OK) return st;
  if (!bytes) return fail(LLAMA_ERR_INVALID_ARG, "output pointer is NULL");
  if (blob >= blob_count(r, m)) return fail(LLAMA_ERR_INVALID_ARG, "blob index out of range");
  *bytes = blob_size(r, m, n, blob);
  return LLAMA_OK;
}

llama_status llama_view_create(const llama_record* rec, const llama_mapping* map, uint32_t rank,
                               const uint64_t* extents, llama_index_type index_type, void* const* blobs,
                               const uint64_t* blob_bytes, uint32_t n_blobs, llama_view** out) {
  clear_error();
  if (!out) return fail(LLAMA_ERR_INVALID_ARG, "output pointer is NULL");
  *out = nullptr;
  std::unique_ptr<llama_view> v(new llama_view);
  llama_status st;
  if ((st = read_record(rec, v->rec)) != LLAMA_OK) return st;
  if ((st = copy_mapping(v->rec, map, v->map)) != LLAMA_OK) return st;
  if ((st = read_extents(rank, extents, v->n)) != LLAMA_OK) return st;
  v->rank = rank;
  for (uint32_t d = 0; d < rank; ++d) v->extents[d] = extents[d];
  v->col_major = (map->flags & LLAMA_FLAG_COL_MAJOR) != 0;
  if ((int)index_type < LLAMA_IDX_I16 || (int)index_type > LLAMA_IDX_U64)
    return fail(LLAMA_ERR_INVALID_ARG, "invalid index type");
  v->index_type = index_type;
  const uint64_t imax = index_max(index_type);
  if (v->n > 0 && v->n - 1 > imax)
    return fail(LLAMA_ERR_INDEX_OVERFLOW, "record count does not fit the index type");
  const uint32_t nb = blob_count(v->rec, v->map);
  if (n_blobs != nb)
    return fail(LLAMA_ERR_INVALID_ARG, "mapping uses " + std::to_string(nb) + " blobs, got " + std::to_string(n_blobs));
  if (nb > 0 && (!blobs || !blob_bytes)) return fail(LLAMA_ERR_INVALID_ARG, "blobs or blob_bytes is NULL");
  for (uint32_t b = 0; b < nb; ++b) {
    const uint64_t need = blob_size(v->rec, v->map, v->n, b);
    if (need > 0 && need - 1 > imax)
      return fail(LLAMA_ERR_INDEX_OVERFLOW, "blob " + std::to_string(b) + " of " + std::to_string(need) +
                                                " bytes does not fit the index type");
    if (need > 0 && !blobs[b]) return fail(LLAMA_ERR_INVALID_ARG, "blob " + std::to_string(b) + " is NULL");
    if (((uintptr_t)blobs[b]) & 15u)
      return fail(LLAMA_ERR_ALIGNMENT, "blob " + std::to_string(b) + " is not 16-byte aligned");
    if (blob_bytes[b] < need)
      return fail(LLAMA_ERR_NO_MEMORY, "blob " + std::to_string(b) + " has " + std::to_string(blob_bytes[b]) +
                                           " bytes, the mapping needs " + std::to_string(need));
    v->blobs.push_back(blobs[b]);
    v->blob_bytes.push_back(need);
  }
  *out = v.release();
  return LLAMA_OK;
}

llama_status llama_view_destroy(llama_view* view) {
  clear_error();
  delete view;
  return LLAMA_OK;
}

llama_status llama_view_records(const llama_view* view, uint64_t* n) {
  clear_error();
  if (!view || !n) return fail(LLAMA_ERR_INVALID_ARG, "NULL argument");
  *n = view->n;
  return LLAMA_OK;
}


// Part `part` (fields [0, k) or [k, F)) of a view that can be divided by
// fields: a SPLIT at k, SOA_MB (one blob per field) or NULL.
static bool part_view(const llama_view* v, uint32_t k, int part, llama_view& out) {
  const Rec& rec = v->rec;
  out.rec.assign(part ? rec.begin() + k : rec.begin(), part ? rec.end() : rec.begin() + k);
  out.rank = v->rank;
  for (int d = 0; d < 8; ++d) out.extents[d] = v->extents[d];
  out.n = v->n;
  out.index_type = v->index_type;
  out.col_major = v->col_major;
  out.blobs.clear();
  out.blob_bytes.clear();
  size_t b0 = 0, b1 = 0;
  if (v->map.kind == LLAMA_MAP_SPLIT) {
    if (v->map.lanes != k) return false;
    clone_map(part ? *v->map.inner2 : *v->map.inner, out.map);
    const Rec r0(rec.begin(), rec.begin() + k);
    const size_t c0 = blob_count(r0, *v->map.inner);
    b0 = part ? c0 : 0;
    b1 = part ? v->blobs.size() : c0;
  } else if (v->map.kind == LLAMA_MAP_SOA_MB) {
    out.map = MapDesc{};
    out.map.kind = LLAMA_MAP_SOA_MB;
    b0 = part ? k : 0;
    b1 = part ? rec.size() : k;
  } else if (v->map.kind == LLAMA_MAP_NULL) {
    out.map = MapDesc{};
    out.map.kind = LLAMA_MAP_NULL;
  } else {
    return false;
  }
  out.blobs.assign(v->blobs.begin() + b0, v->blobs.begin() + b1);
  out.blob_bytes.assign(v->blob_bytes.begin() + b0, v->blob_bytes.begin() + b1);
  return true;
}


static uint32_t log2u(uint64_t x) {
  uint32_t l = 0;
  while ((1ull << l) < x) ++l;
  return l;
}

// Heatmap geometry of inner blob b of a physical mapping.
static HeatGeo heat_geo(const Rec& rec, const MapDesc& m, uint64_t n, uint32_t b, uint32_t G) {
  HeatGeo g;
  g.n = n;
  g.shift = log2u(G);
  uint64_t p = 0, q = 0;
  switch (m.kind) {
    case LLAMA_MAP_AOS: {
      const bool packed = m.flags & LLAMA_FLAG_AOS_PACKED;
      g.period = packed ? packed_size(rec) : aligned_size(rec);
      g.recs = 1;
      for (size_t f = 0; f < rec.size(); ++f) {
        const uint64_t s = scalar_size(rec[f]);
        if (!packed) q = (q + s - 1) / s * s;
        g.run_off[f] = q;
        g.run_lsz[f] = log2u(s);
        q += s;
      }
      g.nruns = (uint32_t)rec.size();
      break;
    }
    case LLAMA_MAP_SOA_SB:
    case LLAMA_MAP_AOSOA: {
      const uint64_t R = m.kind == LLAMA_MAP_AOSOA ? m.lanes : n;
      g.period = R * packed_size(rec);
      g.recs = R;
      for (size_t f = 0; f < rec.size(); ++f) {
        g.run_off[f] = R * p;
        g.run_lsz[f] = log2u(scalar_size(rec[f]));
        p += scalar_size(rec[f]);
      }
      g.nruns = (uint32_t)rec.size();
      break;
    }
    case LLAMA_MAP_SOA_MB:
    default:
      g.period = n * scalar_size(rec[b]);
      g.recs = n;
      g.run_off[0] = 0;
      g.run_lsz[0] = log2u(scalar_size(rec[b]));
      g.nruns = 1;
      break;
  }
  return g;
}

// One launch of a copy.  A copy is planned whole before its first launch, so
// a pair that the kernels do not cover launches nothing.
struct CopyStep {
  enum Kind { DATA, FIELD_COUNT, HEAT } kind = DATA;
  Plan plan;                 // DATA
  void* counters = nullptr;  // FIELD_COUNT, HEAT
  uint32_t nf = 0, which = 0;
  uint64_t n = 0;            // FIELD_COUNT: records
  uint64_t ncounters = 0;    // HEAT
  HeatGeo geo;               // HEAT
};

// The counter updates of one copy on an instrumented view: every field of
// every record loaded once (source) or stored once (destination).
static void count_steps(const llama_view* v, bool store, std::vector<CopyStep>& steps) {
  if (v->n == 0) return;
  const uint32_t c = blob_count(v->rec, *v->map.inner);
  if (v->map.kind == LLAMA_MAP_FIELD_ACCESS_COUNT) {
    CopyStep s;
    s.kind = CopyStep::FIELD_COUNT;
    s.counters = v->blobs[c];
    s.nf = (uint32_t)v->rec.size();
    s.which = store ? 1u : 0u;
    s.n = v->n;
    steps.push_back(s);
    return;
  }
  for (uint32_t b = 0; b < c; ++b) {
    const uint64_t counters = v->blob_bytes[c + b] / 8;
    if (counters == 0) continue;
    CopyStep s;
    s.kind = CopyStep::HEAT;
    s.counters = v->blobs[c + b];
    s.ncounters = counters;
    s.geo = heat_geo(v->rec, *v->map.inner, v->n, b, v->map.lanes);
    steps.push_back(s);
  }
}

// The counter updates of the instrumented views inside a SPLIT tree.
static void count_parts(const llama_view* v, bool store, std::vector<CopyStep>& steps) {
  if (instrumented(v)) {
    count_steps(v, store, steps);
    return;
  }
  if (v->map.kind != LLAMA_MAP_SPLIT) return;
  for (int part = 0; part < 2; ++part) {
    llama_view pv;
    if (part_view(v, v->map.lanes, part, pv)) count_parts(&pv, store, steps);
  }
}

// Plans a copy with the meta-mappings resolved: an instrumented view forwards
// to its inner view and counts afterwards, a NULL destination drops the
// values, a NULL source writes zeros, a SPLIT on either side runs one copy
// per part.
// A pair the tile kernels or the per-leaf copy reject: the value-level copy
// if it takes the pair, else the first planner's reason stays the error.
static llama_status plan_generic_or_keep(const llama_view* src, const llama_view* dst, Plan& plan) {
  const std::string why = g_error;
  if (plan_generic(src, dst, plan) == LLAMA_OK) {
    clear_error();
    return LLAMA_OK;
  }
  g_error = why;
  return LLAMA_ERR_UNSUPPORTED;
}

static llama_status plan_views(const llama_view* src, const llama_view* dst, const llama_launch_params* params,
                               std::vector<CopyStep>& steps) {
  if (!src || !dst) return fail(LLAMA_ERR_INVALID_ARG, "view is NULL");
  if (src->rec != dst->rec) return fail(LLAMA_ERR_RECORD_MISMATCH, "source and destination records differ");
  if (src->n != dst->n) return fail(LLAMA_ERR_RECORD_MISMATCH, "source and destination record counts differ");
  if (orders_differ(src, dst)) {
    bool same = src->rank == dst->rank;
    for (uint32_t d = 0; same && d < src->rank; ++d) same = src->extents[d] == dst->extents[d];
    if (!same)
      return fail(LLAMA_ERR_RECORD_MISMATCH, "views linearised in different orders need the same extents");
  }
  if (instrumented(src) || instrumented(dst)) {
    llama_view is, id;
    if (instrumented(src)) inner_view(src, is);
    if (instrumented(dst)) inner_view(dst, id);
    llama_status s = plan_views(instrumented(src) ? &is : src, instrumented(dst) ? &id : dst, params, steps);
    if (s != LLAMA_OK) return s;
    if (instrumented(src)) count_steps(src, false, steps);
    if (instrumented(dst)) count_steps(dst, true, steps);
    return LLAMA_OK;
  }
  const bool ssplit = src->map.kind == LLAMA_MAP_SPLIT, dsplit = dst->map.kind == LLAMA_MAP_SPLIT;
  // A SPLIT source is divided before a NULL destination drops the values:
  // an instrumented part still counts the loads of its fields (Sec. 4).
  if (ssplit || dsplit) {
    const uint32_t k = ssplit ? src->map.lanes : dst->map.lanes;
    llama_view ps[2], pd[2];
    bool parts = true;
    for (int part = 0; part < 2; ++part) parts = parts && part_view(src, k, part, ps[part]) && part_view(dst, k, part, pd[part]);
    if (parts) {
      for (int part = 0; part < 2; ++part) {
        llama_status s = plan_views(&ps[part], &pd[part], params, steps);
        if (s != LLAMA_OK) return s;
      }
      return LLAMA_OK;
    }
    // any other partner: one per-leaf copy over both mapping trees (value by
    // value where a part is computed), then the counters of their
    // instrumented parts
    CopyStep step;
    llama_status s = plan_mixed(src, dst, step.plan);
    if (s == LLAMA_ERR_UNSUPPORTED) s = plan_generic_or_keep(src, dst, step.plan);
    if (s != LLAMA_OK) return s;
    steps.push_back(step);
    count_parts(src, false, steps);
    count_parts(dst, true, steps);
    return LLAMA_OK;
  }
  if (dst->map.kind == LLAMA_MAP_NULL) return LLAMA_OK;
  CopyStep step;
  llama_status s;
  if (mixed_record(dst->rec)) s = plan_mixed(src, dst, step.plan);  // leaves of several sizes
  else if (src->map.kind == LLAMA_MAP_NULL) s = plan_zero(dst, step.plan);  // zeros in any order
  else if (orders_differ(src, dst)) s = plan_xpose(src, dst, step.plan);
  else s = plan_copy(src, dst, params, step.plan);
  // what the tile kernels do not move (two computed views, integer
  // ChangeType, codes over 32 bits, ...) is copied value by value
  if (s == LLAMA_ERR_UNSUPPORTED) s = plan_generic_or_keep(src, dst, step.plan);
  if (s != LLAMA_OK) return s;
  steps.push_back(step);
  return LLAMA_OK;
}

static llama_status copy_views(const llama_view* src, llama_view* dst, const llama_launch_params* params,
                               hipStream_t st) {
  std::vector<CopyStep> steps;
  llama_status s = plan_views(src, dst, params, steps);
  if (s != LLAMA_OK) return s;
  int cus = 0;
  for (const CopyStep& step : steps) {
    switch (step.kind) {
      case CopyStep::DATA:
        if ((s = launch_plan(step.plan, st)) != LLAMA_OK) return s;
        break;
      case CopyStep::FIELD_COUNT:
        launch_field_count(step.counters, step.nf, step.which, step.n, st);
        break;
      case CopyStep::HEAT:
        if (cus <= 0) {
          int dev = 0;
          (void)hipGetDevice(&dev);
          if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        }
        launch_heatmap(step.counters, step.ncounters, step.geo, cus, st);
        break;
    }
  }
  return LLAMA_OK;
}

llama_status llama_copy_ex(const llama_view* src, llama_view* dst, const llama_launch_params* params,
                           void* stream) {
  clear_error();
  return copy_views(src, dst, params, (hipStream_t)stream);
}

llama_status llama_copy(const llama_view* src, llama_view* dst, void* stream) {
  return llama_copy_ex(src, dst, nullptr, stream);
}

static bool computed(const llama_view* v) {
  const llama_map_kind k = instrumented(v) ? v->map.inner->kind : v->map.kind;
  return k == LLAMA_MAP_CHANGETYPE || k == LLAMA_MAP_BITPACK_INT_SOA || k == LLAMA_MAP_BITPACK_FLOAT_SOA;
}

llama_status llama_pack(const llama_view* src, llama_view* dst, void* stream) {
  clear_error();
  if (!src || !dst) return fail(LLAMA_ERR_INVALID_ARG, "view is NULL");
  if (computed(src) || !computed(dst))
    return fail(LLAMA_ERR_UNSUPPORTED, "pack needs a physical source and a computed destination");
  return llama_copy_ex(src, dst, nullptr, stream);
}

llama_status llama_unpack(const llama_view* src, llama_view* dst, void* stream) {
  clear_error();
  if (!src || !dst) return fail(LLAMA_ERR_INVALID_ARG, "view is NULL");
  if (!computed(src) || computed(dst))
    return fail(LLAMA_ERR_UNSUPPORTED, "unpack needs a computed source and a physical destination");
  return llama_copy_ex(src, dst, nullptr, stream);
}

}  // extern "C"
