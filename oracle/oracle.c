/*
 * oracle.c - TEST INFRASTRUCTURE ONLY.
 *
 * Plain CPU definition of the LLAMA hot path (arXiv 2302.08251), written to
 * be checked by eye against the paper and the readings listed with it:
 * every copy is "for each record, for each leaf field: load the user value
 * through the source mapping, store it through the destination mapping",
 * and every load/store walks single bytes or single bits.  No tiling, no
 * vector tricks.  Only tests, the smoke check and the benchmark's CPU
 * baseline may call it.
 *
 * Readings where the paper is silent (the paper defines no mapping at the
 * byte or bit level; it names them in Sec. 3 and Sec. 5):
 *   - leaf fields are the record's leaves in declaration order;
 *   - AoS uses C-struct alignment unless packed; SoA single-blob puts the
 *     field planes back to back; SoA multi-blob uses blob f for field f;
 *   - AoSoA-L blocks hold L records field-major, the last block is padded;
 *   - Bytesplit byte k of a field is its k-th byte in memory (little-endian);
 *   - bit streams are LSB-first, one per field, tail bits zero;
 *   - float narrowing in ChangeType rounds to nearest even, bit-packed float
 *     encoding truncates toward zero, overflow gives Inf, NaN keeps its top
 *     payload bits and becomes quiet.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Scalar types                                                              */
/* ------------------------------------------------------------------------ */

EXPORT uint32_t orc_type_size(int t) {
  switch (t) {
    case ORC_I8: case ORC_U8: return 1;
    case ORC_I16: case ORC_U16: case ORC_F16: case ORC_BF16: return 2;
    case ORC_F32: case ORC_I32: case ORC_U32: return 4;
    case ORC_F64: case ORC_I64: case ORC_U64: return 8;
  }
  return 0;
}

static int is_float(int t) {
  return t == ORC_F32 || t == ORC_F64 || t == ORC_F16 || t == ORC_BF16;
}

static int is_signed_int(int t) {
  return t == ORC_I8 || t == ORC_I16 || t == ORC_I32 || t == ORC_I64;
}

/* IEEE-754 binary interchange formats: exponent and mantissa field widths. */
static void float_format(int t, uint32_t* E, uint32_t* M) {
  switch (t) {
    case ORC_F16: *E = 5; *M = 10; return;
    case ORC_BF16: *E = 8; *M = 7; return;
    case ORC_F32: *E = 8; *M = 23; return;
    case ORC_F64: *E = 11; *M = 52; return;
  }
  *E = 0; *M = 0;
}

static uint64_t low_mask(uint32_t bits) {
  return bits >= 64 ? ~0ull : ((1ull << bits) - 1ull);
}

/* ------------------------------------------------------------------------ */
/* IEEE binary-format conversions, written from the format definition:      */
/*   value = (-1)^s * 1.m * 2^(e - bias)   for 0 < e < all-ones              */
/*         = (-1)^s * 0.m * 2^(1 - bias)   for e = 0                          */
/*   e = all-ones: m = 0 is Inf, m != 0 is NaN.                               */
/* ------------------------------------------------------------------------ */

/* Narrow (Ed <= Es, Md <= Ms).  rne = 1: round to nearest, ties to even.
 * rne = 0: truncate toward zero.  Overflow gives Inf.  NaN: top Md payload
 * bits, quiet bit (mantissa MSB) forced; with Md = 0 a NaN becomes Inf. */
static uint64_t ieee_narrow(uint64_t bits, uint32_t Es, uint32_t Ms, uint32_t Ed, uint32_t Md,
                            int rne) {
  const uint64_t sign = (bits >> (Es + Ms)) & 1ull;
  const uint64_t e = (bits >> Ms) & low_mask(Es);
  const uint64_t m = bits & low_mask(Ms);
  const uint64_t emax_s = low_mask(Es), emax_d = low_mask(Ed);
  const int64_t bias_s = (int64_t)low_mask(Es - 1), bias_d = (int64_t)low_mask(Ed - 1);
  const uint64_t out_sign = sign << (Ed + Md);
  const uint64_t out_inf = out_sign | (emax_d << Md);

  if (e == emax_s) {
    if (m == 0) return out_inf;                      /* +-Inf stays Inf      */
    if (Md == 0) return out_inf;                     /* NaN has no room: Inf */
    return out_inf | (m >> (Ms - Md)) | (1ull << (Md - 1)); /* quiet NaN     */
  }
  if (e == 0 && m == 0) return out_sign;             /* +-0                  */

  /* significand (integer) and unbiased exponent of its leading position */
  uint64_t sig;
  int64_t u;
  int hidden;
  if (e == 0) { sig = m; u = 1 - bias_s; hidden = 0; }
  else { sig = m | (1ull << Ms); u = (int64_t)e - bias_s; hidden = 1; }

  if (hidden && u >= 1 - bias_d) {
    /* target normal: keep Md mantissa bits */
    uint32_t drop = Ms - Md;
    uint64_t q = sig >> drop; /* includes hidden bit at position Md */
    int64_t eo = u + bias_d;
    if (rne && drop > 0) {
      uint64_t rem = sig & low_mask(drop);
      uint64_t half = 1ull << (drop - 1);
      if (rem > half || (rem == half && (q & 1ull))) q += 1;
      if (q >> (Md + 1)) { q >>= 1; eo += 1; } /* mantissa carried out */
    }
    if (eo >= (int64_t)emax_d) return out_inf;       /* overflow -> Inf      */
    return out_sign | ((uint64_t)eo << Md) | (q & low_mask(Md));
  }

  /* target subnormal (or zero): quantum 2^(1 - bias_d - Md).
   * value = sig * 2^(u - Ms), so the code is sig / 2^d with: */
  int64_t d = (1 - bias_d) - u + (int64_t)Ms - (int64_t)Md;
  /* sig < 2^53, so for d >= 64 the value is below half the smallest
   * subnormal: both roundings give zero */
  if (d >= 64) return out_sign;
  uint64_t q = sig >> d;
  if (rne && d > 0) {
    uint64_t rem = sig & low_mask((uint32_t)d);
    uint64_t half = 1ull << (d - 1);
    if (rem > half || (rem == half && (q & 1ull))) q += 1;
  }
  /* q == 2^Md means the rounded value is the smallest normal: the bit
   * pattern (exponent 1, mantissa 0) is exactly q. */
  return out_sign | q;
}

/* Widen (Ed >= Es, Md >= Ms): exact.  NaN payload is shifted up; with
 * force_quiet the quiet bit of the result is set. */
static uint64_t ieee_widen(uint64_t bits, uint32_t Es, uint32_t Ms, uint32_t Ed, uint32_t Md,
                           int force_quiet) {
  const uint64_t sign = (bits >> (Es + Ms)) & 1ull;
  const uint64_t e = (bits >> Ms) & low_mask(Es);
  const uint64_t m = bits & low_mask(Ms);
  const uint64_t emax_s = low_mask(Es), emax_d = low_mask(Ed);
  const int64_t bias_s = (int64_t)low_mask(Es - 1), bias_d = (int64_t)low_mask(Ed - 1);
  const uint64_t out_sign = sign << (Ed + Md);

  if (e == emax_s) {
    uint64_t mo = m << (Md - Ms);
    if (m != 0 && force_quiet) mo |= 1ull << (Md - 1);
    return out_sign | (emax_d << Md) | mo;
  }
  if (e == 0 && m == 0) return out_sign;
  if (e == 0) {
    /* subnormal source: m * 2^(1 - bias_s - Ms); leading one at bit p */
    int p = 63;
    while (!((m >> p) & 1ull)) --p;
    int64_t u = 1 - bias_s - (int64_t)Ms + p;
    if (u >= 1 - bias_d) {
      uint64_t frac = m & low_mask((uint32_t)p);
      return out_sign | ((uint64_t)(u + bias_d) << Md) | (frac << (Md - (uint32_t)p));
    }
    /* still subnormal in the target: the value m * 2^(1 - bias_s - Ms) in
     * units of the target quantum 2^(1 - bias_d - Md) */
    return out_sign | (m << ((uint64_t)(bias_d - bias_s) + Md - Ms));
  }
  int64_t u = (int64_t)e - bias_s;
  return out_sign | ((uint64_t)(u + bias_d) << Md) | (m << (Md - Ms));
}

/* Value conversion between scalar types as ChangeType defines it. */
static uint64_t convert_value(uint64_t bits, int from, int to) {
  if (from == to) return bits;
  if (is_float(from) && is_float(to)) {
    uint32_t Es, Ms, Ed, Md;
    float_format(from, &Es, &Ms);
    float_format(to, &Ed, &Md);
    if (Ed >= Es && Md >= Ms) return ieee_widen(bits, Es, Ms, Ed, Md, 1);
    return ieee_narrow(bits, Es, Ms, Ed, Md, 1);
  }
  /* integers: narrowing keeps the low bits, widening extends by the source's
   * signedness */
  uint32_t wf = 8 * orc_type_size(from), wt = 8 * orc_type_size(to);
  uint64_t v = bits & low_mask(wf);
  if (wt > wf && is_signed_int(from) && ((v >> (wf - 1)) & 1ull)) v |= ~low_mask(wf);
  return v & low_mask(wt);
}

EXPORT int orc_conversion_supported(int from, int to) {
  if (from == to) return 1;
  if (is_float(from) && is_float(to)) {
    uint32_t Es, Ms, Ed, Md;
    float_format(from, &Es, &Ms);
    float_format(to, &Ed, &Md);
    return (Ed >= Es && Md >= Ms) || (Ed <= Es && Md <= Ms);
  }
  return !is_float(from) && !is_float(to);
}

EXPORT uint64_t orc_convert(uint64_t bits, int from, int to) { return convert_value(bits, from, to); }

/* BitPackedFloat code of a value of float type t (E <= E_t, M <= M_t).  The
 * mantissa is truncated (Sec. 3 leaves the rounding open); the _rne variant
 * rounds it to nearest, ties to even, the opt-in mode of the mapping. */
EXPORT uint64_t orc_float_encode(uint64_t bits, int t, uint32_t E, uint32_t M) {
  uint32_t Et, Mt;
  float_format(t, &Et, &Mt);
  return ieee_narrow(bits, Et, Mt, E, M, 0);
}

EXPORT uint64_t orc_float_encode_rne(uint64_t bits, int t, uint32_t E, uint32_t M) {
  uint32_t Et, Mt;
  float_format(t, &Et, &Mt);
  return ieee_narrow(bits, Et, Mt, E, M, 1);
}

EXPORT uint64_t orc_float_decode(uint64_t code, int t, uint32_t E, uint32_t M) {
  uint32_t Et, Mt;
  float_format(t, &Et, &Mt);
  return ieee_widen(code, E, M, Et, Mt, 0);
}

/* ------------------------------------------------------------------------ */
/* Record geometry                                                          */
/* ------------------------------------------------------------------------ */

static uint64_t packed_offset(const orc_rec* r, uint32_t f) {
  uint64_t o = 0;
  for (uint32_t g = 0; g < f; ++g) o += orc_type_size(r->types[g]);
  return o;
}

static uint64_t packed_size(const orc_rec* r) { return packed_offset(r, r->nf); }

static uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

/* C-struct placement: each field at the next multiple of its size. */
static uint64_t aligned_offset(const orc_rec* r, uint32_t f) {
  uint64_t o = 0;
  for (uint32_t g = 0; g < r->nf; ++g) {
    uint64_t s = orc_type_size(r->types[g]);
    o = align_up(o, s);
    if (g == f) return o;
    o += s;
  }
  return o;
}

static uint64_t aligned_size(const orc_rec* r) {
  uint64_t o = 0, maxs = 1;
  for (uint32_t g = 0; g < r->nf; ++g) {
    uint64_t s = orc_type_size(r->types[g]);
    o = align_up(o, s) + s;
    if (s > maxs) maxs = s;
  }
  return align_up(o, maxs);
}

/* The byte record a Bytesplit mapping forwards: one u8 field per byte. */
static const int g_bytes[4096] = {[0 ... 4095] = ORC_U8};

static orc_rec byte_record(const orc_rec* r) {
  orc_rec b = {(uint32_t)packed_size(r), g_bytes};
  return b;
}

static orc_rec stored_record(const orc_rec* r, const orc_map* m) {
  orc_rec s = {r->nf, m->stored_types};
  return s;
}

static uint32_t code_bits(const orc_map* m) {
  return m->kind == ORC_BITPACK_INT ? m->bits : 1 + m->exp_bits + m->man_bits;
}

/* ------------------------------------------------------------------------ */
/* Mapping: where does byte k of leaf f of record i live?                    */
/* ------------------------------------------------------------------------ */

/* Split (Sec. 3): fields [0, k) form the record of part 0 (mapping
 * inner[0]), fields [k, F) that of part 1 (inner[1]); the view's blobs are
 * part 0's followed by part 1's.  Null (Sec. 3) has no blobs: a load gives
 * zero, a store is dropped. */
static orc_rec split_part(const orc_rec* rec, const orc_map* m, int part) {
  orc_rec r;
  r.nf = part ? rec->nf - m->lanes : m->lanes;
  r.types = part ? rec->types + m->lanes : rec->types;
  return r;
}

EXPORT uint32_t orc_blob_count(const orc_rec* rec, const orc_map* m);
EXPORT uint64_t orc_blob_size(const orc_rec* rec, const orc_map* m, uint64_t n, uint32_t b);

/* Instrumentation (Sec. 4).  Both mappings forward every location, load and
 * store to the inner mapping and, as a side effect of each access, add one to
 * counters held in extra blobs placed after the inner mapping's blobs:
 *  - FieldAccessCount: one extra blob of 2F 64-bit counters; counter 2f counts
 *    the loads of field f and counter 2f+1 its stores;
 *  - Heatmap(G): one extra blob per inner blob b, holding one 64-bit counter
 *    per G bytes of b.  An access to a field adds one to every counter whose
 *    G bytes contain at least one byte of the field (loads and stores alike).
 * The increments are atomic, so the parallel copy below counts exactly. */
static void count_one(uint8_t* blob, uint64_t idx) {
  __atomic_fetch_add((uint64_t*)(blob + 8 * idx), (uint64_t)1, __ATOMIC_RELAXED);
}

EXPORT int orc_locate(const orc_rec* rec, const orc_map* m, uint64_t n, uint64_t i, uint32_t f,
                      uint32_t k, uint32_t* blob, uint64_t* off);

static void count_access(const orc_rec* rec, const orc_map* m, uint64_t n, uint8_t* const* blobs,
                         uint64_t i, uint32_t f, int is_store) {
  const uint32_t c = orc_blob_count(rec, m->inner);
  if (m->kind == ORC_FIELD_ACCESS_COUNT) {
    count_one(blobs[c], 2ull * f + (is_store ? 1 : 0));
    return;
  }
  /* Heatmap: the distinct (blob, counter) pairs over the field's bytes */
  uint32_t cb[8];
  uint64_t cg[8];
  uint32_t nc = 0;
  for (uint32_t k = 0; k < orc_type_size(rec->types[f]); ++k) {
    uint32_t b;
    uint64_t o;
    orc_locate(rec, m->inner, n, i, f, k, &b, &o);
    const uint64_t g = o / m->lanes;
    int seen = 0;
    for (uint32_t q = 0; q < nc; ++q) seen |= cb[q] == b && cg[q] == g;
    if (!seen) {
      cb[nc] = b;
      cg[nc] = g;
      ++nc;
    }
  }
  for (uint32_t q = 0; q < nc; ++q) count_one(blobs[c + cb[q]], cg[q]);
}

EXPORT int orc_locate(const orc_rec* rec, const orc_map* m, uint64_t n, uint64_t i, uint32_t f,
                      uint32_t k, uint32_t* blob, uint64_t* off) {
  const uint64_t s = orc_type_size(rec->types[f]);
  switch (m->kind) {
    case ORC_AOS: {
      uint64_t S = m->aos_packed ? packed_size(rec) : aligned_size(rec);
      uint64_t q = m->aos_packed ? packed_offset(rec, f) : aligned_offset(rec, f);
      *blob = 0;
      *off = i * S + q + k;
      return 0;
    }
    case ORC_SOA_SB:
      *blob = 0;
      *off = n * packed_offset(rec, f) + i * s + k;
      return 0;
    case ORC_SOA_MB:
      *blob = f;
      *off = i * s + k;
      return 0;
    case ORC_AOSOA: {
      uint64_t L = m->lanes, S = packed_size(rec);
      *blob = 0;
      *off = (i / L) * L * S + L * packed_offset(rec, f) + (i % L) * s + k;
      return 0;
    }
    case ORC_BYTESPLIT: {
      orc_rec br = byte_record(rec);
      return orc_locate(&br, m->inner, n, i, (uint32_t)(packed_offset(rec, f) + k), 0, blob, off);
    }
    case ORC_SPLIT: {
      const int part = f >= m->lanes;
      orc_rec pr = split_part(rec, m, part);
      if (!part) return orc_locate(&pr, &m->inner[0], n, i, f, k, blob, off);
      orc_rec p0 = split_part(rec, m, 0);
      int rc = orc_locate(&pr, &m->inner[1], n, i, f - m->lanes, k, blob, off);
      *blob += orc_blob_count(&p0, &m->inner[0]);
      return rc;
    }
    case ORC_FIELD_ACCESS_COUNT:
    case ORC_HEATMAP:
      return orc_locate(rec, m->inner, n, i, f, k, blob, off);
  }
  return -1;  /* Null and the computed mappings have no byte locations */
}

EXPORT uint32_t orc_blob_count(const orc_rec* rec, const orc_map* m) {
  switch (m->kind) {
    case ORC_AOS: case ORC_SOA_SB: case ORC_AOSOA: return 1;
    case ORC_SOA_MB: case ORC_BITPACK_INT: case ORC_BITPACK_FLOAT: return rec->nf;
    case ORC_BYTESPLIT: { orc_rec br = byte_record(rec); return orc_blob_count(&br, m->inner); }
    case ORC_CHANGETYPE: { orc_rec sr = stored_record(rec, m); return orc_blob_count(&sr, m->inner); }
    case ORC_NULL: return 0;
    case ORC_SPLIT: {
      orc_rec p0 = split_part(rec, m, 0), p1 = split_part(rec, m, 1);
      return orc_blob_count(&p0, &m->inner[0]) + orc_blob_count(&p1, &m->inner[1]);
    }
    case ORC_FIELD_ACCESS_COUNT: return orc_blob_count(rec, m->inner) + 1;
    case ORC_HEATMAP: return 2 * orc_blob_count(rec, m->inner);
  }
  return 0;
}

EXPORT uint64_t orc_blob_size(const orc_rec* rec, const orc_map* m, uint64_t n, uint32_t b) {
  switch (m->kind) {
    case ORC_AOS: return n * (m->aos_packed ? packed_size(rec) : aligned_size(rec));
    case ORC_SOA_SB: return n * packed_size(rec);
    case ORC_SOA_MB: return n * orc_type_size(rec->types[b]);
    case ORC_AOSOA: return (n + m->lanes - 1) / m->lanes * m->lanes * packed_size(rec);
    case ORC_BYTESPLIT: { orc_rec br = byte_record(rec); return orc_blob_size(&br, m->inner, n, b); }
    case ORC_CHANGETYPE: { orc_rec sr = stored_record(rec, m); return orc_blob_size(&sr, m->inner, n, b); }
    case ORC_BITPACK_INT:
    case ORC_BITPACK_FLOAT: return 4 * ((n * code_bits(m) + 31) / 32);
    case ORC_NULL: return 0;
    case ORC_SPLIT: {
      orc_rec p0 = split_part(rec, m, 0), p1 = split_part(rec, m, 1);
      const uint32_t c0 = orc_blob_count(&p0, &m->inner[0]);
      return b < c0 ? orc_blob_size(&p0, &m->inner[0], n, b) : orc_blob_size(&p1, &m->inner[1], n, b - c0);
    }
    case ORC_FIELD_ACCESS_COUNT: {
      const uint32_t c = orc_blob_count(rec, m->inner);
      return b < c ? orc_blob_size(rec, m->inner, n, b) : 16ull * rec->nf;
    }
    case ORC_HEATMAP: {
      const uint32_t c = orc_blob_count(rec, m->inner);
      if (b < c) return orc_blob_size(rec, m->inner, n, b);
      return 8 * ((orc_blob_size(rec, m->inner, n, b - c) + m->lanes - 1) / m->lanes);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Bit streams: stream bit q is bit (q mod 8) of byte q/8.                   */
/* ------------------------------------------------------------------------ */

static uint64_t stream_get(const uint8_t* blob, uint64_t pos, uint32_t B) {
  uint64_t v = 0;
  for (uint32_t j = 0; j < B; ++j) {
    uint64_t q = pos + j;
    uint64_t bit = (blob[q >> 3] >> (q & 7)) & 1u;
    v |= bit << j;
  }
  return v;
}

static void stream_put(uint8_t* blob, uint64_t pos, uint32_t B, uint64_t v) {
  for (uint32_t j = 0; j < B; ++j) {
    uint64_t q = pos + j;
    uint8_t bit = (uint8_t)(1u << (q & 7));
    if ((v >> j) & 1ull) blob[q >> 3] |= bit;
    else blob[q >> 3] &= (uint8_t)~bit;
  }
}

/* ------------------------------------------------------------------------ */
/* Load / store one user value (bit pattern, zero-extended to 64 bits).     */
/* ------------------------------------------------------------------------ */

EXPORT uint64_t orc_load(const orc_rec* rec, const orc_map* m, uint64_t n, uint8_t* const* blobs,
                         uint64_t i, uint32_t f) {
  const int t = rec->types[f];
  switch (m->kind) {
    case ORC_AOS: case ORC_SOA_SB: case ORC_SOA_MB: case ORC_AOSOA: case ORC_BYTESPLIT: {
      uint64_t v = 0;
      for (uint32_t k = 0; k < orc_type_size(t); ++k) {
        uint32_t b;
        uint64_t o;
        orc_locate(rec, m, n, i, f, k, &b, &o);
        v |= (uint64_t)blobs[b][o] << (8 * k);
      }
      return v;
    }
    case ORC_CHANGETYPE: {
      orc_rec sr = stored_record(rec, m);
      uint64_t raw = orc_load(&sr, m->inner, n, blobs, i, f);
      return convert_value(raw, m->stored_types[f], t);
    }
    case ORC_BITPACK_INT: {
      uint32_t B = m->bits, w = 8 * orc_type_size(t);
      uint64_t c = stream_get(blobs[f], i * B, B);
      if (is_signed_int(t) && B < 64 && ((c >> (B - 1)) & 1ull)) c |= ~low_mask(B);
      return c & low_mask(w);
    }
    case ORC_BITPACK_FLOAT: {
      uint32_t B = code_bits(m);
      uint64_t c = stream_get(blobs[f], i * B, B);
      return orc_float_decode(c, t, m->exp_bits, m->man_bits);
    }
    case ORC_NULL: return 0;
    case ORC_SPLIT: {
      orc_rec p0 = split_part(rec, m, 0);
      if (f < m->lanes) return orc_load(&p0, &m->inner[0], n, blobs, i, f);
      orc_rec p1 = split_part(rec, m, 1);
      return orc_load(&p1, &m->inner[1], n, blobs + orc_blob_count(&p0, &m->inner[0]), i, f - m->lanes);
    }
    case ORC_FIELD_ACCESS_COUNT:
    case ORC_HEATMAP:
      count_access(rec, m, n, blobs, i, f, 0);
      return orc_load(rec, m->inner, n, blobs, i, f);
  }
  return 0;
}

EXPORT void orc_store(const orc_rec* rec, const orc_map* m, uint64_t n, uint8_t* const* blobs,
                      uint64_t i, uint32_t f, uint64_t v) {
  const int t = rec->types[f];
  switch (m->kind) {
    case ORC_AOS: case ORC_SOA_SB: case ORC_SOA_MB: case ORC_AOSOA: case ORC_BYTESPLIT:
      for (uint32_t k = 0; k < orc_type_size(t); ++k) {
        uint32_t b;
        uint64_t o;
        orc_locate(rec, m, n, i, f, k, &b, &o);
        blobs[b][o] = (uint8_t)(v >> (8 * k));
      }
      return;
    case ORC_CHANGETYPE: {
      orc_rec sr = stored_record(rec, m);
      orc_store(&sr, m->inner, n, blobs, i, f, convert_value(v, t, m->stored_types[f]));
      return;
    }
    case ORC_BITPACK_INT:
      stream_put(blobs[f], i * m->bits, m->bits, v & low_mask(m->bits));
      return;
    case ORC_BITPACK_FLOAT: {
      uint32_t B = code_bits(m);
      stream_put(blobs[f], i * B, B,
                 m->round_rne ? orc_float_encode_rne(v, t, m->exp_bits, m->man_bits)
                              : orc_float_encode(v, t, m->exp_bits, m->man_bits));
      return;
    }
    case ORC_NULL: return;
    case ORC_SPLIT: {
      orc_rec p0 = split_part(rec, m, 0);
      if (f < m->lanes) {
        orc_store(&p0, &m->inner[0], n, blobs, i, f, v);
      } else {
        orc_rec p1 = split_part(rec, m, 1);
        orc_store(&p1, &m->inner[1], n, blobs + orc_blob_count(&p0, &m->inner[0]), i, f - m->lanes, v);
      }
      return;
    }
    case ORC_FIELD_ACCESS_COUNT:
    case ORC_HEATMAP:
      count_access(rec, m, n, blobs, i, f, 1);
      orc_store(rec, m->inner, n, blobs, i, f, v);
      return;
  }
}

/* ------------------------------------------------------------------------ */
/* Layout-aware copy: dst(i).f = src(i).f for all i < n, all leaves f.       */
/* ------------------------------------------------------------------------ */

static int is_bitpacked(const orc_map* m) {
  return m->kind == ORC_BITPACK_INT || m->kind == ORC_BITPACK_FLOAT;
}

/* the stream bits past the last value up to the word end are zero (also in
 * the parts of a Split) */
static void clear_stream_tails(const orc_rec* rec, const orc_map* m, uint8_t* const* blobs, uint64_t n) {
  if (m->kind == ORC_SPLIT) {
    orc_rec p0 = split_part(rec, m, 0), p1 = split_part(rec, m, 1);
    clear_stream_tails(&p0, &m->inner[0], blobs, n);
    clear_stream_tails(&p1, &m->inner[1], blobs + orc_blob_count(&p0, &m->inner[0]), n);
    return;
  }
  if (m->kind == ORC_FIELD_ACCESS_COUNT || m->kind == ORC_HEATMAP) {
    clear_stream_tails(rec, m->inner, blobs, n);
    return;
  }
  if (!is_bitpacked(m)) return;
  const uint32_t B = code_bits(m);
  for (uint32_t f = 0; f < rec->nf; ++f) {
    const uint64_t end = 8 * orc_blob_size(rec, m, n, f);
    for (uint64_t q = n * B; q < end; ++q) blobs[f][q >> 3] &= (uint8_t)~(1u << (q & 7));
  }
}

EXPORT int orc_copy(const orc_rec* rec, const orc_map* src, uint8_t* const* sblobs,
                    const orc_map* dst, uint8_t* const* dblobs, uint64_t n, int threads) {
  /* records are visited in blocks of 64 so that two threads never share a
   * byte of a bit stream (64 records * B bits is a whole number of bytes) */
  const int64_t nblk = (int64_t)((n + 63) / 64);
#ifdef _OPENMP
  if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(threads)
#endif
  for (int64_t blk = 0; blk < nblk; ++blk) {
    uint64_t i_end = (uint64_t)(blk + 1) * 64;
    if (i_end > n) i_end = n;
    for (uint64_t i = (uint64_t)blk * 64; i < i_end; ++i)
      for (uint32_t f = 0; f < rec->nf; ++f)
        orc_store(rec, dst, n, dblobs, i, f, orc_load(rec, src, n, sblobs, i, f));
  }
  clear_stream_tails(rec, dst, dblobs, n);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Array extents and their linearisation (Sec. 2 array extents).  The       */
/* record at multi-index a = (a_0 .. a_{r-1}) of extents e sits at linear    */
/* index  sum_k a_k * prod_{m>k} e_m  (row-major: last extent fastest) or    */
/*        sum_k a_k * prod_{m<k} e_m  (column-major: first extent fastest).  */
/* ------------------------------------------------------------------------ */

EXPORT uint64_t orc_linearize(uint32_t rank, const uint64_t* ext, const uint64_t* a, int col_major) {
  uint64_t lin = 0;
  if (col_major) {
    for (int k = (int)rank - 1; k >= 0; --k) lin = lin * ext[k] + a[k];
  } else {
    for (uint32_t k = 0; k < rank; ++k) lin = lin * ext[k] + a[k];
  }
  return lin;
}

/* dst(a).f = src(a).f for every multi-index a of the extents and every leaf
 * f, each side linearised in its own order.  Multi-indices are visited in
 * row-major order, one at a time. */
EXPORT int orc_copy_nd(const orc_rec* rec, const orc_map* src, uint8_t* const* sblobs, int src_col_major,
                       const orc_map* dst, uint8_t* const* dblobs, int dst_col_major, uint32_t rank,
                       const uint64_t* ext) {
  uint64_t n = 1, a[8] = {0};
  if (rank < 1 || rank > 8) return -1;
  for (uint32_t k = 0; k < rank; ++k) n *= ext[k];
  for (uint64_t c = 0; c < n; ++c) {
    const uint64_t is = orc_linearize(rank, ext, a, src_col_major);
    const uint64_t id = orc_linearize(rank, ext, a, dst_col_major);
    for (uint32_t f = 0; f < rec->nf; ++f) orc_store(rec, dst, n, dblobs, id, f, orc_load(rec, src, n, sblobs, is, f));
    for (int k = (int)rank - 1; k >= 0; --k) {  /* next multi-index, last extent fastest */
      if (++a[k] < ext[k]) break;
      a[k] = 0;
    }
  }
  clear_stream_tails(rec, dst, dblobs, n);
  return 0;
}

/* Batched helpers for tests: values and locations of sampled elements. */
EXPORT void orc_load_many(const orc_rec* rec, const orc_map* m, uint64_t n, uint8_t* const* blobs,
                          const uint64_t* idx, const uint32_t* fields, uint64_t count,
                          uint64_t* out) {
  for (uint64_t c = 0; c < count; ++c) out[c] = orc_load(rec, m, n, blobs, idx[c], fields[c]);
}

EXPORT void orc_locate_many(const orc_rec* rec, const orc_map* m, uint64_t n, const uint64_t* idx,
                            const uint32_t* fields, const uint32_t* bytes, uint64_t count,
                            uint32_t* blob, uint64_t* off) {
  for (uint64_t c = 0; c < count; ++c)
    orc_locate(rec, m, n, idx[c], fields[c], bytes[c], &blob[c], &off[c]);
}

/* Element-wise conversions over arrays (exhaustive tests). */
static uint64_t read_elem(const void* p, uint32_t s, uint64_t i) {
  uint64_t v = 0;
  memcpy(&v, (const uint8_t*)p + i * s, s);
  return v;
}

static void write_elem(void* p, uint32_t s, uint64_t i, uint64_t v) {
  memcpy((uint8_t*)p + i * s, &v, s);
}

EXPORT void orc_convert_array(const void* in, int from, void* out, int to, uint64_t n, int threads) {
  const uint32_t si = orc_type_size(from), so = orc_type_size(to);
#ifdef _OPENMP
  if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(threads)
#endif
  for (int64_t i = 0; i < (int64_t)n; ++i)
    write_elem(out, so, (uint64_t)i, convert_value(read_elem(in, si, (uint64_t)i), from, to));
}

/* codes are stored one per uint64 for arrays */
EXPORT void orc_float_encode_array(const void* in, int t, uint32_t E, uint32_t M, uint64_t* codes,
                                   uint64_t n, int threads, int rne) {
  const uint32_t s = orc_type_size(t);
#ifdef _OPENMP
  if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(threads)
#endif
  for (int64_t i = 0; i < (int64_t)n; ++i) {
    const uint64_t v = read_elem(in, s, (uint64_t)i);
    codes[i] = rne ? orc_float_encode_rne(v, t, E, M) : orc_float_encode(v, t, E, M);
  }
}

EXPORT void orc_float_decode_array(const uint64_t* codes, int t, uint32_t E, uint32_t M, void* out,
                                   uint64_t n, int threads) {
  const uint32_t s = orc_type_size(t);
#ifdef _OPENMP
  if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(threads)
#endif
  for (int64_t i = 0; i < (int64_t)n; ++i)
    write_elem(out, s, (uint64_t)i, orc_float_decode(codes[i], t, E, M));
}

/* ------------------------------------------------------------------------ */
/* n-body in FP64 (Sec. 5 update then move; textbook softened gravity, G=1). */
/*   a_i = sum_j m_j (x_j - x_i) / (|x_j - x_i|^2 + eps2)^(3/2)               */
/*   v_i += dt a_i for every i (from the positions before the step)          */
/*   x_i += dt v_i                                                           */
/* pos and vel are n x 3, row-major.                                         */
/* ------------------------------------------------------------------------ */

EXPORT void orc_nbody(double* pos, double* vel, const double* mass, uint64_t n, uint32_t steps,
                      double dt, double eps2, int threads) {
  double* acc = (double*)malloc(sizeof(double) * 3 * (n ? n : 1));
#ifdef _OPENMP
  if (threads <= 0) threads = omp_get_max_threads();
#endif
  for (uint32_t step = 0; step < steps; ++step) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(threads)
#endif
    for (int64_t i = 0; i < (int64_t)n; ++i) {
      double ax = 0, ay = 0, az = 0;
      for (uint64_t j = 0; j < n; ++j) {
        double dx = pos[3 * j + 0] - pos[3 * i + 0];
        double dy = pos[3 * j + 1] - pos[3 * i + 1];
        double dz = pos[3 * j + 2] - pos[3 * i + 2];
        double r2 = dx * dx + dy * dy + dz * dz + eps2;
        double w = mass[j] / (r2 * sqrt(r2));
        ax += dx * w;
        ay += dy * w;
        az += dz * w;
      }
      acc[3 * i + 0] = ax;
      acc[3 * i + 1] = ay;
      acc[3 * i + 2] = az;
    }
    for (uint64_t i = 0; i < 3 * n; ++i) vel[i] += dt * acc[i];
    for (uint64_t i = 0; i < 3 * n; ++i) pos[i] += dt * vel[i];
  }
  free(acc);
}

/* E = 1/2 sum m_i |v_i|^2 - sum_{i<j} m_i m_j / sqrt(|x_i - x_j|^2 + eps2) */
EXPORT double orc_energy(const double* pos, const double* vel, const double* mass, uint64_t n,
                         double eps2, int threads) {
  double kin = 0, pot = 0;
  for (uint64_t i = 0; i < n; ++i)
    kin += 0.5 * mass[i] *
           (vel[3 * i] * vel[3 * i] + vel[3 * i + 1] * vel[3 * i + 1] + vel[3 * i + 2] * vel[3 * i + 2]);
#ifdef _OPENMP
  if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : pot) num_threads(threads)
#endif
  for (int64_t i = 0; i < (int64_t)n; ++i) {
    double p = 0;
    for (uint64_t j = (uint64_t)i + 1; j < n; ++j) {
      double dx = pos[3 * i] - pos[3 * j], dy = pos[3 * i + 1] - pos[3 * j + 1],
             dz = pos[3 * i + 2] - pos[3 * j + 2];
      p += mass[j] / sqrt(dx * dx + dy * dy + dz * dz + eps2);
    }
    pot += mass[i] * p;
  }
  return kin - pot;
}

/* ------------------------------------------------------------------------ */
/* The n-body consumer through a mapping (Sec. 5, instrumented as in Sec. 4) */
/* Same steps as orc_nbody, in FP64, but every value is loaded from and      */
/* stored to the particle view's blobs through the mapping, one access at a  */
/* time, in the access pattern of an update that stages j-particles in tiles: */
/*   per step: each particle's position once; for each block of `tile`      */
/*   i-particles, every j-particle's position and mass once; then for every  */
/*   particle and component c: load v_c, store v_c + dt a_c, load x_c, store */
/*   x_c + dt v_c.  An instrumented mapping counts them all.                 */
/* Leaves: pos.x pos.y pos.z vel.x vel.y vel.z mass, all F32 or all F64.     */
/* ------------------------------------------------------------------------ */

static double as_double(uint64_t bits, int t) {
  if (t == ORC_F64) { double d; memcpy(&d, &bits, 8); return d; }
  uint32_t u = (uint32_t)bits;
  float f;
  memcpy(&f, &u, 4);
  return (double)f;
}

static uint64_t from_double(double d, int t) {
  if (t == ORC_F64) { uint64_t b; memcpy(&b, &d, 8); return b; }
  float f = (float)d;
  uint32_t u;
  memcpy(&u, &f, 4);
  return u;
}

EXPORT void orc_nbody_view(const orc_rec* rec, const orc_map* m, uint8_t* const* blobs, uint64_t n,
                           uint32_t steps, double dt, double eps2, uint32_t tile) {
  const int t = rec->types[0];
  double* xi = (double*)malloc(sizeof(double) * 3 * (n ? n : 1));
  double* acc = (double*)malloc(sizeof(double) * 3 * (n ? n : 1));
  for (uint32_t step = 0; step < steps; ++step) {
    for (uint64_t i = 0; i < n; ++i)
      for (uint32_t c = 0; c < 3; ++c) xi[3 * i + c] = as_double(orc_load(rec, m, n, blobs, i, c), t);
    for (uint64_t i = 0; i < 3 * n; ++i) acc[i] = 0;
    for (uint64_t b = 0; b < n; b += tile) {
      const uint64_t e = b + tile < n ? b + tile : n;
      for (uint64_t j = 0; j < n; ++j) {
        double xj[3], mj;
        for (uint32_t c = 0; c < 3; ++c) xj[c] = as_double(orc_load(rec, m, n, blobs, j, c), t);
        mj = as_double(orc_load(rec, m, n, blobs, j, 6), t);
        for (uint64_t i = b; i < e; ++i) {
          double d[3], r2 = eps2;
          for (uint32_t c = 0; c < 3; ++c) {
            d[c] = xj[c] - xi[3 * i + c];
            r2 += d[c] * d[c];
          }
          const double w = mj / (r2 * sqrt(r2));
          for (uint32_t c = 0; c < 3; ++c) acc[3 * i + c] += d[c] * w;
        }
      }
    }
    for (uint64_t i = 0; i < n; ++i)
      for (uint32_t c = 0; c < 3; ++c) {
        const double v = as_double(orc_load(rec, m, n, blobs, i, 3 + c), t) + dt * acc[3 * i + c];
        orc_store(rec, m, n, blobs, i, 3 + c, from_double(v, t));
        const double x = as_double(orc_load(rec, m, n, blobs, i, c), t) + dt * v;
        orc_store(rec, m, n, blobs, i, c, from_double(x, t));
      }
  }
  free(xi);
  free(acc);
}

/* Energy through the mapping: every leaf of every particle loaded once. */
EXPORT double orc_energy_view(const orc_rec* rec, const orc_map* m, uint8_t* const* blobs, uint64_t n,
                              double eps2) {
  const int t = rec->types[0];
  double* p = (double*)malloc(sizeof(double) * 7 * (n ? n : 1));
  for (uint64_t i = 0; i < n; ++i)
    for (uint32_t f = 0; f < 7; ++f) p[7 * i + f] = as_double(orc_load(rec, m, n, blobs, i, f), t);
  double kin = 0, pot = 0;
  for (uint64_t i = 0; i < n; ++i) {
    const double* a = p + 7 * i;
    kin += 0.5 * a[6] * (a[3] * a[3] + a[4] * a[4] + a[5] * a[5]);
    for (uint64_t j = i + 1; j < n; ++j) {
      const double* b = p + 7 * j;
      const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
      pot += a[6] * b[6] / sqrt(dx * dx + dy * dy + dz * dz + eps2);
    }
  }
  free(p);
  return kin - pot;
}

EXPORT int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
