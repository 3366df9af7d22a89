/*
 * llama_mi.h - C ABI of the MI355X (gfx950) layout-copy / pack library.
 *
 * The library implements the data-parallel hot path of "Updates on the
 * Low-Level Abstraction of Memory Access" (LLAMA, arXiv 2302.08251):
 * structured records (a record dimension of leaf fields spanned over array
 * extents, Sec. 1) are stored through exchangeable memory mappings, and this
 * library moves them between mappings on one GPU:
 *   - layout-aware copy between the physical mappings AoS, SoA single-blob,
 *     SoA multi-blob, AoSoA-L and Bytesplit (Sec. 1 layout-aware copy,
 *     Sec. 3 Bytesplit, Sec. 5 AoS / SoA MB / AoSoA);
 *   - pack / unpack through the computed mappings ChangeType,
 *     BitPackedIntSoA and BitPackedFloatSoA (Sec. 3);
 *   - one record-streaming consumer, an all-pairs n-body step that reads
 *     and writes particles through a mapping (Sec. 5, n-body update / move).
 *
 * Conventions shared by every entry point
 *   - Every function returns llama_status; 0 (LLAMA_OK) is success.  On an
 *     error nothing is enqueued, and llama_last_error() returns a message
 *     (thread-local, valid until the next failing call on the same thread).
 *     No C++ exception ever crosses this interface.
 *   - Argument validation is synchronous and happens on the host before any
 *     GPU work.  GPU work is asynchronous on the given stream: `stream` is a
 *     hipStream_t passed as void* (NULL = the default stream).  A failing
 *     kernel launch returns LLAMA_ERR_HIP with the HIP error string.
 *   - Blobs are caller-owned device memory (for example torch tensors).
 *     Views and batches are library-owned handles that only hold pointers;
 *     the caller keeps blobs alive until work on the stream has completed.
 *   - All multi-byte values are little-endian.  Array extents are linearised
 *     row-major (last extent fastest) unless the view's mapping sets
 *     LLAMA_FLAG_COL_MAJOR; every operation works on the linearised record
 *     index i in [0, N), N = product of the extents.
 */
#ifndef LLAMA_MI_H
#define LLAMA_MI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum llama_status {
  LLAMA_OK = 0,
  LLAMA_ERR_INVALID_ARG = -1,     /* malformed descriptor, null pointer, bad parameter  */
  LLAMA_ERR_UNSUPPORTED = -2,     /* well-formed but not implemented by the GPU path    */
  LLAMA_ERR_INDEX_OVERFLOW = -3,  /* extents or blob sizes do not fit the index type    */
  LLAMA_ERR_RECORD_MISMATCH = -4, /* source and destination records differ              */
  LLAMA_ERR_ALIGNMENT = -5,       /* blob base not 16-byte aligned                      */
  LLAMA_ERR_HIP = -6,             /* HIP runtime error                                  */
  LLAMA_ERR_NO_MEMORY = -7,       /* host or device allocation failed, blob too small   */
} llama_status;

/* Type used for index arithmetic of a view (Sec. 2, compile-time array
 * extents: one index type for all index and offset computations).  A view is
 * rejected when its record count or any blob byte size does not fit the
 * type.  The kernels always compute per-lane offsets in 32 bits relative to a
 * per-tile 64-bit scalar base, so the narrowest type that fits is free. */
typedef enum llama_index_type {
  LLAMA_IDX_I16 = 0, LLAMA_IDX_U16 = 1,
  LLAMA_IDX_I32 = 2, LLAMA_IDX_U32 = 3,
  LLAMA_IDX_I64 = 4, LLAMA_IDX_U64 = 5,
} llama_index_type;

/* Scalar leaf types.  F16 / BF16 are accepted as ChangeType storage types
 * (Sec. 3, extended floating-point types). */
typedef enum llama_scalar {
  LLAMA_F32 = 0, LLAMA_F64 = 1,
  LLAMA_I8 = 2,  LLAMA_U8 = 3, LLAMA_I16 = 4, LLAMA_U16 = 5,
  LLAMA_I32 = 6, LLAMA_U32 = 7, LLAMA_I64 = 8, LLAMA_U64 = 9,
  LLAMA_F16 = 10, LLAMA_BF16 = 11,
} llama_scalar;

/* Record dimension (Sec. 1): the leaf fields of a possibly nested record,
 * flattened depth-first in declaration order, e.g. the n-body particle
 * {pos.x, pos.y, pos.z, vel.x, vel.y, vel.z, mass}.  At most 64 leaves. */
typedef struct llama_record {
  uint32_t n_fields;
  const llama_scalar* types; /* n_fields entries */
} llama_record;

typedef enum llama_map_kind {
  /* Physical mappings.  s_f = size of leaf f, p_f = sum of s_g for g < f,
   * S = sum of s_f.  Locations of byte k of field f of record i:          */
  LLAMA_MAP_AOS = 0,       /* 1 blob: i*S' + q_f + k; q_f are C-struct offsets
                              and S' the C-struct size (or p_f and S with
                              LLAMA_FLAG_AOS_PACKED).                         */
  LLAMA_MAP_SOA_SB = 1,    /* 1 blob: N*p_f + i*s_f + k (planes back to back) */
  LLAMA_MAP_SOA_MB = 2,    /* one blob per field: blob f, i*s_f + k           */
  LLAMA_MAP_AOSOA = 3,     /* 1 blob of ceil(N/L)*L*S bytes:
                              (i/L)*L*S + L*p_f + (i%L)*s_f + k; the lanes past
                              N in the last block are padding that no copy
                              writes.                                         */
  LLAMA_MAP_BYTESPLIT = 4, /* Sec. 3 Bytesplit: every field becomes s_f one-byte
                              fields (byte k = k-th byte in memory order) and the
                              resulting byte record is placed by `inner`, which
                              must be AOS, SOA_SB, SOA_MB or AOSOA.           */
  /* Computed mappings (Sec. 3): values are converted on store and on load. */
  LLAMA_MAP_CHANGETYPE = 5,        /* field f is stored as stored_types[f] and
                                      the storage record is placed by `inner`
                                      (physical or BYTESPLIT).  Float narrowing
                                      rounds to nearest even, widening is exact;
                                      NaN keeps its sign and top payload bits
                                      and is made quiet.                       */
  LLAMA_MAP_BITPACK_INT_SOA = 6,   /* integer fields kept to `bits` bits, one
                                      LSB-first bitstream per field (blob f);
                                      value i occupies stream bits [i*B, i*B+B).
                                      Store keeps the low B bits (wraps); load
                                      sign-extends signed types.  Blob f has
                                      4*ceil(N*B/32) bytes, tail bits are 0.   */
  LLAMA_MAP_BITPACK_FLOAT_SOA = 7, /* float fields kept as [sign|E|M] codes of
                                      1+E+M bits, streams as above.  Exponent
                                      bias 2^(E-1)-1; mantissa truncated toward
                                      zero; overflow gives +-Inf; underflow is
                                      gradual then +-0; Inf kept; NaN kept with
                                      its top M payload bits and the quiet bit
                                      set (M = 0 turns NaN into Inf).  Decoding
                                      is exact.                                 */
  /* Meta-mappings (Sec. 3). */
  LLAMA_MAP_NULL = 8,              /* no blobs: loads give zero, stores are
                                      dropped.  On the GPU a copy from NULL
                                      writes zero to every mapped byte of the
                                      destination (AoSoA padding untouched) and
                                      a copy to NULL does nothing.            */
  LLAMA_MAP_SPLIT = 9,             /* the first `lanes` leaf fields (1 <= lanes
                                      < n_fields) are placed by inner[0], the
                                      rest by inner[1]: `inner` points to an
                                      array of two mappings.  Blobs: inner[0]'s,
                                      then inner[1]'s.  Against another SPLIT
                                      with the same split point, SOA_MB or NULL
                                      a copy runs once per part; against any
                                      other partner it moves each record leaf
                                      by leaf (value by value where a part is
                                      computed), within 8 physical parts per
                                      SPLIT tree and 64 storage columns per
                                      side (UNSUPPORTED beyond; batches take no
                                      SPLIT or NULL views).                   */
  /* Instrumentation (Sec. 4): locations, loads and stores go to `inner`;
   * every access also adds one to 64-bit counters held in extra blobs placed
   * after the inner mapping's blobs.  The caller owns those blobs and zeroes
   * them (or keeps counting across calls); a copy adds, it never clears.
   * A copy adds its counts after its data kernels, on the same stream, one
   * add per counter; copies that overlap in time on views sharing counter
   * blobs race, as overlapping writes to any blob do. */
  LLAMA_MAP_FIELD_ACCESS_COUNT = 10, /* one extra blob of 2*n_fields counters:
                                        counter 2f counts the loads of field f,
                                        counter 2f+1 its stores.  `inner`: any
                                        mapping of kinds 0-7.  A copy loads
                                        every field of every record of the
                                        source once and stores it once into
                                        the destination.                      */
  LLAMA_MAP_HEATMAP = 11,            /* `lanes` = G, bytes per counter, a power
                                        of two in [1, 2^20].  One extra blob per
                                        inner blob b: ceil(size_b / G) counters;
                                        counter g of b counts the accesses that
                                        touch at least one of the bytes
                                        [g*G, g*G+G) of blob b.  G = 1 costs 8
                                        bytes of counters per byte.  `inner`:
                                        AOS, SOA_SB, SOA_MB or AOSOA.          */
} llama_map_kind;

#define LLAMA_FLAG_AOS_PACKED 0x1u /* AOS: no alignment padding between fields */
#define LLAMA_FLAG_COL_MAJOR 0x4u  /* Sec. 2 array extents: the view linearises its
                                      multi-index column-major, first extent fastest:
                                      record (a_0 .. a_{r-1}) sits at linear index
                                      sum_k a_k * prod_{m<k} e_m (row-major, the
                                      default: sum_k a_k * prod_{m>k} e_m).  Valid on
                                      the outermost mapping of a view only (INVALID_ARG
                                      on an inner one).  llama_copy copies dst(a) =
                                      src(a) for every multi-index a: views in the same
                                      order (or whose extents have at most one entry
                                      above 1) copy by linear index as usual; views in
                                      different orders must have the same extents
                                      (RECORD_MISMATCH otherwise), and the copy is a
                                      record permutation: a tiled transpose between
                                      physical mappings with leaves of one size, a
                                      per-leaf or value-level copy otherwise
                                      (UNSUPPORTED in batches). */
#define LLAMA_FLAG_ROUND_RNE 0x2u  /* BITPACK_FLOAT: round the mantissa to nearest,
                                      ties to even (ties compare the
                                      significand's last bit: with M = 0 the
                                      hidden bit, so a tie rounds away from
                                      zero), instead of truncating it; a value
                                      that rounds past the largest finite code
                                      gives +-Inf.  Other mappings: INVALID_ARG. */

typedef struct llama_mapping {
  llama_map_kind kind;
  uint32_t lanes;     /* AOSOA: L >= 1; SPLIT: split point; HEATMAP: G               */
  uint32_t bits;      /* BITPACK_INT: 1 <= B <= bit width of every field type        */
  uint32_t exp_bits;  /* BITPACK_FLOAT: 2 <= E <= exponent width of every field type  */
  uint32_t man_bits;  /* BITPACK_FLOAT: 0 <= M <= mantissa width of every field type  */
  uint32_t flags;     /* LLAMA_FLAG_*                                               */
  const llama_scalar* stored_types;  /* CHANGETYPE: n_fields storage types          */
  const struct llama_mapping* inner; /* BYTESPLIT / CHANGETYPE / instrumentation:
                                        forwarded mapping; SPLIT: array of two    */
} llama_mapping;

typedef struct llama_view llama_view;   /* opaque */
typedef struct llama_batch llama_batch; /* opaque */

/* Sec. 2 separates a view's blobs from the allocator that provides them: a
 * mapping only states how many blobs it needs and how large each one is,
 * and the caller allocates them.  The next two calls answer those questions.
 * Errors: INVALID_ARG (malformed record or mapping, NULL output, blob index
 * out of range), INDEX_OVERFLOW (extents overflow 64 bits).
 *
 * Number of blobs a mapping uses for a record (AOS, SOA_SB, AOSOA: 1;
 * SOA_MB: n_fields; BYTESPLIT/CHANGETYPE: the inner mapping's count over the
 * byte / storage record; BITPACK_*: n_fields; NULL: 0; SPLIT: the sum of its
 * parts'; FIELD_ACCESS_COUNT: the inner count + 1; HEATMAP: twice the inner
 * count). */
llama_status llama_mapping_blob_count(const llama_record* rec, const llama_mapping* map,
                                      uint32_t* n_blobs);

/* Byte size of blob `blob` for the given extents (rank 1..8), row-major
 * unless the mapping sets LLAMA_FLAG_COL_MAJOR (the size does not depend on
 * the order). */
llama_status llama_mapping_blob_size(const llama_record* rec, const llama_mapping* map,
                                     uint32_t rank, const uint64_t* extents, uint32_t blob,
                                     uint64_t* bytes);

/* Creates a view: mapping + extents + index type over caller-owned blobs
 * (Sec. 1 View, Sec. 2 index type).  `blobs[b]` is a device pointer, 16-byte
 * aligned, of at least `blob_bytes[b]` bytes, which must be >= the mapping's
 * size for blob b.  The descriptor is deep-copied.  Errors: INVALID_ARG,
 * INDEX_OVERFLOW, ALIGNMENT, NO_MEMORY (a blob smaller than required). */
llama_status llama_view_create(const llama_record* rec, const llama_mapping* map,
                               uint32_t rank, const uint64_t* extents,
                               llama_index_type index_type, void* const* blobs,
                               const uint64_t* blob_bytes, uint32_t n_blobs,
                               llama_view** out);
/* Destroys a view handle (Sec. 1: a view binds a mapping to blobs it does
 * not own).  The blobs are untouched and stay the caller's.  NULL is a no-op.
 * Work already enqueued on a stream keeps its own copy of the descriptors,
 * so a view may be destroyed before that work completes. */
llama_status llama_view_destroy(llama_view* view);

/* Number of records of a view. */
llama_status llama_view_records(const llama_view* view, uint64_t* n);

/* Layout-aware copy (Sec. 1): for every record i < N and leaf field f,
 * dst(i).f = src(i).f.  Both views must have the same record and N.  Between
 * physical mappings this moves bits (NaN payloads and denormals survive);
 * through computed mappings the values are encoded on store and decoded on
 * load.  AoSoA padding lanes of dst are never written.  Meta-mappings and
 * instrumentation: see LLAMA_MAP_NULL, _SPLIT, _FIELD_ACCESS_COUNT and
 * _HEATMAP (an instrumented source counts loads even into a NULL dst).
 * Records whose leaves differ in size (Sec. 1 record dimension, e.g. the C
 * struct {u8; f64; i16; f32}: 24-byte aligned AoS records, 15 packed) copy
 * between the physical mappings, their Bytesplit forms and NULL, leaf by leaf;
 * padding bytes of dst are never written.  A Bytesplit side of such a record
 * may hold at most 64 bytes per record.
 * Pairs the layout kernels do not move (two computed views, integer
 * ChangeType, bit-packed codes of 33 to 64 bits, bit-packed f16 / bf16 leaves,
 * SPLIT trees with computed parts against a partner of another form) are
 * copied value by value: load through src's mapping, store through dst's.  A
 * copy between two converting ChangeType views thus converts twice, and a
 * signalling NaN comes out quiet.
 * Errors: RECORD_MISMATCH (records or N differ), UNSUPPORTED (nothing is
 * launched: more than 8 physical parts in one SPLIT tree against a partner of
 * another form, or more than 64 storage columns - blobs, byte columns, bit
 * streams - on one side), INVALID_ARG. */
llama_status llama_copy(const llama_view* src, llama_view* dst, void* stream);

/* Sec. 3 computed mappings convert values when they are stored to memory
 * (pack) and when they are loaded from it (unpack).  Pack: src physical,
 * dst computed (CHANGETYPE, BITPACK_INT_SOA or BITPACK_FLOAT_SOA): every
 * value of src is encoded through dst's mapping.  Unpack: src computed, dst
 * physical: every code of src is decoded into dst.  Otherwise UNSUPPORTED,
 * and nothing is enqueued.  Layouts, ownership, streams and the other errors
 * are as for llama_copy. */
llama_status llama_pack(const llama_view* src, llama_view* dst, void* stream);
llama_status llama_unpack(const llama_view* src, llama_view* dst, void* stream);

/* Launch parameters of one copy: tile_records = records per tile (0 = the
 * library's choice; otherwise a multiple of 128 and of every AoSoA lane count
 * involved), grid = workgroups (0 = one per tile; otherwise a persistent grid
 * that loops over tiles). */
typedef struct llama_launch_params {
  uint32_t tile_records;
  uint32_t grid;
} llama_launch_params;

/* llama_copy with explicit launch parameters (used by the autotuner).
 * `params` may be NULL.  INVALID_ARG when tile_records violates the rules
 * above or the tile does not fit in LDS. */
llama_status llama_copy_ex(const llama_view* src, llama_view* dst,
                           const llama_launch_params* params, void* stream);

/* Batched copy (many views of uneven sizes and mixed mapping pairs in one
 * persistent launch).  srcs[v] -> dsts[v] for v < n; every pair must be
 * valid for llama_copy and no two destinations may overlap.  The views must
 * outlive the batch.  `tune_cache` names a JSON file of tuned launch
 * parameters: read when it holds an entry for this device and batch shape,
 * otherwise the autotuner times candidates on the batch itself (this
 * overwrites destination blobs) and writes the entry.  NULL = always tune,
 * write nothing.  Creation synchronizes the device first.  The launch is
 * captured into a hipGraph at creation. */
llama_status llama_batch_create(uint32_t n, const llama_view* const* srcs,
                                llama_view* const* dsts, const char* tune_cache,
                                llama_batch** out);
/* Replays the batch's graph: one persistent kernel for all views. */
llama_status llama_batch_launch(llama_batch* batch, void* stream);
/* The baseline the batch is measured against: one llama_copy launch per
 * view, back to back on the stream, each with its tuned parameters. */
llama_status llama_batch_launch_per_view(llama_batch* batch, void* stream);
typedef struct llama_batch_info {
  uint32_t n_views;
  uint32_t tile_records;     /* chosen tile size (0: each view's default tile,
                                1: the same capped to 16 KiB of LDS, 2: each
                                view's tile grown to the LDS of the largest
                                default tile; else records per tile)           */
  uint32_t grid;             /* persistent workgroups                          */
  uint64_t total_tiles;
  uint64_t algorithmic_bytes;/* mapped bytes read + mapped bytes written       */
  double tune_seconds;       /* wall time spent autotuning at create (0 = cached) */
  uint32_t tile_map;         /* 1: one workgroup per tile, each of the 8 XCDs taking a
                                contiguous run of tiles (chosen by the autotuner) */
  uint32_t reserved;
} llama_batch_info;
llama_status llama_batch_get_info(const llama_batch* batch, llama_batch_info* info);
llama_status llama_batch_destroy(llama_batch* batch);

/* All-pairs n-body (Sec. 5, n-body update then move), reading and writing the
 * particles through the view's mapping.  Record: 7 float leaves
 * {pos.x, pos.y, pos.z, vel.x, vel.y, vel.z, mass}, all F32 or all F64.
 * Supported mappings: physical over F32 leaves; CHANGETYPE(F64 -> F32, physical
 * inner); BITPACK_FLOAT_SOA with E <= 8, M <= 23.  Per step, in FP32:
 *   a_i = sum_j m_j (x_j - x_i) (|x_j - x_i|^2 + eps2)^(-3/2)   (G = 1)
 *   v_i <- v_i + dt a_i  (all i, from the positions before the step)
 *   x_i <- x_i + dt v_i  (with v_i as stored through the mapping)
 * Scratch memory is allocated by the library on first use per device.
 * Instrumented views (Sec. 4): a FIELD_ACCESS_COUNT view over any of the
 * storage forms above, or a HEATMAP view over physical F32 storage, counts
 * every access the step makes through it: per step, each particle's
 * position leaves are loaded once by the update and once per block of 256
 * i-particles as a j-tile entry (with its mass), and the move loads and
 * stores each position and velocity leaf once.  Counts add to the counter
 * blobs as for llama_copy. */
llama_status nbody_step(llama_view* particles, uint32_t steps, float dt, float eps2,
                        void* stream);

/* nbody_step for callers that cannot allocate device memory: code under
 * hipGraph stream capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same kernels, arguments and results as nbody_step (bit for
 * bit), but no library allocation on any call: the per-slice partial
 * accelerations live in a static device array of 16 MiB that each GPU the
 * library runs on holds until the process ends.  That array fits at most
 * 1398101 particles (12 bytes of partial sums per particle once a view has
 * 2^19 particles or more); a larger view returns LLAMA_ERR_NO_MEMORY and
 * nothing is enqueued.  Every call on one GPU shares that GPU's array and
 * writes every element it reads, so nothing needs clearing between calls;
 * calls that overlap in time on one GPU (other streams, other threads) race
 * on it and must be serialised by the caller.  Errors as for nbody_step. */
llama_status nbody_step_noalloc(llama_view* particles, uint32_t steps, float dt, float eps2,
                                void* stream);

/* Total energy  E = 1/2 sum_i m_i |v_i|^2 - sum_{i<j} m_i m_j (|x_i-x_j|^2+eps2)^(-1/2)
 * computed on the GPU in FP64 with a fixed reduction order (deterministic),
 * from the values as decoded through the mapping.  Blocks until the result
 * is on the host.  An instrumented view counts one load of every leaf of
 * every particle. */
llama_status nbody_energy(const llama_view* particles, float eps2, double* energy,
                          void* stream);

/* Message describing the last error on this thread ("" if none). */
const char* llama_last_error(void);

/* Library version string. */
const char* llama_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LLAMA_MI_H */
