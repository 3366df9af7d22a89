// Internal descriptors shared by the host runtime and the HIP kernels.
//
// A copy moves the records of a tile [i0, i0 + nt) between two "sides".  A
// side is the structural form of a mapping after Bytesplit and ChangeType
// have been resolved:
//   LY_AOS     one segment of nt*S bytes (record-major)
//   LY_PLANAR  one segment per storage column (SoA single/multi blob)
//   LY_AOSOA   one segment of ceil(nt/L)*L*S bytes (blocks of L records)
//   LY_STREAM  one LSB-first bit stream per field (BitPacked*SoA)
// A storage column is a leaf field (cs = element size), or one byte of a
// leaf when the mapping is a Bytesplit (cs = 1, Sec. 3 Bytesplit).
#pragma once
#include <stdint.h>

#include "../../include/llama_mi.h"

namespace lm {

constexpr uint32_t kMaxFields = 64;
constexpr uint32_t kMaxCols = 64;
constexpr uint32_t kThreads = 256;            // threads per workgroup of the tile kernels
constexpr uint32_t kMaxTileLds = 64 * 1024;   // LDS bytes per tile
// Items (4 records x 1 field) per thread that the in-place merge of a
// Bytesplit source into an AoS image holds in registers, by leaf bytes.
template <int ES> constexpr int kMergeInPlaceItems = ES == 8 ? 4 : 8;
inline uint32_t merge_in_place_items(uint32_t es) { return es == 8 ? 4u : 8u; }

enum Layout : uint32_t { LY_AOS = 0, LY_PLANAR = 1, LY_AOSOA = 2, LY_STREAM = 3 };

// How a side's stored element relates to the user value.
enum ValueKind : uint32_t {
  VK_RAW = 0,    // stored bits are the user bits
  VK_CONV = 1,   // ChangeType: stored type differs from the user type
  VK_INT = 2,    // BitPackedIntSoA code
  VK_FLOAT = 3,  // BitPackedFloatSoA code
};

// Exact x / d for x * d < 2^32: q = (d power of two) ? x >> sh : umulhi(x, m),
// m = ceil(2^32 / d).
struct Div {
  uint32_t d, m, sh, pow2;
};

struct Side {
  uint32_t layout;     // Layout
  uint32_t vkind;      // ValueKind
  uint32_t cs;         // storage column size in bytes (1, 2, 4, 8)
  uint32_t log2cs;
  uint32_t ncols;      // storage columns (fields, or bytes of the record for Bytesplit)
  uint32_t rec_bytes;  // S: bytes of one stored record (ncols * cs)
  uint32_t es;         // stored element bytes (user size for RAW, storage size for CONV)
  uint32_t lanes;      // AoSoA L
  uint32_t mb;         // planar: 1 = one blob per column
  uint32_t bits;       // stream: code bits (1..32)
  uint32_t exp_bits, man_bits;
  uint32_t is_signed;  // VK_INT: sign-extend on decode
  uint32_t lds_stride; // planar / stream: LDS bytes per column or field plane
  uint32_t n_mod16;    // n mod 16 (phase of single-blob planes)
  uint32_t rne;        // stream: float codes round to nearest even (else truncate)
  uint64_t n;          // records
  uint64_t blob_size;  // bytes the mapping uses in each blob (all blobs of a side are equal)
  Div div_S;           // S
  Div div_LS;          // L * S
  Div div_Lcs;         // L * cs
  Div div_L;           // L
  Div div_B;           // stream code bits
  const void* blob[kMaxCols];
};

// Conversions between the two sides' elements.
enum Conv : uint32_t {
  CV_NONE = 0,
  CV_F64_F32 = 1,  // narrowing, round to nearest even
  CV_F32_F64 = 2,  // widening, exact
  CV_F32_F16 = 3,  // the rest: narrowing (RNE) or widening (exact) through
  CV_F32_BF16 = 4, //   the generic IEEE conversions
  CV_F64_F16 = 5,
  CV_F64_BF16 = 6,
  CV_F16_F32 = 7,
  CV_BF16_F32 = 8,
  CV_F16_F64 = 9,
  CV_BF16_F64 = 10,
};

// Bit-packed codecs by user element type.
enum Codec : uint32_t {
  CD_U8 = 0, CD_I8, CD_U16, CD_I16, CD_U32, CD_I32, CD_U64, CD_I64, CD_F32, CD_F64,
};

// Geometry of a tile image in LDS (the fields the source address function
// reads).  For a relayout it describes the canonical planar image.
struct Geo {
  uint32_t layout, cs, log2cs, ncols, rec_bytes, lanes, mb, n_mod16, lds_stride, pad;
  Div div_L;
};

// Raw-copy modes: how the source tile reaches Phase B.
enum RawMode : uint32_t {
  RM_DIRECT = 0,  // Phase B gathers from the verbatim source image
  RM_MERGE = 1,   // Bytesplit source: byte columns merged into element planes first
  RM_SPLIT = 2,   // Bytesplit destination: element columns split into byte planes first
  RM_MERGE_FUSED = 3,  // as RM_MERGE, transposed in registers and stored directly
  RM_SPLIT_FUSED = 4,  // as RM_SPLIT, transposed in registers and stored directly
  RM_LINE = 5,    // single-blob planar destination off the line grid: destination
                  // planes built in LDS, every 128-byte line written whole by one tile
};

struct TileArgs {
  Side src;
  Side dst;
  uint32_t tile;        // records per tile
  uint32_t ntiles_lo;   // number of tiles (low 32 bits; tiles < 2^32)
  uint32_t conv;        // Conv
  uint32_t codec;       // Codec (pack / unpack)
  uint32_t mode;        // RawMode
  uint32_t colrun;      // 1: destination chunks are runs of one column (copied 16 bytes at a time)
  uint32_t can_off;     // LDS offset of the canonical image (MERGE / SPLIT / LINE)
  uint32_t halo;        // LINE: records loaded past the tile (128 / destination column bytes)
  Geo can;              // canonical image geometry (MERGE / SPLIT / LINE)
};

// A copy between two views linearised in different orders (row- and
// column-major, Sec. 2 array extents): a batched 2-D transpose of records.
// Axis P is the destination's fastest axis, axis Q the source's; the other
// ("middle") axes are fixed per tile.  A tile holds T x T records: T
// consecutive source records (along Q) for each of T values along P.
// Records move in units of U bytes (U = the smaller column size of the two
// sides).  Counts and strides are in records.
struct XposeArgs {
  Side src;
  Side dst;
  uint32_t nunits;          // units per record
  uint32_t T, log2T;        // tile edge (a power of two)
  uint32_t src_rec_major;   // the source keeps a record's units together (AoS)
  uint32_t dst_rec_major;
  uint32_t nmid;            // middle axes
  Div div_units;
  uint64_t src_lmag, dst_lmag;  // AoSoA: ceil(2^64 / L) (0: L is a power of two)
  uint64_t eP, eQ;          // extents of the two tile axes
  uint64_t sP, dQ;          // source stride of axis P, destination stride of axis Q
  uint64_t nPt, nQt, ntiles;
  uint64_t mext[8], msrc[8], mdst[8];  // middle axes: extent, source and destination strides
};

// A copy that the tile engine does not cover: records whose leaves differ in
// size (Sec. 1 record dimension, e.g. a C struct {u8; f64; i16; f32} with its
// alignment padding), or SPLIT views (Sec. 3) with a partner of another form.
// Each record's leaves move one element at a time, or byte by byte where a
// side splits the leaf into byte columns or does not align it.  A side is a
// list of groups, one per physical mapping in its mapping tree (a SPLIT has
// one per part); leaf f belongs to group grp[f] and its element (or its first
// byte column) is col[cidx[f]].  Record i's leaf, or byte column, c lives at
//   col[c] + i * size                              (L = 0: planar, SoA)
//   col[c] + (i / L) * block + (i % L) * size      (L >= 1: AoS is L = 1)
// with size the leaf's bytes, or 1 for byte columns.
constexpr uint32_t kMaxGroups = 8;
enum MixKind : uint32_t { MX_ELEM = 0, MX_BYTES = 1, MX_NULL = 2 };

struct MixGroup {
  uint64_t block;  // bytes between blocks of L records
  uint32_t L;      // records per block (0: planar)
  uint32_t log2L;  // log2 L when L is a power of two, else 64
  uint32_t kind;   // MixKind: whole leaves, byte columns, or NULL (loads 0, stores dropped)
  uint32_t pad;
};

struct MixSide {
  const uint8_t* col[kMaxCols];
  MixGroup g[kMaxGroups];
  uint64_t elem_ok;            // bit f: leaf f moves as one aligned element
  uint8_t grp[kMaxFields];
  uint8_t cidx[kMaxFields];
};

// Views linearised in different orders (Sec. 2): the extents and both
// orders, so that a destination index converts to the source's.
struct Order {
  uint32_t rank;
  uint32_t reorder;               // 0: both sides use the same linear index
  uint32_t src_col_major, dst_col_major;
  uint64_t ext[8];
};

struct MixArgs {
  MixSide src, dst;
  Order order;
  uint64_t n;
  uint32_t nf;
  uint32_t pad;
  uint8_t lsz[kMaxFields];        // log2 of each leaf's bytes
};

// A value-level copy (computed mappings on both sides, integer ChangeType,
// bit-packed codes up to 64 bits, SPLIT trees with computed parts): every
// value is loaded through the source mapping and stored through the
// destination mapping.  Each leaf has its own kind, so one side may mix the
// mapping kinds of a SPLIT tree's parts.
enum GenKind : uint32_t {
  GK_PHYS = 0,        // physical or Bytesplit: the leaf's bits as stored
  GK_CONV = 1,        // ChangeType over a physical mapping of the stored record
  GK_BITS_INT = 2,    // BitPackedIntSoA: col[cidx[f]] is leaf f's bit stream
  GK_BITS_FLOAT = 3,  // BitPackedFloatSoA
  GK_NULL = 4,        // loads give 0, stores are dropped
};

struct GenSide {
  MixSide m;                      // physical groups of the tree, and the bit streams
  uint8_t kind[kMaxFields];       // GenKind of each leaf
  uint8_t bits[kMaxFields];       // code bits (bit-packed leaves)
  uint8_t E[kMaxFields];          // float code exponent bits
  uint8_t M[kMaxFields];          // float code mantissa bits
  uint8_t rne[kMaxFields];        // float codes round to nearest even (else truncate)
  uint8_t stored_t[kMaxFields];   // GK_CONV: stored scalar type of the leaf
};

struct GenArgs {
  GenSide src, dst;
  Order order;
  uint64_t n;
  uint32_t nf;
  uint32_t pad;
  uint8_t user_t[kMaxFields];    // scalar type of each leaf
};

// Pack of planes of 32-bit integers into BitPackedIntSoA streams, one plane
// and one stream per field.
struct PlanarPackArgs {
  const uint8_t* src[kMaxCols];  // field f's plane of n values
  uint8_t* dst[kMaxCols];        // field f's stream of 4 * ceil(n * bits / 32) bytes
  uint64_t n;
  uint32_t nf;
  uint32_t bits;                 // code bits B, 1..32: the low B bits of each value
};

}  // namespace lm
