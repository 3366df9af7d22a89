// Host-side view representation, validation and copy planning.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "internal.hpp"

namespace lm {

// Deep copy of a mapping descriptor.
struct MapDesc {
  llama_map_kind kind = LLAMA_MAP_AOS;
  uint32_t lanes = 0, bits = 0, exp_bits = 0, man_bits = 0, flags = 0;
  std::vector<llama_scalar> stored;
  std::unique_ptr<MapDesc> inner;   // Bytesplit / ChangeType; Split: part 0
  std::unique_ptr<MapDesc> inner2;  // Split: part 1
};

using Rec = std::vector<llama_scalar>;

uint32_t scalar_size(llama_scalar t);
bool scalar_valid(int t);
bool scalar_is_float(llama_scalar t);
bool scalar_is_signed(llama_scalar t);

llama_status fail(llama_status s, const std::string& msg);
void clear_error();

// Validates `map` for record `rec` and deep-copies it.
llama_status copy_mapping(const Rec& rec, const llama_mapping* map, MapDesc& out, int depth = 0);
uint32_t blob_count(const Rec& rec, const MapDesc& m);
uint64_t blob_size(const Rec& rec, const MapDesc& m, uint64_t n, uint32_t b);
// Mapped bytes of all records (excludes AoS alignment and AoSoA padding; bit
// streams count ceil(n * B / 8) per field).
uint64_t mapped_bytes(const Rec& rec, const MapDesc& m, uint64_t n);

}  // namespace lm

struct llama_view {
  lm::Rec rec;
  lm::MapDesc map;
  uint32_t rank = 1;
  uint64_t extents[8] = {0};
  uint64_t n = 0;
  llama_index_type index_type = LLAMA_IDX_I64;
  bool col_major = false;  // extents linearised column-major (LLAMA_FLAG_COL_MAJOR)
  std::vector<void*> blobs;
  std::vector<uint64_t> blob_bytes;  // bytes the mapping uses per blob
};

namespace lm {

enum PlanKind : uint32_t { PK_RAW = 0, PK_CONV = 1, PK_PACK = 2, PK_UNPACK = 3, PK_ZERO = 4, PK_XPOSE = 5, PK_MIXED = 6, PK_GENERIC = 7,
                          PK_PACK_PLANAR = 8 };

struct Plan {
  PlanKind kind = PK_RAW;
  uint32_t unit = 0;
  uint32_t grid = 0;
  uint32_t lds = 0;
  uint64_t alg_bytes = 0;  // mapped bytes read + mapped bytes written
  uint64_t ntiles = 0;
  TileArgs args{};
  XposeArgs xa{};  // PK_XPOSE
  MixArgs ma{};    // PK_MIXED
  GenArgs ga{};    // PK_GENERIC
  PlanarPackArgs pp{};  // PK_PACK_PLANAR
};

// Builds the device description of a view.  UNSUPPORTED when the tile
// engine does not cover the mapping.
llama_status make_side(const llama_view* v, Side& s, llama_scalar& user_t, llama_scalar& stored_t);

// Tile-size granule (records) for a pair of sides: a multiple of 128 and of
// every AoSoA lane count.
uint64_t tile_granule(const Side& s, const Side& d);
uint32_t tile_lds_bytes(const Side& s, uint32_t tile);

// lds_cap (bytes, 0 = none) bounds the LDS of the default tile choice
// (tile_records == 0): the tile shrinks until it fits; with `fill` it also
// grows to the largest tile within the cap.
llama_status plan_copy(const llama_view* src, const llama_view* dst, const llama_launch_params* p,
                       Plan& plan, uint32_t lds_cap = 0, bool fill = false);
llama_status launch_plan(const Plan& plan, hipStream_t st);

// Zero fill of every mapped byte of dst (a copy from a NULL view).
llama_status plan_zero(const llama_view* dst, Plan& plan);

// FIELD_ACCESS_COUNT or HEATMAP view, and the view its inner mapping forms
// over the leading (data) blobs.
bool instrumented(const llama_view* v);
void inner_view(const llama_view* v, llama_view& out);

// True when two views place some record at different linear positions
// because their linearisation orders differ (more than one extent above 1).
bool orders_differ(const llama_view* a, const llama_view* b);
// Copy between views of different linearisation orders (same extents).
llama_status plan_xpose(const llama_view* src, const llama_view* dst, Plan& plan);
// True when the record's leaves are not all of one size.
bool mixed_record(const Rec& r);
// Per-leaf copy (records of mixed leaf sizes, SPLIT trees against any
// partner, NULL parts), in either linearisation order.
llama_status plan_mixed(const llama_view* src, const llama_view* dst, Plan& plan);
// Value-level copy: each value loaded through the source mapping and stored
// through the destination mapping (computed mappings on both sides, integer
// ChangeType, bit-packed codes up to 64 bits, bit-packed f16 / bf16).
llama_status plan_generic(const llama_view* src, const llama_view* dst, Plan& plan);

// Geometry of one blob of a physical layout for Heatmap counting: records
// come in periods of `period` bytes holding `recs` records each (AoS: one
// record; AoSoA: L; SoA: all n).  Inside a period, run f starts at byte
// run_off[f] and holds the records' elements of 2^run_lsz[f] bytes back to
// back.
struct HeatGeo {
  uint64_t n = 0;
  uint64_t period = 0;
  uint64_t recs = 0;
  uint32_t nruns = 0;
  uint32_t shift = 0;  // log2 of the bytes per counter
  uint64_t run_off[kMaxFields] = {};
  uint32_t run_lsz[kMaxFields] = {};
};

// counts[2f + which] += n for f < nf (FieldAccessCount after a copy).
void launch_field_count(void* counts, uint32_t nf, uint32_t which, uint64_t n, hipStream_t st);
// ctr[q] += accesses touching bytes [q G, q G + G) of the blob (Heatmap).
void launch_heatmap(void* ctr, uint64_t ncounters, const HeatGeo& g, int num_cus, hipStream_t st);

Div make_div(uint32_t d);

}  // namespace lm
