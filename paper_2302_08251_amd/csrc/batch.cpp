// Batched copy: many views of uneven sizes and mixed mapping pairs moved by
// one persistent kernel, captured once into a hipGraph and replayed.  The
// tile size and the persistent grid are chosen by an autotuner that times
// candidates on the batch itself; results are cached in a JSON file keyed by
// device and batch shape.  The per-view baseline launches each view's own
// copy back to back with its own tuned tile size.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <fstream>
#include <functional>
#include <sstream>

#include "batch.hpp"
#include "host.hpp"
#include "kernels.hpp"

using namespace lm;

struct llama_batch {
  std::vector<const llama_view*> srcs;
  std::vector<llama_view*> dsts;
  uint32_t tile = 0, grid = 0, lds = 0, pv_tile = 0;
  uint32_t tile_map = 0;  // 1: one workgroup per tile, each XCD taking a contiguous run of tiles
  uint64_t total_tiles = 0, alg_bytes = 0;
  double tune_seconds = 0;
  BatchItem* d_items = nullptr;
  uint32_t* d_prefix = nullptr;
  uint32_t* d_tile_view = nullptr;  // view of every tile
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<Plan> pv;
  std::vector<BatchGroup> groups;  // views by leaf size: one kernel each
};

namespace {

llama_status hip_fail(hipError_t e, const char* what) {
  return fail(LLAMA_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

void release_device(llama_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_prefix) (void)hipFree(b->d_prefix);
  if (b->d_tile_view) (void)hipFree(b->d_tile_view);
  b->d_items = nullptr;
  b->d_prefix = nullptr;
  b->d_tile_view = nullptr;
}

// Work list for tile size T: per-view plans, tile prefix sums, max LDS.  The
// views are ordered by copy variant (leaf bytes, relayout mode, layouts) so
// that the persistent workgroups, which walk the tile space in order, keep
// one variant's code hot at a time.
llama_status build_items(llama_batch* b, uint32_t T, std::vector<BatchItem>& items, std::vector<uint32_t>& prefix,
                         uint32_t& lds, std::vector<BatchGroup>* groups = nullptr) {
  const size_t n = b->srcs.size();
  std::vector<BatchItem> plans(n);
  std::vector<uint64_t> tiles(n);
  std::vector<uint64_t> key(n);
  std::vector<uint32_t> plan_lds(n);
  // T = 2: every view's tile grown to the LDS that the largest default tile
  // needs (one launch allocates that much for every workgroup anyway)
  uint32_t fill_cap = 0;
  if (T == 2) {
    for (size_t v = 0; v < n; ++v) {
      Plan p;
      llama_status st = plan_copy(b->srcs[v], b->dsts[v], nullptr, p);
      if (st != LLAMA_OK) return st;
      fill_cap = std::max(fill_cap, p.lds);
    }
  }
  lds = 0;
  for (size_t v = 0; v < n; ++v) {
    Plan p;
    // T = 0: each view's default tile; T = 1: the same, capped to 16 KiB of
    // LDS so that one kernel keeps full occupancy for every view
    llama_launch_params lp{T > 2 ? T : 0u, 0};
    llama_status st = plan_copy(b->srcs[v], b->dsts[v], &lp, p, T == 1 ? 16384u : fill_cap, T == 2);
    if (st != LLAMA_OK) return st;
    if (p.kind != PK_RAW) return fail(LLAMA_ERR_UNSUPPORTED, "batched copies move physical layouts only");
    plans[v] = BatchItem{};
    plans[v].args = p.args;
    plans[v].unit = p.unit;
    plans[v].variant = raw_variant(p.args, p.unit);
    tiles[v] = p.ntiles;
    key[v] = ((uint64_t)p.unit << 40) | ((uint64_t)plans[v].variant << 32) | ((uint64_t)p.args.dst.layout << 24) |
             ((uint64_t)p.args.src.layout << 16) | ((uint64_t)p.args.colrun << 8);
    lds = std::max(lds, p.lds);
    plan_lds[v] = p.lds;
  }
  std::vector<size_t> order(n);
  for (size_t v = 0; v < n; ++v) order[v] = v;
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return key[x] < key[y]; });
  items.assign(n, BatchItem{});
  prefix.assign(n + 1, 0);
  uint64_t total = 0;
  for (size_t k = 0; k < n; ++k) {
    items[k] = plans[order[k]];
    total += tiles[order[k]];
    if (total >= 0x80000000ull) return fail(LLAMA_ERR_INDEX_OVERFLOW, "batch has too many tiles");
    prefix[k + 1] = (uint32_t)total;
  }
  if (groups) {  // runs of one leaf size (the sort key's top field)
    groups->clear();
    for (size_t k = 0; k < n; ++k) {
      if (groups->empty() || groups->back().unit != items[k].unit)
        groups->push_back(BatchGroup{items[k].unit, prefix[k], prefix[k], (uint32_t)k, (uint32_t)k, 0u, 0u});
      BatchGroup& g = groups->back();
      g.t_end = prefix[k + 1];
      g.v_end = (uint32_t)k + 1;
      g.lds = std::max(g.lds, plan_lds[order[k]]);
    }
  }
  return LLAMA_OK;
}

// One launch per leaf-size group; a persistent grid G is shared out by the
// groups' tile counts, and G >= the batch's tiles means one workgroup per
// tile (then M = 1 gives each XCD a contiguous run of the group's tiles).
hipError_t launch_groups(const llama_batch* b, uint32_t G, uint32_t M, hipStream_t st) {
  for (BatchGroup g : b->groups) {
    g.tile_map = M;
    const uint64_t nt = g.t_end - g.t_begin;
    if (nt == 0) continue;
    uint64_t gg = G >= b->total_tiles ? nt : (G * nt + b->total_tiles - 1) / b->total_tiles;
    gg = std::max<uint64_t>(1, std::min<uint64_t>(gg, nt));
    hipError_t e = launch_batch(b->d_items, b->d_prefix, b->d_tile_view, g, (uint32_t)gg, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

llama_status upload(llama_batch* b, uint32_t T) {
  std::vector<BatchItem> items;
  std::vector<uint32_t> prefix;
  uint32_t lds;
  std::vector<BatchGroup> groups;
  llama_status st = build_items(b, T, items, prefix, lds, &groups);
  if (st != LLAMA_OK) return st;
  release_device(b);
  b->groups = groups;
  hipError_t e;
  if ((e = hipMalloc(&b->d_items, items.size() * sizeof(BatchItem))) != hipSuccess) return hip_fail(e, "hipMalloc");
  if ((e = hipMalloc(&b->d_prefix, prefix.size() * sizeof(uint32_t))) != hipSuccess) return hip_fail(e, "hipMalloc");
  if ((e = hipMemcpy(b->d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hipMemcpy");
  if ((e = hipMemcpy(b->d_prefix, prefix.data(), prefix.size() * sizeof(uint32_t), hipMemcpyHostToDevice)) !=
      hipSuccess)
    return hip_fail(e, "hipMemcpy");
  // tile -> view table (4 bytes per tile) for one-workgroup-per-tile
  // launches; very large batches (over 64 Mi tiles) search instead
  std::vector<uint32_t> tv(prefix.back() <= (64u << 20) ? prefix.back() : 0u);
  if (!tv.empty())
    for (size_t k = 0; k + 1 < prefix.size(); ++k)
      std::fill(tv.begin() + prefix[k], tv.begin() + prefix[k + 1], (uint32_t)k);
  if (!tv.empty()) {
    if ((e = hipMalloc(&b->d_tile_view, tv.size() * sizeof(uint32_t))) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = hipMemcpy(b->d_tile_view, tv.data(), tv.size() * sizeof(uint32_t), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "hipMemcpy");
  }
  b->tile = T;
  b->lds = lds;
  b->total_tiles = prefix.back();
  return LLAMA_OK;
}

llama_status capture(llama_batch* b) {
  hipError_t e;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  if ((e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return hip_fail(e, "hipStreamBeginCapture");
  hipError_t le = launch_groups(b, b->grid, b->tile_map, b->cap);
  e = hipStreamEndCapture(b->cap, &b->graph);
  if (le != hipSuccess) return hip_fail(le, "batched launch");
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess)
    return hip_fail(e, "hipGraphInstantiate");
  return LLAMA_OK;
}

llama_status per_view_plans(llama_batch* b, uint32_t T, std::vector<Plan>& out) {
  out.resize(b->srcs.size());
  for (size_t v = 0; v < b->srcs.size(); ++v) {
    llama_launch_params lp{T, 0};
    llama_status st = plan_copy(b->srcs[v], b->dsts[v], &lp, out[v]);
    if (st != LLAMA_OK) return st;
  }
  return LLAMA_OK;
}

// median of `reps` timings (ms) of fn on stream s
template <typename F>
double time_ms(hipStream_t s, int reps, F&& fn) {
  hipEvent_t a, c;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&c);
  std::vector<double> t;
  for (int r = 0; r < reps; ++r) {
    (void)hipEventRecord(a, s);
    fn();
    (void)hipEventRecord(c, s);
    (void)hipEventSynchronize(c);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, c);
    t.push_back(ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(c);
  std::sort(t.begin(), t.end());
  return t[t.size() / 2];
}

std::string device_key(const llama_batch* b) {
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  hipDeviceProp_t prop;
  std::string arch = "gpu";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  for (auto& ch : arch)
    if (ch == '"' || ch == '\\') ch = '_';
  uint64_t recs = 0, h = 1469598103934665603ull;
  auto mix = [&](uint64_t x) { h = (h ^ x) * 1099511628211ull; };
  // every descriptor field that changes a plan: kinds, lanes, flags, code
  // widths and storage types down the inner chain, leaf types, index type
  std::function<void(const MapDesc&)> mix_map = [&](const MapDesc& m) {
    mix(((uint64_t)m.kind << 48) ^ ((uint64_t)m.lanes << 16) ^ m.flags);
    mix(((uint64_t)m.bits << 32) ^ ((uint64_t)m.exp_bits << 16) ^ m.man_bits);
    for (auto t : m.stored) mix(0x100 + (uint64_t)t);
    if (m.inner) mix_map(*m.inner);
    if (m.inner2) mix_map(*m.inner2);
    mix(0xFFFF);
  };
  for (size_t v = 0; v < b->srcs.size(); ++v) {
    recs += b->srcs[v]->n;
    mix(b->srcs[v]->n);
    for (auto t : b->srcs[v]->rec) mix(0x200 + (uint64_t)t);
    mix_map(b->srcs[v]->map);
    mix_map(b->dsts[v]->map);
    mix(((uint64_t)b->srcs[v]->index_type << 8) | (uint64_t)b->dsts[v]->index_type);
  }
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s|cu%d|views%zu|records%llu|shape%016llx", arch.c_str(), cus, b->srcs.size(),
                (unsigned long long)recs, (unsigned long long)h);
  return buf;
}

bool cache_lookup(const char* path, const std::string& key, uint32_t& T, uint32_t& G, uint32_t& P, uint32_t& M) {
  std::ifstream f(path);
  if (!f) return false;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  const size_t k = s.find("\"" + key + "\"");
  if (k == std::string::npos) return false;
  const size_t end = s.find('\n', k);  // the entry's own line
  auto num = [&](const char* name, uint32_t& out) {
    size_t p = s.find(std::string("\"") + name + "\"", k);
    if (p == std::string::npos || p > end) return false;
    p = s.find(':', p);
    if (p == std::string::npos) return false;
    out = (uint32_t)std::strtoul(s.c_str() + p + 1, nullptr, 10);
    return true;
  };
  if (!num("tile_map", M)) M = 0;
  return num("tile_records", T) && num("grid", G) && num("per_view_tile", P) && G > 0 && M <= 1;
}

void cache_store(const char* path, const std::string& key, uint32_t T, uint32_t G, uint32_t P, uint32_t M) {
  // keep the other entries: the file holds one entry per line
  std::vector<std::string> lines;
  {
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line))
      if (line.rfind("  \"", 0) == 0 && line.find("\"" + key + "\"") == std::string::npos) {
        if (!line.empty() && line.back() == ',') line.pop_back();
        lines.push_back(line);
      }
  }
  char buf[512];
  std::snprintf(buf, sizeof(buf),
                "  \"%s\": {\"tile_records\": %u, \"grid\": %u, \"per_view_tile\": %u, \"tile_map\": %u}",
                key.c_str(), T, G, P, M);
  lines.push_back(buf);
  std::ofstream o(path, std::ios::trunc);
  if (!o) return;
  o << "{\n";
  for (size_t i = 0; i < lines.size(); ++i) o << lines[i] << (i + 1 < lines.size() ? ",\n" : "\n");
  o << "}\n";
}

llama_status autotune(llama_batch* b, uint64_t granule, uint32_t& bestT, uint32_t& bestG, uint32_t& bestP,
                      uint32_t& bestM) {
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  // tile candidates: 0 (each view's default tile), 1 (default tile capped to
  // 16 KiB of LDS), 2 (tiles grown to the largest default tile's LDS) and
  // fixed sizes
  std::vector<uint32_t> tiles = {0u, 1u, 2u};
  for (uint32_t T : {512u, 768u, 1024u, 1536u})
    if (T % granule == 0) tiles.push_back(T);
  double best_pv = 1e30;
  bestT = bestG = bestP = bestM = 0;
  struct Cand {
    double ms;
    uint32_t T, G, M;
  };
  std::vector<Cand> cands1;  // first pass: every candidate once
  for (uint32_t T : tiles) {
    if (upload(b, T) != LLAMA_OK) continue;  // e.g. a tile that does not fit in LDS
    // grids of 8, 32, 128 workgroups per CU, or one per tile (0), that one
    // also with each XCD taking a contiguous run of tiles (neighbouring
    // tiles then share lines in one L2)
    const uint32_t cands[5][2] = {{8u, 0u}, {32u, 0u}, {128u, 0u}, {0u, 0u}, {0u, 1u}};
    for (const auto& cm : cands) {
      const uint32_t mult = cm[0], M = cm[1];
      const uint32_t G = (uint32_t)std::max<uint64_t>(
          1, std::min<uint64_t>(mult ? (uint64_t)cus * mult : b->total_tiles, b->total_tiles));
      hipError_t le = hipSuccess;
      auto run = [&]() {
        hipError_t e = launch_groups(b, G, M, b->cap);
        if (e != hipSuccess) le = e;
      };
      run();
      const double ms = time_ms(b->cap, 3, run);
      if (le != hipSuccess) return hip_fail(le, "batched launch");
      cands1.push_back(Cand{ms, T, G, M});
    }
    std::vector<Plan> pv;
    if (T == 1 || T == 2 || per_view_plans(b, T, pv) != LLAMA_OK) continue;  // per-view launches need no cap
    auto run_pv = [&]() {
      for (auto& p : pv) (void)launch_plan(p, b->cap);
    };
    run_pv();
    const double ms = time_ms(b->cap, 2, run_pv);
    if (ms < best_pv) {
      best_pv = ms;
      bestP = T;
    }
  }
  if (cands1.empty()) return fail(LLAMA_ERR_UNSUPPORTED, "no tile size fits every view of the batch");
  // Second pass: the three fastest, timed again in turn (A B C A B C ...) so that
  // a drift of the clocks during tuning does not favour the early candidates
  std::sort(cands1.begin(), cands1.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
  const size_t nc = std::min<size_t>(3, cands1.size());
  std::vector<std::vector<double>> t2(nc);
  for (int rep = 0; rep < 5; ++rep)
    for (size_t c = 0; c < nc; ++c) {
      const Cand& k = cands1[c];
      if (b->tile != k.T || b->groups.empty()) {
        llama_status st = upload(b, k.T);
        if (st != LLAMA_OK) return st;
      }
      hipError_t le = hipSuccess;
      auto run = [&]() {
        hipError_t e = launch_groups(b, k.G, k.M, b->cap);
        if (e != hipSuccess) le = e;
      };
      run();
      t2[c].push_back(time_ms(b->cap, 1, run));
      if (le != hipSuccess) return hip_fail(le, "batched launch");
    }
  double best = 1e30;
  for (size_t c = 0; c < nc; ++c) {
    std::sort(t2[c].begin(), t2[c].end());
    const double ms = t2[c][t2[c].size() / 2];
    if (ms < best) {
      best = ms;
      bestT = cands1[c].T;
      bestG = cands1[c].G;
      bestM = cands1[c].M;
    }
  }
  return LLAMA_OK;
}

}  // namespace

extern "C" {

llama_status llama_batch_create(uint32_t n, const llama_view* const* srcs, llama_view* const* dsts,
                                const char* tune_cache, llama_batch** out) {
  clear_error();
  if (!out) return fail(LLAMA_ERR_INVALID_ARG, "output pointer is NULL");
  *out = nullptr;
  if (n == 0 || !srcs || !dsts) return fail(LLAMA_ERR_INVALID_ARG, "empty batch");
  std::unique_ptr<llama_batch> b(new llama_batch);
  uint64_t granule = 128;
  for (uint32_t v = 0; v < n; ++v) {
    if (!srcs[v] || !dsts[v]) return fail(LLAMA_ERR_INVALID_ARG, "view is NULL");
    if (orders_differ(srcs[v], dsts[v]))
      return fail(LLAMA_ERR_UNSUPPORTED, "view " + std::to_string(v) +
                                             ": batches copy views of one linearisation order only");
    Plan p;
    llama_status st = plan_copy(srcs[v], dsts[v], nullptr, p);
    if (st != LLAMA_OK) return fail(st, "view " + std::to_string(v) + ": " + llama_last_error());
    if (p.kind != PK_RAW) return fail(LLAMA_ERR_UNSUPPORTED, "batched copies move physical layouts only");
    granule = std::max<uint64_t>(granule, tile_granule(p.args.src, p.args.dst));
    if (granule % tile_granule(p.args.src, p.args.dst)) return fail(LLAMA_ERR_UNSUPPORTED, "incompatible AoSoA lanes");
    b->srcs.push_back(srcs[v]);
    b->dsts.push_back(dsts[v]);
    b->alg_bytes += p.alg_bytes;
  }
  // the autotuner runs copies on a private stream: earlier work on any stream
  // (for example the writes that fill the sources) must be complete
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  e = hipStreamCreate(&b->cap);
  if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
  const std::string key = device_key(b.get());
  uint32_t T = 0, G = 0, P = 0, M = 0;
  llama_status st;
  const bool cached = tune_cache && cache_lookup(tune_cache, key, T, G, P, M);
  // a cached entry whose tile sizes no longer plan for these views (for
  // example a tile that does not fit the LDS of wider leaves) is tuned anew
  bool usable = cached;
  if (cached) {
    std::vector<BatchItem> items;
    std::vector<uint32_t> prefix;
    std::vector<Plan> pv;
    uint32_t lds = 0;
    usable = build_items(b.get(), T, items, prefix, lds) == LLAMA_OK && per_view_plans(b.get(), P, pv) == LLAMA_OK;
    clear_error();
  }
  if (!usable) {
    const auto t0 = std::chrono::steady_clock::now();
    if ((st = autotune(b.get(), granule, T, G, P, M)) != LLAMA_OK) {
      release_device(b.get());
      (void)hipStreamDestroy(b->cap);
      return st;
    }
    b->tune_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (tune_cache) cache_store(tune_cache, key, T, G, P, M);
  }
  b->grid = G;
  b->tile_map = M;
  b->pv_tile = P;
  (void)hipStreamSynchronize(b->cap);
  st = upload(b.get(), T);
  if (st == LLAMA_OK) st = per_view_plans(b.get(), P, b->pv);
  if (st == LLAMA_OK) {
    // a cached grid may exceed this batch's tile count
    b->grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(b->grid, b->total_tiles));
    st = capture(b.get());
  }
  if (st != LLAMA_OK) {
    release_device(b.get());
    (void)hipStreamDestroy(b->cap);
    return st;
  }
  *out = b.release();
  return LLAMA_OK;
}

llama_status llama_batch_launch(llama_batch* b, void* stream) {
  clear_error();
  if (!b || !b->exec) return fail(LLAMA_ERR_INVALID_ARG, "batch is NULL");
  hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return LLAMA_OK;
}

llama_status llama_batch_launch_per_view(llama_batch* b, void* stream) {
  clear_error();
  if (!b) return fail(LLAMA_ERR_INVALID_ARG, "batch is NULL");
  for (auto& p : b->pv) {
    llama_status st = launch_plan(p, (hipStream_t)stream);
    if (st != LLAMA_OK) return st;
  }
  return LLAMA_OK;
}

llama_status llama_batch_get_info(const llama_batch* b, llama_batch_info* info) {
  clear_error();
  if (!b || !info) return fail(LLAMA_ERR_INVALID_ARG, "NULL argument");
  info->n_views = (uint32_t)b->srcs.size();
  info->tile_records = b->tile;
  info->grid = b->grid;
  info->total_tiles = b->total_tiles;
  info->algorithmic_bytes = b->alg_bytes;
  info->tune_seconds = b->tune_seconds;
  info->tile_map = b->tile_map;
  info->reserved = 0;
  return LLAMA_OK;
}

llama_status llama_batch_destroy(llama_batch* b) {
  clear_error();
  if (!b) return LLAMA_OK;
  if (b->cap) (void)hipStreamSynchronize(b->cap);
  release_device(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return LLAMA_OK;
}

}  // extern "C"
