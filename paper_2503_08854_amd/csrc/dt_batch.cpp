// dt_batch.cpp -- batched uneven patches: one persistent stack launch over
// all patches, optional pre-pass and per-patch top-k, captured once into a
// HIP graph and replayed; plus the launch-shape autotuner and its cache.
#include <string>

#include "dt_internal.hpp"

namespace dtk {

struct BatchGraph {
  std::vector<uint64_t> key;
  std::vector<dt_patch*> patches;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  StackArgs* d_descs = nullptr;
  WorkItem* d_items = nullptr;
  unsigned int* d_counter = nullptr;
  void* d_topk = nullptr;
  size_t n_descs = 0, n_items = 0, topk_bytes = 0;
  // all patches' top-k in two launches (when every patch's tiles fit)
  bool seg = false;
  void* d_seg = nullptr;
  size_t seg_bytes = 0;
  SegTopkArgs seg_args{};
  int seg_tiles = 0;
};

namespace {

struct BatchPlan {
  std::vector<StackArgs> descs;
  std::vector<WorkItem> items;
  int64_t max_n = 0;
  double samples = 0.0;
};

dt_status check_batch(dt_ctx* c, dt_patch* const* patches, const dt_orbits* sets, int32_t n_patches,
                      float* const* d_snr, int32_t k, const int64_t* d_topk_idx, const float* d_topk_val,
                      const int32_t* d_topk_count) {
  if (!c || !c->alive) return fail(DT_E_ARG, "invalid context");
  if (n_patches <= 0 || !patches || !sets) return fail(DT_E_ARG, "need n_patches > 0 and non-NULL arrays");
  if (k < 0 || k > 4096) return fail(DT_E_ARG, "k must be in [0, 4096]");
  if (k > 0 && (!d_snr || !d_topk_idx || !d_topk_val || !d_topk_count))
    return fail(DT_E_ARG, "top-k needs S/N outputs and top-k buffers");
  for (int p = 0; p < n_patches; ++p) {
    if (!patches[p] || patches[p]->ctx != c) return fail(DT_E_ARG, "patch %d is invalid or from another context", p);
    dt_status st = check_orbits(&sets[p]);
    if (st != DT_OK) return st;
    if (k > 0 && sets[p].n > 0 && !d_snr[p]) return fail(DT_E_ARG, "patch %d: top-k needs its S/N output", p);
  }
  return DT_OK;
}

BatchPlan make_plan(dt_patch* const* patches, const dt_orbits* sets, int32_t n_patches, float* const* d_snr,
                    float* const* d_flux, int32_t* const* d_nvalid, int chunk) {
  BatchPlan pl;
  for (int p = 0; p < n_patches; ++p) {
    StackArgs a = stack_args(patches[p], &sets[p]);
    a.snr = d_snr ? d_snr[p] : nullptr;
    a.flux = d_flux ? d_flux[p] : nullptr;
    a.nvalid = d_nvalid ? d_nvalid[p] : nullptr;
    pl.descs.push_back(a);
    pl.max_n = std::max<int64_t>(pl.max_n, sets[p].n);
    pl.samples += (double)sets[p].n * patches[p]->n_exp;
    for (int64_t b = 0; b < sets[p].n; b += chunk)
      pl.items.push_back(WorkItem{p, (int32_t)std::min<int64_t>(chunk, sets[p].n - b), b});
  }
  // largest first (cost = exposures x orbits); ties keep patch / chunk order
  std::stable_sort(pl.items.begin(), pl.items.end(), [&](const WorkItem& x, const WorkItem& y) {
    return (int64_t)patches[x.patch]->n_exp * x.count > (int64_t)patches[y.patch]->n_exp * y.count;
  });
  // the kernel's wavefronts pull 64 orbits at a time, in this order
  std::vector<WorkItem> waves;
  for (const WorkItem& w : pl.items)
    for (int32_t j = 0; j < w.count; j += 64)
      waves.push_back(WorkItem{w.patch, std::min<int32_t>(64, w.count - j), w.begin + j});
  pl.items.swap(waves);
  return pl;
}

int cu_count(int device) {
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n <= 0) n = 256;
  return n;
}

dt_status check_cfg(const dt_batch_config& cfg) {
  if (cfg.chunk < 256 || cfg.chunk > 65536 || cfg.chunk % 256)
    return fail(DT_E_ARG, "chunk must be a multiple of 256 in [256, 65536]");
  if (cfg.wg_per_cu < 1 || cfg.wg_per_cu > 16) return fail(DT_E_ARG, "wg_per_cu must be in [1, 16]");
  return DT_OK;
}

void graph_free(dt_ctx* c, BatchGraph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  ctx_free(c, g->d_descs, sizeof(StackArgs) * g->n_descs);
  ctx_free(c, g->d_items, sizeof(WorkItem) * g->n_items);
  ctx_free(c, g->d_counter, sizeof(unsigned int));
  ctx_free(c, g->d_topk, g->topk_bytes);
  ctx_free(c, g->d_seg, g->seg_bytes);
  delete g;
}

// Enqueue the whole batched sequence on stream s using g's device buffers.
dt_status enqueue(dt_ctx* c, BatchGraph* g, dt_patch* const* patches, const dt_orbits* sets, int32_t n_patches,
                  float* const* d_snr, int32_t k, float thr, int64_t* d_topk_idx, float* d_topk_val,
                  int32_t* d_topk_count, const dt_batch_config& cfg, uint32_t flags, hipStream_t s) {
  if (flags & DT_BATCH_PREPASS) {
    for (int p = 0; p < n_patches; ++p) {
      dt_status st = run_prepass(patches[p], s);
      if (st != DT_OK) return st;
    }
  }
  hipError_t e = launch_batched(g->d_descs, g->d_items, (int)g->n_items, g->d_counter, cfg.wg_per_cu * cu_count(c->device), s);
  if (e != hipSuccess) return hip_fail(e, "batched stack launch");
  if (k > 0 && g->seg) {
    e = launch_topk_segmented(g->seg_args, g->seg_tiles, n_patches, s);
    if (e != hipSuccess) return hip_fail(e, "batched top-k launch");
  } else if (k > 0) {
    for (int p = 0; p < n_patches; ++p) {
      e = launch_topk(d_snr[p], sets[p].n, k, thr, d_topk_idx + (int64_t)p * k, d_topk_val + (int64_t)p * k,
                      d_topk_count + p, g->d_topk, s);
      if (e != hipSuccess) return hip_fail(e, "batched top-k launch");
    }
  }
  return DT_OK;
}

// The tables of the two-launch top-k over all patches, in one device buffer:
// S/N pointers, orbit counts, first tile per patch, patch per tile, and the
// tiles' surviving keys.  Returns false (per-patch top-k) when a patch has
// more survivors than one workgroup selects from.
bool seg_tables(const dt_orbits* sets, int32_t n_patches, int32_t k, float* const* d_snr,
                std::vector<unsigned char>& host, size_t& key_off, int& n_tiles) {
  const int64_t T = topk_seg_tile();
  std::vector<int64_t> first(n_patches + 1, 0);
  for (int p = 0; p < n_patches; ++p) {
    const int64_t t = (sets[p].n + T - 1) / T;
    if (t * k > topk_seg_max_keys()) return false;
    first[p + 1] = first[p] + t;
  }
  if (first[n_patches] > (int64_t)1 << 30) return false;
  n_tiles = (int)first[n_patches];
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t o_snr = 0, o_n = align(o_snr + 8 * (size_t)n_patches), o_first = align(o_n + 8 * (size_t)n_patches);
  const size_t o_tp = align(o_first + 8 * (size_t)(n_patches + 1));
  key_off = align(o_tp + 4 * (size_t)n_tiles);
  host.assign(key_off, 0);
  for (int p = 0; p < n_patches; ++p) {
    const float* sp = d_snr[p];
    std::memcpy(&host[o_snr + 8 * p], &sp, 8);
    std::memcpy(&host[o_n + 8 * p], &sets[p].n, 8);
    for (int64_t t = first[p]; t < first[p + 1]; ++t) {
      const int32_t pp = p;
      std::memcpy(&host[o_tp + 4 * t], &pp, 4);
    }
  }
  std::memcpy(&host[o_first], first.data(), 8 * (size_t)(n_patches + 1));
  return true;
}

// Build (allocate + upload) a BatchGraph's buffers for a plan.
dt_status prepare(dt_ctx* c, const BatchPlan& pl, const dt_orbits* sets, int32_t n_patches, int32_t k,
                  float* const* d_snr, float thr, int64_t* d_topk_idx, float* d_topk_val, int32_t* d_topk_count,
                  BatchGraph** out) {
  BatchGraph* g = new BatchGraph();
  dt_status st = ctx_alloc(c, (void**)&g->d_descs, sizeof(StackArgs) * pl.descs.size(), "batch descriptors");
  g->n_descs = pl.descs.size();
  if (st == DT_OK) st = ctx_alloc(c, (void**)&g->d_items, sizeof(WorkItem) * pl.items.size(), "batch work items");
  g->n_items = pl.items.size();
  if (st == DT_OK) st = ctx_alloc(c, (void**)&g->d_counter, sizeof(unsigned int), "batch counter");
  std::vector<unsigned char> seg_host;
  size_t key_off = 0;
  if (st == DT_OK && k > 0 && seg_tables(sets, n_patches, k, d_snr, seg_host, key_off, g->seg_tiles)) {
    g->seg_bytes = key_off + 8 * (size_t)g->seg_tiles * (size_t)k;
    st = ctx_alloc(c, &g->d_seg, g->seg_bytes, "batch top-k tables");
    if (st == DT_OK) {
      unsigned char* b = static_cast<unsigned char*>(g->d_seg);
      const size_t o_n = ((8 * (size_t)n_patches) + 255) & ~(size_t)255;
      const size_t o_first = (o_n + 8 * (size_t)n_patches + 255) & ~(size_t)255;
      const size_t o_tp = (o_first + 8 * (size_t)(n_patches + 1) + 255) & ~(size_t)255;
      g->seg = true;
      g->seg_args.snr = reinterpret_cast<const float* const*>(b);
      g->seg_args.n = reinterpret_cast<const int64_t*>(b + o_n);
      g->seg_args.tile_first = reinterpret_cast<const int64_t*>(b + o_first);
      g->seg_args.tile_patch = reinterpret_cast<const int32_t*>(b + o_tp);
      g->seg_args.keys = reinterpret_cast<uint64_t*>(b + key_off);
      g->seg_args.thr = thr;
      g->seg_args.k = k;
      g->seg_args.idx = d_topk_idx;
      g->seg_args.val = d_topk_val;
      g->seg_args.cnt = d_topk_count;
    }
  } else if (st == DT_OK && k > 0) {
    g->topk_bytes = topk_scratch_bytes(pl.max_n, k);
    st = ctx_alloc(c, &g->d_topk, g->topk_bytes, "batch top-k scratch");
  }
  if (st != DT_OK) {
    graph_free(c, g);
    return st;
  }
  hipError_t e = hipMemcpyAsync(g->d_descs, pl.descs.data(), sizeof(StackArgs) * pl.descs.size(),
                                hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && !pl.items.empty())
    e = hipMemcpyAsync(g->d_items, pl.items.data(), sizeof(WorkItem) * pl.items.size(), hipMemcpyHostToDevice,
                       c->stream);
  if (e == hipSuccess && g->seg)
    e = hipMemcpyAsync(g->d_seg, seg_host.data(), seg_host.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // host vectors are about to go away
  if (e != hipSuccess) {
    graph_free(c, g);
    return hip_fail(e, "batch upload");
  }
  *out = g;
  return DT_OK;
}

std::vector<uint64_t> make_key(dt_patch* const* patches, const dt_orbits* sets, int32_t n_patches,
                               float* const* d_snr, float* const* d_flux, int32_t* const* d_nvalid, int32_t k,
                               float thr, const int64_t* ti, const float* tv, const int32_t* tc,
                               const dt_batch_config& cfg, uint32_t flags) {
  std::vector<uint64_t> key;
  auto P = [&](const void* q) { key.push_back((uint64_t)(uintptr_t)q); };
  uint32_t tb;
  std::memcpy(&tb, &thr, 4);
  key.push_back(((uint64_t)(uint32_t)k << 32) | tb);
  key.push_back(((uint64_t)(uint32_t)cfg.chunk << 32) | (uint32_t)cfg.wg_per_cu);
  key.push_back(flags);
  P(ti);
  P(tv);
  P(tc);
  for (int p = 0; p < n_patches; ++p) {
    P(patches[p]);
    const dt_orbits& o = sets[p];
    key.push_back((uint64_t)o.n);
    uint64_t ep;
    std::memcpy(&ep, &o.epoch, 8);
    key.push_back(ep);
    P(o.a); P(o.e); P(o.inc); P(o.node); P(o.peri); P(o.m0);
    P(d_snr ? d_snr[p] : nullptr);
    P(d_flux ? d_flux[p] : nullptr);
    P(d_nvalid ? d_nvalid[p] : nullptr);
  }
  return key;
}

std::string shape_key(dt_patch* const* patches, const dt_orbits* sets, int32_t n_patches) {
  double samples = 0.0, maxo = 0.0;
  int maxe = 0;
  for (int p = 0; p < n_patches; ++p) {
    samples += (double)sets[p].n * patches[p]->n_exp;
    maxo = std::max(maxo, (double)sets[p].n);
    maxe = std::max(maxe, (int)patches[p]->n_exp);
  }
  char buf[160];
  std::snprintf(buf, sizeof(buf), "np%d_s%d_o%d_e%d", n_patches, (int)std::lround(std::log2(std::max(samples, 1.0))),
                (int)std::lround(std::log2(std::max(maxo, 1.0))), (int)std::lround(std::log2(std::max(maxe, 1))));
  return buf;
}

bool cache_lookup(const char* path, const std::string& key, dt_batch_config* cfg) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char k[160];
  int chunk, wg;
  double ms;
  bool found = false;
  while (std::fscanf(f, "%159s %d %d %lf", k, &chunk, &wg, &ms) == 4) {
    if (key == k) {
      cfg->chunk = chunk;
      cfg->wg_per_cu = wg;
      found = true;  // the last entry for a key wins
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, const dt_batch_config& cfg, double ms) {
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %.4f\n", key.c_str(), cfg.chunk, cfg.wg_per_cu, ms);
  std::fclose(f);
}

}  // namespace

void batch_graph_drop(dt_ctx* c) {
  if (!c || !c->graph) return;
  (void)hipStreamSynchronize(c->stream);
  graph_free(c, c->graph);
  c->graph = nullptr;
}

bool batch_graph_uses(const dt_ctx* c, const dt_patch* p) {
  if (!c || !c->graph) return false;
  for (dt_patch* q : c->graph->patches)
    if (q == p) return true;
  return false;
}

}  // namespace dtk

using namespace dtk;

extern "C" {

dt_status dt_stack_batched(dt_ctx* c, dt_patch* const* patches, const dt_orbits* sets, int32_t n_patches,
                           float* const* d_snr, float* const* d_flux, int32_t* const* d_nvalid, int32_t k,
                           float threshold, int64_t* d_topk_idx, float* d_topk_val, int32_t* d_topk_count,
                           const dt_batch_config* cfg_in, uint32_t flags) {
  dt_status st = check_batch(c, patches, sets, n_patches, d_snr, k, d_topk_idx, d_topk_val, d_topk_count);
  if (st != DT_OK) return st;
  if (std::isnan(threshold)) return fail(DT_E_ARG, "threshold is NaN");
  if (flags & ~(uint32_t)(DT_BATCH_PREPASS | DT_BATCH_EAGER)) return fail(DT_E_ARG, "unknown flags 0x%x", flags);
  dt_batch_config cfg = cfg_in ? *cfg_in : dt_batch_config{1024, 4};
  st = check_cfg(cfg);
  if (st != DT_OK) return st;
  for (int p = 0; p < n_patches && (flags & DT_BATCH_PREPASS); ++p)
    if (patches[p]->images_released) return fail(DT_E_STATE, "patch %d: images released, no pre-pass possible", p);
  DeviceGuard guard(c->device);
  std::vector<uint64_t> key = make_key(patches, sets, n_patches, d_snr, d_flux, d_nvalid, k, threshold, d_topk_idx,
                                       d_topk_val, d_topk_count, cfg, flags & DT_BATCH_PREPASS);
  if (flags & DT_BATCH_EAGER) {
    BatchPlan pl = make_plan(patches, sets, n_patches, d_snr, d_flux, d_nvalid, cfg.chunk);
    BatchGraph* g = nullptr;
    st = prepare(c, pl, sets, n_patches, k, d_snr, threshold, d_topk_idx, d_topk_val, d_topk_count, &g);
    if (st != DT_OK) return st;
    st = enqueue(c, g, patches, sets, n_patches, d_snr, k, threshold, d_topk_idx, d_topk_val, d_topk_count, cfg,
                 flags, c->stream);
    (void)hipStreamSynchronize(c->stream);  // buffers are freed below
    graph_free(c, g);
    return st;
  }
  if (!c->graph || c->graph->key != key) {
    batch_graph_drop(c);
    BatchPlan pl = make_plan(patches, sets, n_patches, d_snr, d_flux, d_nvalid, cfg.chunk);
    BatchGraph* g = nullptr;
    st = prepare(c, pl, sets, n_patches, k, d_snr, threshold, d_topk_idx, d_topk_val, d_topk_count, &g);
    if (st != DT_OK) return st;
    g->key = key;
    g->patches.assign(patches, patches + n_patches);
    hipError_t e = hipSuccess;
    if (!c->capture_stream) e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      graph_free(c, g);
      return hip_fail(e, "graph capture start");
    }
    st = enqueue(c, g, patches, sets, n_patches, d_snr, k, threshold, d_topk_idx, d_topk_val, d_topk_count, cfg,
                 flags, c->capture_stream);
    e = hipStreamEndCapture(c->capture_stream, &g->graph);
    if (st != DT_OK || e != hipSuccess) {
      graph_free(c, g);
      return st != DT_OK ? st : hip_fail(e, "graph capture end");
    }
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      graph_free(c, g);
      return hip_fail(e, "graph instantiate");
    }
    c->graph = g;
  }
  hipError_t e = hipGraphLaunch(c->graph->exec, c->stream);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  return DT_OK;
}

dt_status dt_autotune_batched(dt_ctx* c, dt_patch* const* patches, const dt_orbits* sets, int32_t n_patches,
                              float* const* d_snr, float* const* d_flux, int32_t* const* d_nvalid,
                              const char* cache_path, dt_batch_config* best, double* best_ms) {
  dt_status st = check_batch(c, patches, sets, n_patches, d_snr, 0, nullptr, nullptr, nullptr);
  if (st != DT_OK) return st;
  if (!best) return fail(DT_E_ARG, "best is NULL");
  std::string skey = shape_key(patches, sets, n_patches);
  if (cache_lookup(cache_path, skey, best)) {
    if (best_ms) *best_ms = -1.0;
    return check_cfg(*best);
  }
  DeviceGuard guard(c->device);
  static const int chunks[] = {256, 512, 1024, 2048, 4096};
  static const int wgs[] = {2, 4, 8};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(DT_E_HIP, "event create failed");
  double best_t = 1e300;
  dt_batch_config bc{1024, 4};
  for (int ch : chunks) {
    BatchPlan pl = make_plan(patches, sets, n_patches, d_snr, d_flux, d_nvalid, ch);
    BatchGraph* g = nullptr;
    st = prepare(c, pl, sets, n_patches, 0, nullptr, 0.f, nullptr, nullptr, nullptr, &g);
    if (st != DT_OK) break;
    for (int wg : wgs) {
      dt_batch_config cfg{ch, wg};
      float ms = 0.f, tot = 0.f;
      hipError_t e = hipSuccess;
      for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, c->stream);
        if (e == hipSuccess)
          e = launch_batched(g->d_descs, g->d_items, (int)g->n_items, g->d_counter, wg * cu_count(c->device),
                             c->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) tot += ms;  // the first run warms caches
      }
      if (e != hipSuccess) {
        st = hip_fail(e, "autotune launch");
        break;
      }
      double t = tot / 2.0;
      if (t < best_t) {
        best_t = t;
        bc = cfg;
      }
    }
    (void)hipStreamSynchronize(c->stream);
    graph_free(c, g);
    if (st != DT_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != DT_OK) return st;
  *best = bc;
  if (best_ms) *best_ms = best_t;
  cache_store(cache_path, skey, bc, best_t);
  return DT_OK;
}

}  // extern "C"
