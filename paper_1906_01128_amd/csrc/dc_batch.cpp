// libdc batched form: relocation and the leaf kernel of every structure of a
// plan, as one persistent launch or as three ordinary ones, its capture in a
// HIP graph, and the autotuner that picks between the shapes.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <algorithm>
#include <string>
#include <vector>

#include "dc_host.h"

namespace dc {

#ifndef DC_BUILD_ID
#define DC_BUILD_ID "unversioned"
#endif

// without a tuned choice: the fused launch over 1024-chunk tiles, the fastest
// form measured on the MD workload and one that any plan can take
static const dc_tune kDefaultTune = {256, 4, 1024, 3, 0};
static const uint32_t kDefaultSpin = 1u << 24;  // polls of a persistent workgroup's wait

static dc_status check_tune(const dc_tune& t) {
  if (t.launches > 4) return fail(DC_E_INVAL, "tune.launches %u (0 to 4)", t.launches);
  if (t.block != 256 && t.block != 512 && t.block != 1024) return fail(DC_E_INVAL, "tune.block %u", t.block);
  if (t.wg_per_cu < 1 || t.wg_per_cu > 32) return fail(DC_E_INVAL, "tune.wg_per_cu %u", t.wg_per_cu);
  // the persistent fused launch: 256-thread workgroups, all resident at once
  if (t.launches == 4 && (t.block != 256 || t.wg_per_cu > 8))
    return fail(DC_E_INVAL, "tune.launches 4 takes block 256 and at most 8 workgroups per CU (%u, %u)", t.block,
                t.wg_per_cu);
  if (t.tile_chunks < kTileMinChunks || t.tile_chunks > kTileMaxChunks || (t.tile_chunks & (t.tile_chunks - 1)))
    return fail(DC_E_INVAL, "tune.tile_chunks %u (power of two in %u..%u)", t.tile_chunks, kTileMinChunks,
                kTileMaxChunks);
  return DC_OK;
}

// ---- tuning cache: one JSON object per line -----------------------------------------------

static std::string cache_path() {
  const char* p = getenv("DC_TUNE_CACHE");
  if (p && *p) return p;
  const char* home = getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/dc_tune.json";
}

// workload shape: coarse buckets so that similar trees share a choice
static std::string tune_key(dc_tree t) {
  dc_plan p = t->plan;
  auto bucket = [](uint64_t x) {
    int b = 0;
    while (x > 1) {
      x >>= 1;
      b++;
    }
    return b;
  };
  char buf[160];
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  const char* arch = hipGetDeviceProperties(&prop, dev) == hipSuccess ? prop.gcnArchName : "unknown";
  // the library build is part of the key: a choice measured with other
  // kernels is not reused
  snprintf(buf, sizeof(buf), "%s/%s/cu%d/seg%d/leaf%d/chunk%d/u%d", DC_BUILD_ID, arch, t->ctx->ncu,
           bucket(p->segs.size()), bucket(p->leaves.size()), bucket(p->total_chunks), p->unit_leaves ? 1 : 0);
  return buf;
}

static bool cache_lookup(const std::string& key, dc_tune* out) {
  FILE* f = fopen(cache_path().c_str(), "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    char k[200];
    dc_tune tu{};
    if (sscanf(line, "{\"key\": \"%199[^\"]\", \"block\": %u, \"wg_per_cu\": %u, \"tile_chunks\": %u, \"launches\": %u",
               k, &tu.block, &tu.wg_per_cu, &tu.tile_chunks, &tu.launches) == 5 &&
        key == k && check_tune(tu) == DC_OK) {
      *out = tu;
      found = true;  // the last entry wins
    }
  }
  fclose(f);
  clear_error();
  return found;
}

static void cache_store(const std::string& key, const dc_tune& tu, double us) {
  const std::string path = cache_path();
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) mkdir(path.substr(0, slash).c_str(), 0755);  // may already exist
  FILE* f = fopen(path.c_str(), "a");
  if (!f) return;
  fprintf(f, "{\"key\": \"%s\", \"block\": %u, \"wg_per_cu\": %u, \"tile_chunks\": %u, \"launches\": %u, \"us\": %.1f}\n",
          key.c_str(), tu.block, tu.wg_per_cu, tu.tile_chunks, tu.launches, us);
  fclose(f);
}

static dc_status batch_args(dc_tree t, const dc_kernel_args* a, LeafArgs* la) {
  if (!a) return fail(DC_E_INVAL, "null kernel args");
  if (a->mode != DC_MODE_RESOLVED || a->select != DC_SELECT_ALL_LEAVES || a->iters != 1)
    return fail(DC_E_INVAL, "the batched kernel runs RESOLVED, ALL_LEAVES, one pass");
  memset(la, 0, sizeof(*la));
  la->a = a->a;
  la->b = a->b;
  la->af = a->af;
  la->bf = a->bf;
  la->out = (uint8_t*)a->d_out;
  if (la->out && a->out_bytes < t->plan->out_bytes) return fail(DC_E_RANGE, "d_out smaller than the leaf image");
  if (la->out && ((uintptr_t)la->out & 15)) return fail(DC_E_RANGE, "d_out must be 16-byte aligned");
  return DC_OK;
}

static dc_status resolve_tune(dc_tree t, const dc_tune* tune, dc_tune* out) {
  if (tune) {
    *out = *tune;
    if (!out->block) out->block = kDefaultTune.block;
    if (!out->wg_per_cu) out->wg_per_cu = kDefaultTune.wg_per_cu;
    if (!out->tile_chunks) out->tile_chunks = kDefaultTune.tile_chunks;
  } else if (!cache_lookup(tune_key(t), out)) {
    *out = kDefaultTune;
  }
  return check_tune(*out);
}

// the persistent launch takes one relocation unit with its leaves per item
// when the plan's units own contiguous leaf runs (and no wait is to be forced)
static bool unit_items(dc_tree t, const dc_tune& tu, uint32_t flags) {
  return tu.launches == 0 && t->plan->unit_leaves && !(flags & DC_BATCH_FORCE_WAIT_BOUND);
}

// whether the chosen form reads the tile list
static bool uses_tiles(dc_tree t, const dc_tune& tu, uint32_t flags) {
  return !t->plan->leaves.empty() && !unit_items(t, tu, flags);
}

// enqueue the chosen form on s (the persistent launches after their counter
// reset); under graph capture the tile index must already be built and complete
static dc_status enqueue_batch(dc_tree t, const LeafArgs& la, const dc_tune& tu, uint32_t flags, hipStream_t s,
                               bool capturing = false) {
  dc_plan p = t->plan;
  if (uses_tiles(t, tu, flags) && !capturing) DC_TRY(tree_ensure_tiles(t, tu.tile_chunks, s));
  const uint64_t ntiles = p->leaves.empty() ? 0 : t->ntiles;
  const uint32_t grid = (uint32_t)t->ctx->ncu * tu.wg_per_cu;
  hipError_t e = hipSuccess;
  if (tu.launches == 1) {
    // the same work as three ordinary launches: relocate, every leaf, reverse
    if (flags & DC_BATCH_ATTACH) e = launch_relocate(t->tab, true, s);
    if (e == hipSuccess) e = launch_leaf_tiles(t->tab, la, ntiles, t->tile_T, false, s);
    if (e == hipSuccess && (flags & DC_BATCH_DETACH)) e = launch_relocate(t->tab, false, s);
  } else if (tu.launches == 3) {
    // one launch: every tile relocates the slots of its own leaves
    e = launch_fused(t->tab, la, ntiles, t->tile_T, flags & (DC_BATCH_ATTACH | DC_BATCH_DETACH), s);
  } else if (tu.launches == 4) {
    // the same work in a persistent grid fed by device queues
    e = launch_reset_counters(t->tab.hdr, s);
    if (e == hipSuccess)
      e = launch_fused_persistent(t->tab, la, ntiles, t->tile_T, flags & (DC_BATCH_ATTACH | DC_BATCH_DETACH), grid, s);
  } else if (unit_items(t, tu, flags)) {
    e = launch_reset_counters(t->tab.hdr, s);
    if (e == hipSuccess) e = launch_batch_units(t->tab, la, flags, tu.block, grid, s);
  } else {
    e = launch_reset_counters(t->tab.hdr, s);
    if (e == hipSuccess)
      e = launch_batch(t->tab, la, flags, tu.block, grid, ntiles, tu.spin_limit ? tu.spin_limit : kDefaultSpin, s);
  }
  if (e != hipSuccess) return fail(DC_E_HIP, "batch launch: %s", hipGetErrorString(e));
  return DC_OK;
}

static dc_status batch_state(dc_tree t, uint32_t flags) {
  if (flags & ~(uint32_t)(DC_BATCH_ATTACH | DC_BATCH_DETACH | DC_BATCH_FORCE_WAIT_BOUND))
    return fail(DC_E_INVAL, "flags %#x", flags);
  if ((flags & DC_BATCH_ATTACH) && t->attached) return fail(DC_E_STATE, "ATTACH on an attached tree");
  if (!(flags & DC_BATCH_ATTACH) && !t->attached) return fail(DC_E_STATE, "the tree is staged: pass ATTACH");
  return DC_OK;
}

}  // namespace dc

using namespace dc;

struct dc_graph_s {
  dc_tree tree = nullptr;
  uint32_t tile_T = 0;      // tile size of the tile list the captured launches read
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint8_t* up = nullptr;    // pinned staged image
  uint8_t* down = nullptr;  // pinned arena copy
  uint64_t bytes = 0;       // the arena's size
};

extern "C" {

dc_status dc_batch_run(dc_tree t, const dc_kernel_args* a, const dc_tune* tune, uint32_t flags, void* stream) {
  if (!t || t->released) return fail(DC_E_INVAL, "dc_batch_run: null or released tree");
  DC_TRY(batch_state(t, flags));
  LeafArgs la;
  DC_TRY(batch_args(t, a, &la));
  dc_tune tu;
  DC_TRY(resolve_tune(t, tune, &tu));
  if ((flags & DC_BATCH_FORCE_WAIT_BOUND) && (tu.launches == 1 || tu.launches >= 3))
    return fail(DC_E_INVAL, "FORCE_WAIT_BOUND needs a launch with waits (tune.launches 0 or 2)");
  DC_HIP(hipSetDevice(t->ctx->device));
  DC_TRY(enqueue_batch(t, la, tu, flags, (hipStream_t)stream));
  if (flags & DC_BATCH_DETACH) t->attached = false;
  else t->attached = true;
  return DC_OK;
}

dc_status dc_autotune(dc_tree t, const dc_kernel_args* a, uint32_t reps, dc_tune* out) {
  if (!t || t->released || !out) return fail(DC_E_INVAL, "dc_autotune: null argument");
  if (t->attached) return fail(DC_E_STATE, "dc_autotune needs a staged tree");
  LeafArgs la;
  DC_TRY(batch_args(t, a, &la));
  if (reps == 0) reps = 3;
  DC_HIP(hipSetDevice(t->ctx->device));
  // the candidates run on a stream of their own, which orders nothing with
  // the caller's streams: the tree's deep copy (and whatever else the caller
  // queued on it) must have completed first
  DC_HIP(hipDeviceSynchronize());
  hipStream_t s;
  DC_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    (void)hipStreamDestroy(s);
    return fail(DC_E_HIP, "autotune events");
  }
  const uint32_t flags = DC_BATCH_ATTACH | DC_BATCH_DETACH;
  // Candidates: persistent shapes whose workgroups are all resident at once
  // (at most 2048 threads per compute unit), the per-unit form when the plan
  // allows it, the three-phase form over several tile sizes, three
  // ordinary launches and the fused launch over several tile sizes, and the
  // persistent fused launch at four, six and eight workgroups per CU.
  std::vector<dc_tune> cands;
  const uint32_t phased = t->plan->unit_leaves ? 2u : 0u;
  for (uint32_t block : {256u, 512u, 1024u})
    for (uint32_t wg : {1u, 2u, 4u, 8u}) {
      if (block * wg > 2048 || block * wg < 512) continue;
      if (t->plan->unit_leaves) cands.push_back(dc_tune{block, wg, kDefaultTune.tile_chunks, 0, 0});
      for (uint32_t tile : {4096u, 16384u})
        if (block * wg >= 1024) cands.push_back(dc_tune{block, wg, tile, phased, 0});
    }
  for (uint32_t tile : {512u, 1024u, 2048u, 4096u}) cands.push_back(dc_tune{256, 1, tile, 1, 0});
  for (uint32_t tile : {512u, 1024u, 2048u}) cands.push_back(dc_tune{256, 1, tile, 3, 0});
  for (uint32_t wg : {4u, 6u, 8u})
    for (uint32_t tile : {512u, 1024u, 2048u}) cands.push_back(dc_tune{256, wg, tile, 4, 0});
  clear_error();
  t->tune_table.clear();
  dc_tune best = kDefaultTune;
  double best_us = 1e300;
  dc_status st = DC_OK;
  for (const dc_tune& c : cands) {
    st = enqueue_batch(t, la, c, flags, s);  // warm-up, also builds the tile index
    if (st != DC_OK) break;
    std::vector<float> ms;
    for (uint32_t r = 0; r < reps && st == DC_OK; r++) {
      (void)hipEventRecord(e0, s);
      st = enqueue_batch(t, la, c, flags, s);
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) st = fail(DC_E_HIP, "autotune sync");
      float m = 0;
      (void)hipEventElapsedTime(&m, e0, e1);
      ms.push_back(m);
    }
    if (st != DC_OK) break;
    std::sort(ms.begin(), ms.end());
    const double us = 1000.0 * ms[ms.size() / 2];
    t->tune_table.push_back({c, us});
    if (us < best_us) {
      best_us = us;
      best = c;
    }
  }
  (void)hipStreamSynchronize(s);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  DC_TRY(st);
  DC_TRY(tree_check(t, nullptr));
  cache_store(tune_key(t), best, best_us);
  *out = best;
  return DC_OK;
}

dc_status dc_autotune_results(dc_tree t, dc_tune* tunes, double* us, uint32_t cap, uint32_t* n) {
  if (!t || t->released || !n || (cap && (!tunes || !us))) return fail(DC_E_INVAL, "dc_autotune_results: null argument");
  const uint32_t m = (uint32_t)std::min<size_t>(cap, t->tune_table.size());
  for (uint32_t i = 0; i < m; i++) {
    tunes[i] = t->tune_table[i].first;
    us[i] = t->tune_table[i].second;
  }
  *n = (uint32_t)t->tune_table.size();
  return DC_OK;
}

dc_status dc_graph_create(dc_tree t, const dc_kernel_args* a, const dc_tune* tune, uint32_t flags, int upload,
                          int download, dc_graph* out) {
  if (!out) return fail(DC_E_INVAL, "dc_graph_create: out is null");
  *out = nullptr;
  if (!t || t->released) return fail(DC_E_INVAL, "dc_graph_create: null or released tree");
  if (flags != (DC_BATCH_ATTACH | DC_BATCH_DETACH))
    return fail(DC_E_INVAL, "a graph replays ATTACH|DETACH so that every replay starts from the staged image");
  if (t->attached) return fail(DC_E_STATE, "dc_graph_create needs a staged tree");
  LeafArgs la;
  DC_TRY(batch_args(t, a, &la));
  dc_tune tu;
  DC_TRY(resolve_tune(t, tune, &tu));
  DC_HIP(hipSetDevice(t->ctx->device));
  dc_plan p = t->plan;
  // the capture stream orders nothing with the caller's streams: the tree's
  // deep copy must be complete before the tile list upload and the image
  // read-back below
  DC_HIP(hipDeviceSynchronize());
  hipStream_t cs;
  DC_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  dc_graph g = new dc_graph_s();
  g->tree = t;
  g->bytes = p->arena_bytes;
  auto cleanup = [&](dc_status st) {
    if (cs) (void)hipStreamDestroy(cs);
    dc_graph_destroy(g);
    return st;
  };
  auto hip_fail = [&](hipError_t e, const char* what) {
    return cleanup(fail(DC_E_HIP, "%s: %s", what, hipGetErrorString(e)));
  };
  // the tile index is built outside the graph; the graph only replays the launch
  if (uses_tiles(t, tu, flags)) {
    dc_status st = tree_ensure_tiles(t, tu.tile_chunks, cs);
    if (st != DC_OK) return cleanup(st);
    g->tile_T = tu.tile_chunks;
  }
  hipError_t e;
  if (upload) {
    if (hipHostMalloc((void**)&g->up, std::max<uint64_t>(p->arena_bytes, 1), hipHostMallocDefault) != hipSuccess)
      return cleanup(fail(DC_E_NOMEM, "pinned image of %llu bytes", (unsigned long long)p->arena_bytes));
    // the staged image is what the arena holds now: read it back once
    if (p->arena_bytes &&
        (e = hipMemcpyAsync(g->up, t->arena, p->arena_bytes, hipMemcpyDeviceToHost, cs)) != hipSuccess)
      return hip_fail(e, "image read-back");
  }
  if (download && hipHostMalloc((void**)&g->down, std::max<uint64_t>(p->arena_bytes, 1), hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(DC_E_NOMEM, "pinned image of %llu bytes", (unsigned long long)p->arena_bytes));
  if ((e = hipStreamSynchronize(cs)) != hipSuccess) return hip_fail(e, "graph set-up");
  if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) return hip_fail(e, "begin capture");
  if (upload && p->arena_bytes) (void)hipMemcpyAsync(t->arena, g->up, p->arena_bytes, hipMemcpyHostToDevice, cs);
  dc_status st = enqueue_batch(t, la, tu, flags, cs, true);
  if (download && p->arena_bytes) (void)hipMemcpyAsync(g->down, t->arena, p->arena_bytes, hipMemcpyDeviceToHost, cs);
  e = hipStreamEndCapture(cs, &g->graph);
  (void)hipStreamDestroy(cs);
  cs = nullptr;
  if (st != DC_OK) return cleanup(st);
  if (e != hipSuccess) return cleanup(fail(DC_E_HIP, "graph capture: %s", hipGetErrorString(e)));
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return cleanup(fail(DC_E_HIP, "graph instantiate: %s", hipGetErrorString(e)));
  *out = g;
  return DC_OK;
}

dc_status dc_graph_launch(dc_graph g, void* stream) {
  if (!g || !g->exec) return fail(DC_E_INVAL, "dc_graph_launch: null graph");
  if (g->tree->attached) return fail(DC_E_STATE, "dc_graph_launch needs the tree staged");
  DC_HIP(hipSetDevice(g->tree->ctx->device));
  // the captured launches carry the tile count of the list built at capture;
  // a call with another tile size since then rebuilt the list, so rebuild it
  // back (outside the graph) before the replay reads it
  if (g->tile_T && g->tree->tile_T != g->tile_T) DC_TRY(tree_ensure_tiles(g->tree, g->tile_T, (hipStream_t)stream));
  DC_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return DC_OK;
}

dc_status dc_graph_image(dc_graph g, const void** host, uint64_t* bytes) {
  if (!g || !host || !bytes) return fail(DC_E_INVAL, "dc_graph_image: null argument");
  if (!g->down) return fail(DC_E_STATE, "dc_graph_image: the graph was captured without download");
  *host = g->down;
  *bytes = g->bytes;
  return DC_OK;
}

dc_status dc_graph_destroy(dc_graph g) {
  if (!g) return fail(DC_E_INVAL, "dc_graph_destroy: null graph");
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->up || g->down) (void)hipDeviceSynchronize();
  if (g->up) (void)hipHostFree(g->up);
  if (g->down) (void)hipHostFree(g->down);
  delete g;
  return DC_OK;
}

}  // extern "C"
