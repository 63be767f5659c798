// Host parts of libdc and the CPU oracle, run under sanitizers on the CPU
// (tests/test_sanitizers.py builds this with AddressSanitizer +
// UndefinedBehaviorSanitizer, and again with ThreadSanitizer). The HIP
// runtime is the host-only stand-in of mock_hip.cpp.
//
//   plan     the planner against the oracle's walk and layout on every
//            fixture shape (several thousand roots take the chunked parallel
//            walk), at two alignments, selective plans, and the rejected
//            inputs (a pointer into the middle of an array, an array reached
//            twice with another extent) on both sides
//   copy     deep copies through the pinned staging ring into "device"
//            memory, byte for byte against the image the oracle's layout
//            gives, and copies back into the host tree
//   server   the served form: jobs from several submitting threads, keys
//            reused and evicted under a small budget, a failed admission
//
// Exit status 0 when every check passed; a sanitizer report aborts.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <string>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "dc.h"
#include "fx.h"
#include "oracle.h"

static std::atomic<int> g_fail{0};
#define CHECK(c, ...)                                            \
  do {                                                           \
    if (!(c)) {                                                  \
      fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__);       \
      fprintf(stderr, __VA_ARGS__);                              \
      fprintf(stderr, "\n");                                     \
      g_fail++;                                                  \
    }                                                            \
  } while (0)

struct Tree {
  fx_tree* t = nullptr;
  Tree(int shape, uint64_t seed, std::vector<int64_t> params) {
    t = fx_build(shape, seed, params.data(), (int)params.size());
    if (!t) {
      fprintf(stderr, "fixture %d failed\n", shape);
      exit(2);
    }
  }
  ~Tree() { fx_free(t); }
};

static dc_schema make_schema(const fx_tree* t) {
  dc_schema s = nullptr;
  CHECK(dc_schema_create(&s) == DC_OK, "schema create");
  for (uint32_t i = 0; i < t->ntypes; i++) {
    const fx_type& ty = t->types[i];
    std::vector<dc_field> f(ty.nfields);
    for (uint32_t k = 0; k < ty.nfields; k++) {
      const fx_field& x = ty.fields[k];
      f[k] = dc_field{x.offset, x.kind, x.type, x.count_offset, x.count_bytes, x.count_mult, x.fixed_count};
    }
    uint32_t id = 0;
    CHECK(dc_schema_describe(s, ty.name, ty.size, ty.align, f.data(), ty.nfields, &id) == DC_OK, "describe %s: %s",
          ty.name, dc_last_error());
  }
  return s;
}

static std::vector<or_type> oracle_types(const fx_tree* t) {
  std::vector<or_type> v(t->ntypes);
  for (uint32_t i = 0; i < t->ntypes; i++) {
    memset(&v[i], 0, sizeof(or_type));
    v[i].size = t->types[i].size;
    v[i].nfields = t->types[i].nfields;
    for (uint32_t k = 0; k < v[i].nfields; k++) {
      const fx_field& x = t->types[i].fields[k];
      v[i].fields[k] = or_field{x.offset, x.kind, x.type, x.count_offset, x.count_bytes, x.count_mult, x.fixed_count};
    }
  }
  return v;
}

// the plan's objects equal the oracle's, object by object
static void same_layout(const char* what, dc_plan p, const or_copy* c) {
  uint64_t n = 0;
  dc_plan_objects(p, nullptr, 0, &n);
  std::vector<dc_object> objs(n ? n : 1);
  CHECK(dc_plan_objects(p, objs.data(), n, &n) == DC_OK, "%s: objects", what);
  CHECK(n == or_nobjects(c), "%s: %llu objects, oracle %llu", what, (unsigned long long)n,
        (unsigned long long)or_nobjects(c));
  const or_object* o = or_objects(c);
  for (uint64_t i = 0; i < n && i < or_nobjects(c); i++) {
    const dc_object& a = objs[i];
    if (a.host_addr != o[i].host || a.offset != o[i].off || a.bytes != o[i].bytes || a.count != o[i].count ||
        a.kind != o[i].kind) {
      CHECK(false, "%s: object %llu differs", what, (unsigned long long)i);
      break;
    }
  }
  dc_plan_info info;
  dc_plan_query(p, &info);
  CHECK(info.arena_bytes == or_arena_bytes(c), "%s: arena %llu vs %llu", what, (unsigned long long)info.arena_bytes,
        (unsigned long long)or_arena_bytes(c));
  CHECK(info.nslots_nonnull == or_nslots(c), "%s: slots", what);
}

static void check_plan(const char* what, const fx_tree* t, uint64_t align, const uint32_t* follow = nullptr) {
  dc_schema s = make_schema(t);
  std::vector<or_type> ot = oracle_types(t);
  dc_plan p = nullptr;
  uint64_t ab = 0, sb = 0;
  const dc_status st =
      follow ? dc_plan_create_selective(nullptr, s, t->root_type, (const void* const*)t->roots, t->nroots, align,
                                        follow, t->ntypes, &p, &ab, &sb)
             : dc_plan_create(nullptr, s, t->root_type, (const void* const*)t->roots, t->nroots, align, &p, &ab, &sb);
  CHECK(st == DC_OK, "%s: plan: %s", what, dc_last_error());
  or_copy* c = nullptr;
  const int ost = or_deep_copy_selective(ot.data(), t->ntypes, t->root_type, t->roots, t->nroots, align, 1ull << 40,
                                         follow, &c);
  CHECK(ost == OR_OK, "%s: oracle %d", what, ost);
  if (st == DC_OK && ost == OR_OK) same_layout(what, p, c);
  // the oracle's remaining steps on the same copy
  if (ost == OR_OK) {
    CHECK(or_run_kernel(c, 1, 0, nullptr, nullptr, 0, 2, 1.0001, 0.5, 1.0001f, 0.5f, nullptr, 0) == OR_OK,
          "%s: oracle kernel", what);
    std::vector<uint8_t> out(or_out_bytes(c, 1, 0, nullptr, nullptr, 0) + 1);
    CHECK(or_run_kernel(c, 1, 0, nullptr, nullptr, 0, 1, 0.9999, -0.25, 0.9999f, -0.25f, out.data(), out.size()) ==
              OR_OK,
          "%s: oracle out of place", what);
  }
  if (c) or_free(c);
  if (p) dc_plan_destroy(p);
  dc_schema_destroy(s);
}

static int run_plan() {
  fx_set_threads(4);
  {
    Tree a(FX_SHAPE_PLAIN, 1, {16, 1024});
    check_plan("plain", a.t, 64);
    check_plan("plain a128", a.t, 128);
  }
  for (int scheme = 0; scheme < 2; scheme++) {
    Tree a(FX_SHAPE_LINEAR, 2 + scheme, {8, 1000, scheme});
    check_plan(scheme ? "linear LLinit" : "linear allinit", a.t, 64);
  }
  {
    Tree a(FX_SHAPE_DENSE, 4, {4, 10, 3, 0});
    check_plan("dense", a.t, 64);
    Tree b(FX_SHAPE_DENSE, 5, {3, 5, 3, 0});
    check_plan("dense a16", b.t, 16);
  }
  {
    Tree a(FX_SHAPE_WIDE, 6, {8, 8, 1, 3000});
    check_plan("wide", a.t, 64);
  }
  {
    // thousands of roots: the planner walks chunks of roots on its threads
    Tree a(FX_SHAPE_MD, 7, {3000, 1, 12, 4});
    check_plan("md 3000", a.t, 64);
    Tree b(FX_SHAPE_MD, 8, {40, 8, 64, 16});
    check_plan("md 40", b.t, 256);
    // selective: simulations -> cells -> positions only
    const uint32_t follow[2] = {1u, 1u};
    check_plan("md selective", b.t, 64, follow);
  }
  for (int k = 0; k < 6; k++) {
    Tree a(FX_SHAPE_BROOM, 100 + k, {2, 8, 1, 16, 64, 1 << 16});
    check_plan("broom", a.t, 64);
  }
  // rejected inputs: a pointer into the middle of an array; the same array
  // reached again with another extent
  {
    Tree a(FX_SHAPE_MD, 9, {100, 2, 6, 8});
    dc_schema s = make_schema(a.t);
    std::vector<or_type> ot = oracle_types(a.t);
    struct Cell {
      int64_t natoms;
      double *pos, *vel, *force;
    };
    struct Sim {
      int64_t ncells;
      Cell* cells;
    };
    Sim* sim = (Sim*)a.t->roots[70];
    Cell& cell = sim->cells[1];
    double* keep = cell.vel;
    for (int variant = 0; variant < 2; variant++) {
      if (variant == 0) cell.vel = cell.pos + 3;  // interior of another array
      else {
        cell.vel = sim->cells[0].pos;  // an array reached twice...
        cell.natoms = sim->cells[0].natoms + 1;  // ...with another length
      }
      dc_plan p = nullptr;
      uint64_t ab, sb;
      const dc_status st = dc_plan_create(nullptr, s, a.t->root_type, (const void* const*)a.t->roots, a.t->nroots, 64,
                                          &p, &ab, &sb);
      or_copy* c = nullptr;
      const int ost = or_deep_copy(ot.data(), a.t->ntypes, a.t->root_type, a.t->roots, a.t->nroots, 64, 0, &c);
      CHECK(st == (variant ? DC_E_CONFLICT : DC_E_RANGE) && !p, "rejected input %d: status %d", variant, st);
      CHECK(ost == (variant ? OR_E_CONFLICT : OR_E_RANGE), "oracle on rejected input %d: %d", variant, ost);
      if (p) dc_plan_destroy(p);
      if (c) or_free(c);
    }
    cell.vel = keep;
    dc_schema_destroy(s);
  }
  return 0;
}

// the image the oracle's layout gives before relocation: every object's host
// bytes at its offset, zero between
static std::vector<uint8_t> raw_image(const or_copy* c) {
  std::vector<uint8_t> img(or_arena_bytes(c), 0);
  const or_object* o = or_objects(c);
  for (uint64_t i = 0; i < or_nobjects(c); i++)
    if (o[i].bytes) memcpy(img.data() + o[i].off, (const void*)(uintptr_t)o[i].host, o[i].bytes);
  return img;
}

static int run_copy() {
  fx_set_threads(4);
  dc_ctx ctx = nullptr;
  CHECK(dc_ctx_create(0, &ctx) == DC_OK, "ctx: %s", dc_last_error());
  struct Case {
    int shape;
    std::vector<int64_t> params;
  };
  // from a few KB up to several staging chunks of 32 MiB
  const Case cases[] = {{FX_SHAPE_PLAIN, {16, 1024}},
                        {FX_SHAPE_WIDE, {16, 16, 1, 40000}},
                        {FX_SHAPE_MD, {400, 4, 64, 24}},
                        {FX_SHAPE_LINEAR, {4, 3000000, 0}}};
  uint64_t seed = 50;
  for (const Case& k : cases) {
    Tree a(k.shape, seed++, k.params);
    dc_schema s = make_schema(a.t);
    std::vector<or_type> ot = oracle_types(a.t);
    dc_plan p = nullptr;
    uint64_t ab = 0, sb = 0;
    CHECK(dc_plan_create(ctx, s, a.t->root_type, (const void* const*)a.t->roots, a.t->nroots, 64, &p, &ab, &sb) ==
              DC_OK,
          "plan: %s", dc_last_error());
    void *arena = nullptr, *scratch = nullptr;
    CHECK(hipMalloc(&arena, ab) == hipSuccess && hipMalloc(&scratch, sb) == hipSuccess, "device buffers");
    dc_tree tree = nullptr;
    CHECK(dc_stage_to_device(ctx, p, arena, ab, scratch, sb, nullptr, &tree) == DC_OK, "stage: %s", dc_last_error());
    or_copy* c = nullptr;
    CHECK(or_deep_copy(ot.data(), a.t->ntypes, a.t->root_type, a.t->roots, a.t->nroots, 64, (uint64_t)arena, &c) ==
              OR_OK,
          "oracle copy");
    CHECK(hipDeviceSynchronize() == hipSuccess, "sync");
    const std::vector<uint8_t> want = raw_image(c);
    CHECK(want.size() == ab && memcmp(want.data(), arena, ab) == 0, "shape %d: staged image differs", k.shape);
    // copy back (the mock kernels leave the leaves as they were): the host
    // tree keeps its values and its pointers
    std::vector<uint8_t> before = raw_image(c);
    CHECK(dc_attach(tree, nullptr) == DC_OK, "attach");
    CHECK(dc_copy_back(tree, 1, nullptr) == DC_OK, "copy back: %s", dc_last_error());
    CHECK(raw_image(c) == before, "shape %d: copy back changed the host tree", k.shape);
    CHECK(dc_tree_release(tree) == DC_OK, "release");
    or_free(c);
    (void)hipFree(arena);
    (void)hipFree(scratch);
    dc_plan_destroy(p);
    dc_schema_destroy(s);
  }
  dc_ctx_destroy(ctx);
  return 0;
}

// The batched form's host logic: every form enqueues on a staged MD tree (the
// stand-in kernels compute nothing), shapes each form cannot take are
// refused before anything is enqueued, and the autotuner's candidate list
// holds the persistent fused launch at four, six and eight workgroups per CU.
static int run_batch() {
  fx_set_threads(2);
  dc_ctx ctx = nullptr;
  CHECK(dc_ctx_create(0, &ctx) == DC_OK, "ctx: %s", dc_last_error());
  Tree a(FX_SHAPE_MD, 71, {200, 4, 64, 24});
  dc_schema s = make_schema(a.t);
  dc_plan p = nullptr;
  uint64_t ab = 0, sb = 0;
  CHECK(dc_plan_create(ctx, s, a.t->root_type, (const void* const*)a.t->roots, a.t->nroots, 64, &p, &ab, &sb) == DC_OK,
        "plan: %s", dc_last_error());
  void *arena = nullptr, *scratch = nullptr;
  CHECK(hipMalloc(&arena, ab) == hipSuccess && hipMalloc(&scratch, sb) == hipSuccess, "device buffers");
  dc_tree tree = nullptr;
  CHECK(dc_stage_to_device(ctx, p, arena, ab, scratch, sb, nullptr, &tree) == DC_OK, "stage: %s", dc_last_error());
  dc_kernel_args ka{};
  ka.mode = DC_MODE_RESOLVED;
  ka.select = DC_SELECT_ALL_LEAVES;
  ka.iters = 1;
  ka.a = 1.0001;
  ka.b = 0.5;
  const uint32_t both = DC_BATCH_ATTACH | DC_BATCH_DETACH;
  const dc_tune good[] = {{256, 4, 1024, 0, 0}, {256, 1, 1024, 1, 0}, {512, 2, 4096, 2, 0},
                          {256, 1, 512, 3, 0},  {256, 8, 1024, 4, 0}, {256, 4, 2048, 4, 0}};
  for (const dc_tune& tu : good)
    CHECK(dc_batch_run(tree, &ka, &tu, both, nullptr) == DC_OK, "launches %u block %u x %u: %s", tu.launches, tu.block,
          tu.wg_per_cu, dc_last_error());
  const dc_tune bad[] = {{512, 2, 1024, 4, 0}, {256, 9, 1024, 4, 0}, {256, 4, 1024, 5, 0}, {256, 4, 1000, 3, 0}};
  for (const dc_tune& tu : bad)
    CHECK(dc_batch_run(tree, &ka, &tu, both, nullptr) == DC_E_INVAL, "launches %u block %u x %u tile %u accepted",
          tu.launches, tu.block, tu.wg_per_cu, tu.tile_chunks);
  for (uint32_t l : {1u, 3u, 4u}) {
    const dc_tune tu{256, 4, 1024, l, 0};
    CHECK(dc_batch_run(tree, &ka, &tu, both | DC_BATCH_FORCE_WAIT_BOUND, nullptr) == DC_E_INVAL,
          "forced wait bound accepted with launches %u", l);
  }
  dc_tune best{};
  CHECK(dc_autotune(tree, &ka, 1, &best) == DC_OK, "autotune: %s", dc_last_error());
  uint32_t n = 0;
  CHECK(dc_autotune_results(tree, nullptr, nullptr, 0, &n) == DC_OK && n > 0, "autotune results");
  std::vector<dc_tune> tunes(n);
  std::vector<double> us(n);
  CHECK(dc_autotune_results(tree, tunes.data(), us.data(), n, &n) == DC_OK, "autotune results");
  int persistent_fused = 0;
  for (const dc_tune& tu : tunes) {
    CHECK(tu.launches > 2 || tu.launches == 1 || tu.block * tu.wg_per_cu <= 2048, "candidate over 2048 threads per CU");
    if (tu.launches == 4) {
      persistent_fused++;
      CHECK(tu.block == 256 && (tu.wg_per_cu == 4 || tu.wg_per_cu == 6 || tu.wg_per_cu == 8), "persistent fused %u x %u",
            tu.block, tu.wg_per_cu);
    }
  }
  CHECK(persistent_fused == 9, "%d persistent fused candidates", persistent_fused);
  CHECK(dc_tree_check(tree, nullptr) == DC_OK, "check");
  CHECK(dc_tree_release(tree) == DC_OK, "release");
  (void)hipFree(arena);
  (void)hipFree(scratch);
  dc_plan_destroy(p);
  dc_schema_destroy(s);
  dc_ctx_destroy(ctx);
  return 0;
}

// Jobs from `nthreads` submitting threads on one server, each waiting for
// its own jobs; keys shared between threads, a budget small enough to evict.
static int run_server(int nthreads, int jobs_per_thread, uint32_t fail_copy_at) {
  fx_set_threads(2);
  std::vector<Tree*> pool;
  for (int i = 0; i < 6; i++) pool.push_back(new Tree(FX_SHAPE_BROOM, 900 + i, {2, 6, 1, 12, 64, 1 << 18}));
  dc_schema s = make_schema(pool[0]->t);
  dc_ctx ctx = nullptr;
  CHECK(dc_ctx_create(0, &ctx) == DC_OK, "ctx");
  std::vector<uint64_t> out_bytes;
  uint64_t biggest = 0;
  for (Tree* t : pool) {
    dc_plan p;
    uint64_t ab, sb;
    dc_plan_create(nullptr, s, t->t->root_type, (const void* const*)t->t->roots, 1, 64, &p, &ab, &sb);
    dc_plan_info info;
    dc_plan_query(p, &info);
    out_bytes.push_back(info.out_bytes);
    biggest = std::max<uint64_t>(biggest, ab + sb + info.out_bytes + 1024);
    dc_plan_destroy(p);
  }
  dc_server_config cfg{};
  cfg.budget_bytes = std::max<uint64_t>(3 * biggest, 1 << 20);
  cfg.max_inflight = 4;
  cfg.nstreams = 2;
  cfg.fail_copy_at = fail_copy_at;
  dc_server srv = nullptr;
  CHECK(dc_server_create(ctx, s, &cfg, &srv) == DC_OK, "server: %s", dc_last_error());
  std::atomic<int> failed{0}, done{0};
  std::vector<std::thread> th;
  for (int k = 0; k < nthreads; k++)
    th.emplace_back([&, k] {
      std::vector<std::vector<uint8_t>> outs;
      std::vector<uint64_t> ids;
      for (int j = 0; j < jobs_per_thread; j++) {
        const int si = (k * 7 + j * 3) % 6;
        outs.emplace_back(out_bytes[si] + 1);
        dc_request r{};
        r.root_type = pool[si]->t->root_type;
        r.root = pool[si]->t->roots[0];
        r.key = (j % 3) ? (uint64_t)(si + 1) : 0;
        r.a = 1.0001;
        r.b = 0.5;
        r.af = 1.0001f;
        r.bf = 0.5f;
        r.out_host = outs.back().data();
        r.out_bytes = outs.back().size();
        uint64_t id = 0;
        if (dc_server_submit(srv, &r, &id) == DC_OK) ids.push_back(id);
        else failed++;
      }
      for (uint64_t id : ids) {
        dc_result res;
        if (dc_server_wait(srv, id, 60.0, &res) == DC_OK) done++;
        else failed++;
      }
    });
  std::atomic<bool> stop{false};
  std::thread watcher([&] {
    while (!stop) {
      dc_server_stats st;
      dc_server_stats_get(srv, &st);
      std::this_thread::yield();
    }
  });
  for (auto& t : th) t.join();
  stop = true;
  watcher.join();
  dc_server_stats st;
  dc_server_stats_get(srv, &st);
  CHECK(done + failed == nthreads * jobs_per_thread, "jobs lost");
  CHECK(failed == (fail_copy_at ? 1 : 0), "%d jobs failed", failed.load());
  CHECK(st.completed == (uint64_t)(nthreads * jobs_per_thread), "completed %llu", (unsigned long long)st.completed);
  CHECK(st.peak_bytes <= cfg.budget_bytes, "budget exceeded");
  CHECK(dc_server_destroy(srv) == DC_OK, "destroy");
  dc_ctx_destroy(ctx);
  dc_schema_destroy(s);
  for (Tree* t : pool) delete t;
  printf("server: %d threads, %d jobs done, %d failed, %llu reused, %llu evictions\n", nthreads, done.load(),
         failed.load(), (unsigned long long)st.reused, (unsigned long long)st.evictions);
  return 0;
}

int main(int argc, char** argv) {
  for (int i = 1; i < argc; i++) {
    const std::string m = argv[i];
    if (m == "plan") run_plan();
    else if (m == "copy") run_copy();
    else if (m == "batch") run_batch();
    else if (m == "server") {
      run_server(1, 12, 0);
      run_server(4, 16, 0);
      run_server(3, 8, 2);
    } else {
      fprintf(stderr, "unknown mode %s\n", m.c_str());
      return 2;
    }
    printf("%s: %d failures\n", m.c_str(), g_fail.load());
  }
  return g_fail ? 1 : 0;
}
