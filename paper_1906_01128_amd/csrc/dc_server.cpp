// libdc served form: deep-copy+kernel jobs admitted against a device-memory
// budget, copied structures kept resident for reuse, transfers and kernels
// of several jobs in flight at once on separate streams.
//
// Two threads per server. The issue thread admits queued jobs in arrival
// order while slots and memory allow, packs and transfers each new structure
// (dc_deep_copy_to_device), and enqueues the job's out-of-place leaf kernel
// on the job's stream. The completion thread waits for each job's kernel,
// transfers its leaf image back into the caller's buffer and releases the
// job's device memory. Host-to-device and device-to-host transfers therefore
// run at the same time (the link is full duplex) while kernels of other jobs
// execute.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "dc_host.h"

namespace dc {

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Whether [p, p + n) lies in page-locked host memory, which the copy engine
// can write directly. A failed query (pageable memory) leaves an error that
// a later hipGetLastError of this thread would report: it is cleared.
static bool pinned_host(const void* p, uint64_t n) {
  if (!p || !n) return false;
  hipPointerAttribute_t a, b;
  const bool ok = hipPointerGetAttributes(&a, p) == hipSuccess && a.type == hipMemoryTypeHost &&
                  hipPointerGetAttributes(&b, (const uint8_t*)p + n - 1) == hipSuccess && b.type == hipMemoryTypeHost;
  if (!ok) (void)hipGetLastError();
  return ok;
}

// First-fit allocator over one device allocation of the budget's size.
class DevicePool {
 public:
  dc_status init(uint64_t bytes) {
    size_ = bytes;
    DC_HIP(hipMalloc((void**)&base_, bytes));
    free_[0] = bytes;
    return DC_OK;
  }
  ~DevicePool() {
    if (base_) (void)hipFree(base_);
  }
  // returns nullptr when no free range is large enough
  uint8_t* alloc(uint64_t bytes) {
    bytes = align_up(std::max<uint64_t>(bytes, 1), 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const uint64_t off = it->first, sz = it->second;
      free_.erase(it);
      if (sz > bytes) free_[off + bytes] = sz - bytes;
      used_ += bytes;
      sizes_[off] = bytes;
      return base_ + off;
    }
    return nullptr;
  }
  void release(uint8_t* p) {
    if (!p) return;
    const uint64_t off = p - base_;
    auto s = sizes_.find(off);
    if (s == sizes_.end()) return;
    uint64_t lo = off, sz = s->second;
    used_ -= sz;
    sizes_.erase(s);
    auto next = free_.lower_bound(lo);
    if (next != free_.end() && next->first == lo + sz) {
      sz += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == lo) {
        lo = prev->first;
        sz += prev->second;
        free_.erase(prev);
      }
    }
    free_[lo] = sz;
  }
  uint64_t used() const { return used_; }
  uint64_t size() const { return size_; }

 private:
  uint8_t* base_ = nullptr;
  uint64_t size_ = 0, used_ = 0;
  std::map<uint64_t, uint64_t> free_;   // offset -> size
  std::map<uint64_t, uint64_t> sizes_;  // allocated offset -> size
};

struct Resident {
  uint64_t key = 0;
  dc_plan plan = nullptr;
  dc_tree tree = nullptr;
  uint8_t* arena = nullptr;
  uint8_t* scratch = nullptr;
  uint64_t bytes = 0;  // device bytes held
  int refs = 0;
  bool ok = false;             // admitted whole: copy, tiles and ready event all done
  hipEvent_t ready = nullptr;  // recorded after the deep copy and relocation
  std::list<Resident*>::iterator lru;
};

struct Job {
  uint64_t id = 0;
  dc_request req{};
  dc_plan plan = nullptr;  // the job's own plan (none when its key was resident at submit;
                           // dropped when a resident copy is reused)
  Resident* res = nullptr;
  uint8_t* d_out = nullptr;
  uint64_t out_bytes = 0;
  int stream = 0;
  hipEvent_t done_ev = nullptr;
  double t_submit = 0, t_admit = 0, t_done = 0;
  dc_status status = DC_OK;
  bool reused = false, finished = false;
  std::string error;
};

}  // namespace dc

using namespace dc;

struct dc_server_s {
  dc_ctx issue_ctx = nullptr, done_ctx = nullptr;
  dc_schema schema = nullptr;
  dc_server_config cfg{};
  DevicePool pool;
  std::vector<hipStream_t> streams;
  hipStream_t dl_stream = nullptr;  // transfers back, apart from the issue streams
  int next_stream = 0;

  std::mutex mu;
  std::condition_variable cv_issue, cv_done, cv_wait;
  std::deque<Job*> pending;     // submitted, not admitted
  std::deque<Job*> inflight;    // admitted, kernel enqueued, in issue order
  std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
  std::unordered_map<uint64_t, Resident*> residents;
  std::list<Resident*> lru;     // front = most recently used
  uint64_t next_id = 1;
  uint32_t active = 0;          // admitted, not finished
  uint32_t new_structures = 0;  // admissions that copied a new structure
  bool stop = false;
  dc_server_stats stats{};
  std::thread issue_thr, done_thr;

  // ---- helpers (mu held) ----
  void free_resident(Resident* r) {
    residents.erase(r->key);
    lru.erase(r->lru);
    if (r->tree) dc_tree_release(r->tree);
    if (r->plan) dc_plan_destroy(r->plan);
    pool.release(r->arena);
    pool.release(r->scratch);
    if (r->ready) (void)hipEventDestroy(r->ready);
    stats.resident_bytes -= r->bytes;
    delete r;
  }

  // evicts unreferenced residents, least recently used first, until `need`
  // bytes could be allocated; returns false if even that is not enough
  bool make_room(uint64_t need) {
    for (;;) {
      if (pool.size() - pool.used() >= need) {
        uint8_t* probe = pool.alloc(need);
        if (probe) {
          pool.release(probe);
          return true;
        }
      }
      Resident* victim = nullptr;
      for (auto it = lru.rbegin(); it != lru.rend(); ++it)
        if ((*it)->refs == 0) {
          victim = *it;
          break;
        }
      if (!victim) return false;
      // its last kernels finished: refs is 0 only after completion
      free_resident(victim);
      stats.evictions++;
    }
  }

  void finish(Job* j, dc_status st, const std::string& err) {
    j->status = st;
    j->error = err;
    j->t_done = now_s();
    j->finished = true;
    stats.completed++;
    cv_wait.notify_all();
  }

  void issue_loop();
  void done_loop();
  dc_status admit(Job* j, std::unique_lock<std::mutex>& lk);
};

// Admits one job (mu held on entry and exit; released around device work).
dc_status dc_server_s::admit(Job* j, std::unique_lock<std::mutex>& lk) {
  Resident* r = nullptr;
  if (j->req.key) {
    auto it = residents.find(j->req.key);
    if (it != residents.end()) r = it->second;
  }
  if (!r && !j->plan) {
    // resident at submit, evicted since: plan it now (only this thread
    // creates residents, so the key stays absent meanwhile)
    lk.unlock();
    const void* roots[1] = {j->req.root};
    uint64_t ab = 0, sb = 0;
    dc_status st = dc_plan_create(nullptr, schema, j->req.root_type, roots, 1, cfg.align, &j->plan, &ab, &sb);
    dc_plan_info pi;
    if (st == DC_OK && dc_plan_query(j->plan, &pi) == DC_OK && j->req.out_bytes < pi.out_bytes)
      st = fail(DC_E_RANGE, "out_bytes %llu, the leaf image needs %llu", (unsigned long long)j->req.out_bytes,
                (unsigned long long)pi.out_bytes);
    lk.lock();
    if (st != DC_OK) return st;
  }
  const dc_plan p = r ? r->plan : j->plan;
  dc_plan_info info;
  dc_plan_query(p, &info);
  j->out_bytes = info.out_bytes;
  const uint64_t need_out = align_up(std::max<uint64_t>(info.out_bytes, 1), 256);
  const uint64_t need_tree = r ? 0 : align_up(std::max<uint64_t>(info.arena_bytes, 1), 256) +
                                         align_up(info.scratch_bytes, 256);
  // memory for the structure (if new) and for the output
  if (r) {
    r->refs++;  // pin before making room
    j->res = r;
    if (!make_room(need_out)) {
      r->refs--;
      j->res = nullptr;
      return DC_E_BUDGET;  // not now; retried when memory frees up
    }
  } else if (!make_room(need_tree + need_out)) {
    return DC_E_BUDGET;
  }
  const int si = next_stream;
  next_stream = (next_stream + 1) % (int)streams.size();
  hipStream_t s = streams[si];
  j->stream = si;
  j->d_out = pool.alloc(need_out);
  if (!j->d_out) return fail(DC_E_NOMEM, "device pool allocation of %llu bytes", (unsigned long long)need_out);
  if (!r) {
    r = new Resident();
    r->key = j->req.key;
    r->plan = j->plan;
    j->plan = nullptr;
    r->arena = pool.alloc(align_up(std::max<uint64_t>(info.arena_bytes, 1), 256));
    r->scratch = pool.alloc(align_up(info.scratch_bytes, 256));
    r->bytes = need_tree;
    r->refs = 1;
    if (!r->arena || !r->scratch) {
      pool.release(r->arena);
      pool.release(r->scratch);
      delete r;
      return fail(DC_E_NOMEM, "device pool allocation of %llu bytes", (unsigned long long)need_tree);
    }
    (void)hipEventCreateWithFlags(&r->ready, hipEventDisableTiming);
    lru.push_front(r);
    r->lru = lru.begin();
    if (r->key) residents[r->key] = r;
    stats.resident_bytes += r->bytes;
    j->res = r;
    j->reused = false;
    // pack and transfer outside the lock: the host tree is read here
    lk.unlock();
    dc_status st = dc_deep_copy_to_device(issue_ctx, r->plan, r->arena, info.arena_bytes, r->scratch,
                                          info.scratch_bytes, s, &r->tree);
    // the tile list is part of the resident state that later jobs share
    if (st == DC_OK) st = tree_prepare_leaf_tiles(r->tree, s);
    if (st == DC_OK && cfg.fail_copy_at && ++new_structures == cfg.fail_copy_at)
      st = fail(DC_E_HIP, "admission failure injected after the deep copy of new structure %u", cfg.fail_copy_at);
    if (st == DC_OK && hipEventRecord(r->ready, s) != hipSuccess) st = fail(DC_E_HIP, "event record");
    lk.lock();
    // a failed resident is never reused (the issue loop frees it): its copy
    // may be partial and its ready event unrecorded
    if (st != DC_OK) return st;
    r->ok = true;
    stats.h2d_bytes += info.arena_bytes + info.scratch_bytes;
  } else {
    j->res = r;
    j->reused = true;
    stats.reused++;
    lru.erase(r->lru);
    lru.push_front(r);
    r->lru = lru.begin();
    if (j->plan) {
      dc_plan_destroy(j->plan);
      j->plan = nullptr;
    }
    if (hipStreamWaitEvent(s, r->ready, 0) != hipSuccess) return fail(DC_E_HIP, "stream wait");
  }
  stats.peak_bytes = std::max<uint64_t>(stats.peak_bytes, pool.used());
  dc_kernel_args ka{};
  ka.mode = DC_MODE_RESOLVED;
  ka.select = DC_SELECT_ALL_LEAVES;
  ka.iters = 1;
  ka.a = j->req.a;
  ka.b = j->req.b;
  ka.af = j->req.af;
  ka.bf = j->req.bf;
  ka.d_out = j->d_out;
  ka.out_bytes = need_out;
  lk.unlock();
  dc_status st = dc_run_kernel(r->tree, &ka, s);
  if (st == DC_OK && hipEventRecord(j->done_ev, s) != hipSuccess) st = fail(DC_E_HIP, "event record");
  lk.lock();
  if (st != DC_OK) return st;
  stats.kernel_bytes += 2 * info.leaf_bytes;
  return DC_OK;
}

void dc_server_s::issue_loop() {
  (void)hipSetDevice(issue_ctx->device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_issue.wait(lk, [&] { return stop || (!pending.empty() && active < cfg.max_inflight); });
    if (stop) return;
    Job* j = pending.front();
    const dc_status st = admit(j, lk);
    if (st == DC_E_BUDGET) {
      // with nothing in flight every resident structure is evictable and the
      // whole budget can be freed, so this does not happen; otherwise wait for
      // a completion to free memory and retry the same job (arrival order)
      if (active == 0) {
        pending.pop_front();
        finish(j, DC_E_BUDGET, "job does not fit the budget");
        continue;
      }
      const uint64_t done_before = stats.completed;
      cv_issue.wait(lk, [&] { return stop || stats.completed != done_before; });
      continue;
    }
    pending.pop_front();
    if (st != DC_OK) {
      std::string err = dc_last_error();
      // work the failed admission queued (transfers into the resident's
      // memory, a kernel into d_out) must end before that memory is reused
      lk.unlock();
      (void)hipStreamSynchronize(streams[j->stream]);
      lk.lock();
      if (j->res) {
        j->res->refs--;
        if (!j->res->key || !j->res->ok) free_resident(j->res);
        j->res = nullptr;
      }
      pool.release(j->d_out);
      j->d_out = nullptr;
      finish(j, st, err);
      continue;
    }
    j->t_admit = now_s();
    active++;
    stats.batches += inflight.empty() ? 0 : 1;  // admitted while others were on the device
    inflight.push_back(j);
    cv_done.notify_all();
  }
}

void dc_server_s::done_loop() {
  (void)hipSetDevice(done_ctx->device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_done.wait(lk, [&] { return stop || !inflight.empty(); });
    if (stop && inflight.empty()) return;
    // the oldest job whose kernel has finished (poll briefly in issue order)
    Job* j = nullptr;
    for (;;) {
      for (auto it = inflight.begin(); it != inflight.end(); ++it)
        if (hipEventQuery((*it)->done_ev) == hipSuccess) {
          j = *it;
          inflight.erase(it);
          break;
        }
      if (j || stop) break;
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(50));
      lk.lock();
    }
    if (!j) continue;
    lk.unlock();
    // leaf image back into the caller's buffer
    dc_status st = DC_OK;
    std::string err;
    hipStream_t s = dl_stream;
    uint8_t* out = (uint8_t*)j->req.out_host;
    const dc_plan_s* p = j->res->plan;
    // only the leaves' bytes go to the caller: bytes between leaves in the
    // image are never written, as for an out-of-place dc_run_kernel. Into a
    // page-locked buffer each leaf goes by its own copy, straight from the
    // device (one pass over host memory instead of three: copy into the
    // staging ring, read it, write the buffer)
    if (pinned_host(out, j->out_bytes)) {
      for (size_t l = 0; l < p->leaves.size() && st == DC_OK; l++) {
        const uint64_t a = p->leaf_out[l], n = p->leaf_info[l] & ((1ull << kLeafKindShift) - 1);
        if (n && hipMemcpyAsync(out + a, j->d_out + a, n, hipMemcpyDeviceToHost, s) != hipSuccess)
          st = fail(DC_E_HIP, "leaf copy back");
      }
      if (st == DC_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(DC_E_HIP, "leaf copy back");
    } else {
      st = download(done_ctx, j->d_out, 0, j->out_bytes, s, [&](const uint8_t* buf, uint64_t lo, uint64_t hi) {
        // split the chunk among the pool's threads; each copies the leaf
        // bytes that fall in its part
        const uint64_t part = 1ull << 20;
        const int nparts = (int)((hi - lo + part - 1) / part);
        done_ctx->pool->run(nparts, [&](int k) {
          const uint64_t plo = lo + (uint64_t)k * part, phi = std::min(hi, plo + part);
          size_t l = std::upper_bound(p->leaf_out.begin(), p->leaf_out.end(), plo) - p->leaf_out.begin();
          if (l > 0) l--;
          for (; l < p->leaf_out.size() && p->leaf_out[l] < phi; l++) {
            const uint64_t a = std::max(plo, p->leaf_out[l]);
            const uint64_t b =
                std::min<uint64_t>(phi, p->leaf_out[l] + (p->leaf_info[l] & ((1ull << kLeafKindShift) - 1)));
            if (b > a) copy_stream(out + a, buf + (a - lo), b - a);
          }
        });
      });
    }
    if (st == DC_OK) st = tree_check(j->res->tree, s);
    if (st != DC_OK) err = dc_last_error();
    lk.lock();
    stats.d2h_bytes += j->out_bytes;
    pool.release(j->d_out);
    j->d_out = nullptr;
    Resident* r = j->res;
    r->refs--;
    if (r->key == 0 && r->refs == 0) free_resident(r);
    j->res = nullptr;
    active--;
    finish(j, st, err);
    cv_issue.notify_all();
  }
}

extern "C" {

dc_status dc_server_create(dc_ctx ctx, dc_schema schema, const dc_server_config* cfg, dc_server* out) {
  if (!out) return fail(DC_E_INVAL, "dc_server_create: out is null");
  *out = nullptr;
  if (!ctx || !schema || !cfg) return fail(DC_E_INVAL, "dc_server_create: null argument");
  if (cfg->budget_bytes < (1u << 20)) return fail(DC_E_INVAL, "budget of %llu bytes", (unsigned long long)cfg->budget_bytes);
  std::unique_ptr<dc_server_s> s(new dc_server_s());
  s->schema = schema;
  s->cfg = *cfg;
  if (!s->cfg.max_inflight) s->cfg.max_inflight = 8;
  if (!s->cfg.nstreams) s->cfg.nstreams = 4;
  if (!s->cfg.align) s->cfg.align = 64;
  DC_TRY(dc_ctx_create(ctx->device, &s->issue_ctx));
  dc_status st = dc_ctx_create(ctx->device, &s->done_ctx);
  if (st == DC_OK) st = s->pool.init(s->cfg.budget_bytes);
  for (uint32_t i = 0; st == DC_OK && i < s->cfg.nstreams; i++) {
    hipStream_t h;
    if (hipStreamCreateWithFlags(&h, hipStreamNonBlocking) != hipSuccess) st = fail(DC_E_HIP, "stream create");
    else s->streams.push_back(h);
  }
  if (st == DC_OK && hipStreamCreateWithFlags(&s->dl_stream, hipStreamNonBlocking) != hipSuccess)
    st = fail(DC_E_HIP, "stream create");
  if (st != DC_OK) {
    for (hipStream_t h : s->streams) (void)hipStreamDestroy(h);
    if (s->dl_stream) (void)hipStreamDestroy(s->dl_stream);
    if (s->issue_ctx) dc_ctx_destroy(s->issue_ctx);
    if (s->done_ctx) dc_ctx_destroy(s->done_ctx);
    return st;
  }
  dc_server_s* raw = s.release();
  raw->issue_thr = std::thread([raw] { raw->issue_loop(); });
  raw->done_thr = std::thread([raw] { raw->done_loop(); });
  *out = raw;
  return DC_OK;
}

dc_status dc_server_submit(dc_server s, const dc_request* req, uint64_t* id) {
  if (!s || !req || !id || !req->root || !req->out_host) return fail(DC_E_INVAL, "dc_server_submit: null argument");
  auto j = std::make_unique<Job>();
  j->req = *req;
  j->t_submit = now_s();
  // a key that is resident now names an unchanged structure that was
  // planned already: its plan gives the sizes. Otherwise plan now, on the
  // caller's thread: sizes decide admission (a resident evicted before this
  // job's admission is planned then)
  dc_plan_info info{};
  bool resident = false;
  if (req->key) {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->residents.find(req->key);
    if (it != s->residents.end() && it->second->ok) {
      dc_plan_query(it->second->plan, &info);
      resident = true;
    }
  }
  if (!resident) {
    const void* roots[1] = {req->root};
    uint64_t ab = 0, sb = 0;
    DC_TRY(dc_plan_create(nullptr, s->schema, req->root_type, roots, 1, s->cfg.align, &j->plan, &ab, &sb));
    dc_plan_query(j->plan, &info);
  }
  if (req->out_bytes < info.out_bytes) {
    if (j->plan) dc_plan_destroy(j->plan);
    return fail(DC_E_RANGE, "out_bytes %llu, the leaf image needs %llu", (unsigned long long)req->out_bytes,
                (unsigned long long)info.out_bytes);
  }
  const uint64_t need = align_up(std::max<uint64_t>(info.arena_bytes, 1), 256) + align_up(info.scratch_bytes, 256) +
                        align_up(std::max<uint64_t>(info.out_bytes, 1), 256);
  if (need > s->pool.size()) {
    if (j->plan) dc_plan_destroy(j->plan);
    return fail(DC_E_BUDGET, "job needs %llu device bytes, budget is %llu", (unsigned long long)need,
                (unsigned long long)s->pool.size());
  }
  if (hipEventCreateWithFlags(&j->done_ev, hipEventDisableTiming) != hipSuccess) {
    if (j->plan) dc_plan_destroy(j->plan);
    return fail(DC_E_HIP, "event create");
  }
  std::lock_guard<std::mutex> lk(s->mu);
  j->id = s->next_id++;
  *id = j->id;
  s->pending.push_back(j.get());
  s->jobs[j->id] = std::move(j);
  s->stats.submitted++;
  s->cv_issue.notify_all();
  return DC_OK;
}

dc_status dc_server_wait(dc_server s, uint64_t id, double timeout_s, dc_result* out) {
  if (!s || !out) return fail(DC_E_INVAL, "dc_server_wait: null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return fail(DC_E_INVAL, "unknown job %llu", (unsigned long long)id);
  Job* j = it->second.get();
  auto pred = [&] { return j->finished; };
  if (timeout_s < 0) s->cv_wait.wait(lk, pred);
  else if (!s->cv_wait.wait_for(lk, std::chrono::duration<double>(timeout_s), pred))
    return fail(DC_E_STATE, "job %llu not finished within %.3f s", (unsigned long long)id, timeout_s);
  out->id = j->id;
  out->status = j->status;
  out->reused = j->reused ? 1 : 0;
  out->t_submit = j->t_submit;
  out->t_admit = j->t_admit;
  out->t_done = j->t_done;
  out->out_bytes = j->out_bytes;
  const dc_status st = j->status;
  const std::string err = j->error;
  if (j->done_ev) (void)hipEventDestroy(j->done_ev);
  if (j->plan) dc_plan_destroy(j->plan);
  s->jobs.erase(it);
  if (st != DC_OK) return fail(st, "job failed: %s", err.c_str());
  return DC_OK;
}

dc_status dc_server_stats_get(dc_server s, dc_server_stats* out) {
  if (!s || !out) return fail(DC_E_INVAL, "dc_server_stats_get: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  return DC_OK;
}

dc_status dc_server_destroy(dc_server s) {
  if (!s) return fail(DC_E_INVAL, "dc_server_destroy: null server");
  {
    // let admitted work drain, then stop both threads
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_wait.wait(lk, [&] { return s->active == 0; });
    s->stop = true;
  }
  s->cv_issue.notify_all();
  s->cv_done.notify_all();
  s->issue_thr.join();
  s->done_thr.join();
  for (hipStream_t h : s->streams) (void)hipStreamSynchronize(h);
  (void)hipStreamSynchronize(s->dl_stream);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    while (!s->lru.empty()) s->free_resident(s->lru.front());
    for (auto& kv : s->jobs) {
      if (kv.second->done_ev) (void)hipEventDestroy(kv.second->done_ev);
      if (kv.second->plan) dc_plan_destroy(kv.second->plan);
    }
    s->jobs.clear();
  }
  for (hipStream_t h : s->streams) (void)hipStreamDestroy(h);
  (void)hipStreamDestroy(s->dl_stream);
  dc_ctx_destroy(s->issue_ctx);
  dc_ctx_destroy(s->done_ctx);
  delete s;
  return DC_OK;
}

}  // extern "C"
