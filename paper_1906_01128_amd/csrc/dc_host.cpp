// libdc host core: errors, thread pool, context and pinned staging, schema.
#include <emmintrin.h>
#include <sched.h>
#include <stdlib.h>

#include "dc_host.h"

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

namespace dc {

static thread_local std::string g_err;

dc_status fail(dc_status code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

void clear_error() { g_err.clear(); }

// ---- pool --------------------------------------------------------------------------

Pool::Pool(int nthreads) {
  for (int i = 1; i < nthreads; i++) workers_.emplace_back([this] { loop(); });
}

Pool::~Pool() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  for (auto& w : workers_) w.join();
}

void Pool::loop() {
  uint64_t seen = 0;
  for (;;) {
    const std::function<void(int)>* fn;
    int n;
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
      if (stop_) return;
      seen = gen_;
      fn = fn_;
      n = n_;
    }
    work(seen, fn, n);
  }
}

// Claims and runs items of generation g until none is left. A claim is a
// compare-and-swap on (generation, next index), so a worker that woke for an
// older generation can never take an item of a newer one (whose function it
// does not hold), and the caller's function outlives every item it hands out.
void Pool::work(uint64_t g, const std::function<void(int)>* fn, int n) {
  const uint64_t tag = (g & 0xffffffffull) << 32;
  uint64_t t = ticket_.load();
  for (;;) {
    if ((t & ~0xffffffffull) != tag || (int64_t)(t & 0xffffffffull) >= n) return;
    if (!ticket_.compare_exchange_weak(t, t + 1)) continue;  // t now holds the current value
    (*fn)((int)(t & 0xffffffffull));
    if (done_.fetch_add(1) + 1 == n) {
      std::lock_guard<std::mutex> lk(mu_);
      done_cv_.notify_all();
    }
    t = ticket_.load();
  }
}

void Pool::run(int n, const std::function<void(int)>& fn) {
  if (n <= 0) return;
  if (workers_.empty() || n == 1) {
    for (int i = 0; i < n; i++) fn(i);
    return;
  }
  uint64_t g;
  {
    std::lock_guard<std::mutex> lk(mu_);
    fn_ = &fn;
    n_ = n;
    g = ++gen_;
    done_.store(0);
    ticket_.store((g & 0xffffffffull) << 32);
  }
  cv_.notify_all();
  work(g, &fn, n);
  std::unique_lock<std::mutex> lk(mu_);
  done_cv_.wait(lk, [&] { return done_.load() >= n; });
  fn_ = nullptr;
}

// ---- bulk copies between pageable memory and the pinned ring -----------------------------

// Copies n bytes with non-temporal 16-byte stores (no read-for-ownership of
// the destination, which is written once and not read again on this core).
// On the GPU hosts this moved 125-145 GB/s with 16 threads against 71-75
// GB/s for memcpy, leaving more of the host's memory bandwidth to the DMA
// engines that drain or fill the same ring. Small copies use memcpy.
void copy_stream(void* dst, const void* src, uint64_t n) {
  uint8_t* d = (uint8_t*)dst;
  const uint8_t* s = (const uint8_t*)src;
  if (n < 4096) {
    memcpy(d, s, n);
    return;
  }
  const uint64_t head = (16 - ((uintptr_t)d & 15)) & 15;
  memcpy(d, s, head);
  d += head;
  s += head;
  n -= head;
  uint64_t i = 0;
  for (; i + 64 <= n; i += 64) {
    const __m128i a = _mm_loadu_si128((const __m128i*)(s + i));
    const __m128i b = _mm_loadu_si128((const __m128i*)(s + i + 16));
    const __m128i c = _mm_loadu_si128((const __m128i*)(s + i + 32));
    const __m128i e = _mm_loadu_si128((const __m128i*)(s + i + 48));
    _mm_stream_si128((__m128i*)(d + i), a);
    _mm_stream_si128((__m128i*)(d + i + 16), b);
    _mm_stream_si128((__m128i*)(d + i + 32), c);
    _mm_stream_si128((__m128i*)(d + i + 48), e);
  }
  memcpy(d + i, s + i, n - i);
  _mm_sfence();  // the streamed stores are visible before the caller signals completion
}

// ---- staging ----------------------------------------------------------------------------

// Writes destination range [lo, hi) into buf: the bytes of every piece that
// overlaps it, zeros elsewhere. Split across the pool in 1 MiB parts.
static void pack_range(dc_ctx ctx, uint8_t* buf, uint64_t lo, uint64_t hi, const PieceSource& src) {
  const uint64_t part = 1ull << 20;
  const int nparts = (int)((hi - lo + part - 1) / part);
  ctx->pool->run(nparts, [&](int k) {
    const uint64_t plo = lo + (uint64_t)k * part;
    const uint64_t phi = std::min(hi, plo + part);
    uint64_t cur = plo;
    for (uint64_t i = src.first_ending_after(plo); i < src.n && cur < phi; i++) {
      const Piece pc = src.at(i);
      if (pc.off >= phi) break;
      const uint64_t a = std::max(pc.off, plo);
      const uint64_t b = std::min(pc.off + pc.bytes, phi);
      if (a > cur) memset(buf + (cur - lo), 0, a - cur);
      if (b > a) copy_stream(buf + (a - lo), (const uint8_t*)pc.src + (a - pc.off), b - a);
      cur = std::max(cur, b);
    }
    if (cur < phi) memset(buf + (cur - lo), 0, phi - cur);
  });
}

static dc_status ring_slot(dc_ctx ctx, int* k) {
  *k = ctx->next;
  ctx->next = (ctx->next + 1) % dc_ctx_s::kRing;
  if (ctx->pending[*k]) {
    DC_HIP(hipEventSynchronize(ctx->ev[*k]));
    ctx->pending[*k] = false;
  }
  return DC_OK;
}

dc_status ctx_wait_ring(dc_ctx ctx) {
  for (int k = 0; k < dc_ctx_s::kRing; k++)
    if (ctx->pending[k]) {
      DC_HIP(hipEventSynchronize(ctx->ev[k]));
      ctx->pending[k] = false;
    }
  return DC_OK;
}

// Chunk boundaries of a staged transfer of [lo, hi). ramp_up: sizes double
// from 1 MiB up to the ring's chunk size, so that the first transfer starts
// after a short pack (upload). ramp_down: sizes halve over the last chunks,
// so that the last scatter is short (download). Each copy costs about 10 us
// of DMA setup on top of its bytes, so the ramps are only where they pay.
std::vector<uint64_t> chunk_bounds(uint64_t lo, uint64_t hi, uint64_t max_chunk, bool ramp_up, bool ramp_down) {
  std::vector<uint64_t> b{lo};
  if (max_chunk == 0) max_chunk = 1;
  const uint64_t small = std::min<uint64_t>(1ull << 20, max_chunk);
  uint64_t ramp = ramp_up ? small : max_chunk, pos = lo;
  while (pos < hi) {
    const uint64_t left = hi - pos;
    const uint64_t tail = ramp_down ? std::max(small, (left + 1) / 2) : left;
    uint64_t c = std::min({ramp, max_chunk, tail});
    if (c >= left) c = left;
    pos += c;
    b.push_back(pos);
    ramp = std::min(ramp * 2, max_chunk);  // stays >= 1: the loop always advances
  }
  return b;
}

dc_status upload_source(dc_ctx ctx, uint8_t* dst, uint64_t total, const PieceSource& src, hipStream_t s) {
  const std::vector<uint64_t> bounds = chunk_bounds(0, total, ctx->chunk_bytes, true, false);
  for (size_t i = 0; i + 1 < bounds.size(); i++) {
    const uint64_t lo = bounds[i], hi = bounds[i + 1];
    int k;
    DC_TRY(ring_slot(ctx, &k));
    pack_range(ctx, ctx->ring[k], lo, hi, src);
    DC_HIP(hipMemcpyAsync(dst + lo, ctx->ring[k], hi - lo, hipMemcpyHostToDevice, s));
    DC_HIP(hipEventRecord(ctx->ev[k], s));
    ctx->pending[k] = true;
  }
  return DC_OK;
}

dc_status upload_pieces(dc_ctx ctx, uint8_t* dst, uint64_t total, const std::vector<Piece>& pieces, hipStream_t s) {
  PieceSource src;
  src.n = pieces.size();
  src.at = [&](uint64_t i) { return pieces[i]; };
  src.first_ending_after = [&](uint64_t x) {
    return (uint64_t)(std::upper_bound(pieces.begin(), pieces.end(), x,
                                       [](uint64_t v, const Piece& p) { return v < p.off + p.bytes; }) -
                      pieces.begin());
  };
  return upload_source(ctx, dst, total, src, s);
}

dc_status download(dc_ctx ctx, const uint8_t* src, uint64_t lo, uint64_t hi, hipStream_t s,
                   const std::function<void(const uint8_t*, uint64_t, uint64_t)>& consume) {
  DC_TRY(ctx_wait_ring(ctx));
  const std::vector<uint64_t> bounds =
      hi > lo ? chunk_bounds(lo, hi, ctx->chunk_bytes, false, true) : std::vector<uint64_t>{lo};
  const uint64_t n = bounds.size() - 1;
  const int R = dc_ctx_s::kRing;
  auto issue = [&](uint64_t i) -> dc_status {
    const int k = (int)(i % R);
    const uint64_t a = bounds[i], b = bounds[i + 1];
    DC_HIP(hipMemcpyAsync(ctx->ring[k], src + a, b - a, hipMemcpyDeviceToHost, s));
    DC_HIP(hipEventRecord(ctx->ev[k], s));
    ctx->pending[k] = true;
    return DC_OK;
  };
  for (uint64_t i = 0; i < n && i < (uint64_t)R; i++) DC_TRY(issue(i));
  for (uint64_t i = 0; i < n; i++) {
    const int k = (int)(i % R);
    DC_HIP(hipEventSynchronize(ctx->ev[k]));
    ctx->pending[k] = false;
    const uint64_t a = bounds[i], b = bounds[i + 1];
    consume(ctx->ring[k], a, b);
    if (i + R < n) DC_TRY(issue(i + R));
  }
  return DC_OK;
}

// ---- schema ------------------------------------------------------------------------------

static bool valid_kind(uint32_t k) { return k <= DC_KIND_U8; }

// Threads for packing and scattering: the CPUs this process may run on,
// capped by OMP_NUM_THREADS when that is set and by 32.
int host_threads() {
  int n = 0;
  cpu_set_t set;
  if (sched_getaffinity(0, sizeof(set), &set) == 0) n = CPU_COUNT(&set);
  if (n <= 0) n = (int)std::thread::hardware_concurrency();
  const char* omp = getenv("OMP_NUM_THREADS");
  if (omp && atoi(omp) > 0) n = std::min(n, atoi(omp));
  return std::max(1, std::min(n, 32));
}

}  // namespace dc

using namespace dc;

extern "C" {

const char* dc_last_error(void) { return dc::g_err.c_str(); }

const char* dc_version(void) { return "libdc 0.1 (gfx950)"; }

dc_status dc_ctx_create(int device, dc_ctx* out) {
  if (!out) return fail(DC_E_INVAL, "dc_ctx_create: out is null");
  *out = nullptr;
  int ndev = 0;
  DC_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(DC_E_INVAL, "dc_ctx_create: device %d of %d", device, ndev);
  DC_HIP(hipSetDevice(device));
  dc_ctx c = new dc_ctx_s();
  c->device = device;
  c->ncu = device_cu_count();
  for (int k = 0; k < dc_ctx_s::kRing; k++) {
    if (hipHostMalloc((void**)&c->ring[k], c->chunk_bytes, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev[k], hipEventDisableTiming) != hipSuccess) {
      dc_ctx_destroy(c);
      return fail(DC_E_NOMEM, "dc_ctx_create: pinned staging of %d x %llu bytes", dc_ctx_s::kRing,
                  (unsigned long long)c->chunk_bytes);
    }
  }
  if (hipHostMalloc((void**)&c->small, 4096, hipHostMallocDefault) != hipSuccess) {
    dc_ctx_destroy(c);
    return fail(DC_E_NOMEM, "dc_ctx_create: pinned result buffer");
  }
  if (hipMalloc((void**)&c->dev_hdr, sizeof(DevHeader)) != hipSuccess ||
      hipMemset(c->dev_hdr, 0, sizeof(DevHeader)) != hipSuccess) {
    dc_ctx_destroy(c);
    return fail(DC_E_NOMEM, "dc_ctx_create: device header");
  }
  // the fixed scratch of the no-allocation deep copy: its address on this device
  const dc_status st = noalloc_setup(device);
  if (st != DC_OK) {
    dc_ctx_destroy(c);
    return st;
  }
  c->pool = new Pool(host_threads());
  // Every page of the staging ring written once from the host now: the first
  // host write to each page-locked page costs far more than later ones, and a
  // deep copy packs only into the slots and sizes its chunks reach, so in a
  // fresh context deep copies of a 128 MiB tree ran at 7, 50, 32 and 42 GB/s
  // before settling at about 50 (51 GB/s from the second one on with this).
  c->pool->run(dc_ctx_s::kRing, [&](int k) { memset(c->ring[k], 0, c->chunk_bytes); });
  *out = c;
  clear_error();
  return DC_OK;
}

dc_status dc_ctx_destroy(dc_ctx c) {
  if (!c) return fail(DC_E_INVAL, "dc_ctx_destroy: null context");
  (void)hipSetDevice(c->device);
  for (int k = 0; k < dc_ctx_s::kRing; k++) {
    if (c->pending[k]) (void)hipEventSynchronize(c->ev[k]);
    if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
    if (c->ring[k]) (void)hipHostFree(c->ring[k]);
  }
  if (c->small) (void)hipHostFree(c->small);
  if (c->dev_hdr) (void)hipFree(c->dev_hdr);
  if (c->aux) (void)hipFree(c->aux);
  delete c->pool;
  delete c;
  return DC_OK;
}

dc_status dc_schema_create(dc_schema* out) {
  if (!out) return fail(DC_E_INVAL, "dc_schema_create: out is null");
  *out = new dc_schema_s();
  return DC_OK;
}

dc_status dc_schema_destroy(dc_schema s) {
  if (!s) return fail(DC_E_INVAL, "dc_schema_destroy: null schema");
  delete s;
  return DC_OK;
}

dc_status dc_schema_describe(dc_schema s, const char* name, uint32_t size, uint32_t align, const dc_field* fields,
                             uint32_t nfields, uint32_t* out_type_id) {
  if (!s || (!fields && nfields)) return fail(DC_E_INVAL, "dc_schema_describe: null argument");
  if (s->types.size() >= kMaxTypes) return fail(DC_E_INVAL, "dc_schema_describe: more than %u types", kMaxTypes);
  if (size == 0 || align == 0 || (align & (align - 1)))
    return fail(DC_E_INVAL, "dc_schema_describe(%s): size %u align %u", name ? name : "?", size, align);
  if (nfields > kMaxFields)
    return fail(DC_E_INVAL, "dc_schema_describe(%s): %u pointer fields (max %u)", name ? name : "?", nfields,
                kMaxFields);
  TypeDesc t;
  t.name = name ? name : "";
  t.size = size;
  t.align = align;
  t.described = true;
  t.fields.assign(fields, fields + nfields);
  std::vector<uint8_t> is_ptr(size, 0);
  for (uint32_t i = 0; i < nfields; i++) {
    const dc_field& f = fields[i];
    if (f.offset % 8 || f.offset + 8 > size)
      return fail(DC_E_INVAL, "dc_schema_describe(%s): pointer field %u at offset %u (must be 8-aligned, inside %u)",
                  t.name.c_str(), i, f.offset, size);
    if (!valid_kind(f.kind)) return fail(DC_E_INVAL, "dc_schema_describe(%s): field %u kind %u", t.name.c_str(), i, f.kind);
    if (f.kind == DC_KIND_STRUCT && f.type_id >= kMaxTypes)
      return fail(DC_E_INVAL, "dc_schema_describe(%s): field %u type id %u", t.name.c_str(), i, f.type_id);
    for (uint32_t b = f.offset; b < f.offset + 8; b++) {
      if (is_ptr[b]) return fail(DC_E_INVAL, "dc_schema_describe(%s): pointer fields overlap", t.name.c_str());
      is_ptr[b] = 1;
    }
    if (f.count_offset >= 0) {
      if ((f.count_bytes != 4 && f.count_bytes != 8) || f.count_offset % f.count_bytes ||
          (uint64_t)f.count_offset + f.count_bytes > size)
        return fail(DC_E_INVAL, "dc_schema_describe(%s): field %u count member at %d (%u bytes)", t.name.c_str(), i,
                    f.count_offset, f.count_bytes);
      if (f.count_mult == 0) return fail(DC_E_INVAL, "dc_schema_describe(%s): field %u count_mult 0", t.name.c_str(), i);
    } else if (f.count_offset != -1) {
      return fail(DC_E_INVAL, "dc_schema_describe(%s): field %u count_offset %d", t.name.c_str(), i, f.count_offset);
    }
  }
  for (uint32_t i = 0; i < nfields; i++) {
    const dc_field& f = fields[i];
    if (f.count_offset >= 0)
      for (uint32_t b = (uint32_t)f.count_offset; b < (uint32_t)f.count_offset + f.count_bytes; b++)
        if (is_ptr[b]) return fail(DC_E_INVAL, "dc_schema_describe(%s): count member overlaps a pointer", t.name.c_str());
  }
  t.order.resize(nfields);
  for (uint32_t i = 0; i < nfields; i++) t.order[i] = i;
  std::sort(t.order.begin(), t.order.end(), [&](uint32_t a, uint32_t b) { return fields[a].offset < fields[b].offset; });
  t.pos.resize(nfields);
  for (uint32_t k = 0; k < nfields; k++) t.pos[t.order[k]] = k;
  uint32_t run = 0;
  for (uint32_t k = 0; k <= nfields; k++) {
    const uint32_t end = k < nfields ? fields[t.order[k]].offset : size;
    if (end > run) t.plain_runs.push_back({run, end});
    run = end + 8;
  }
  s->types.push_back(std::move(t));
  if (out_type_id) *out_type_id = (uint32_t)(s->types.size() - 1);
  return DC_OK;
}

}  // extern "C"
