// A host-only stand-in for the HIP runtime calls libdc's host code makes, so
// that the host library (planner, staging ring, deep copy, copy back, server
// threads) can run under AddressSanitizer, UndefinedBehaviorSanitizer and
// ThreadSanitizer on a machine without a GPU.
//
// Device memory is host memory. Every stream is a worker thread that runs its
// queued operations (copies, event records, waits on events, kernel launches)
// in order, asynchronously to the caller, as a GPU stream would: a host thread
// that touches a buffer a queued copy still writes is a race the sanitizers
// can see. Kernel launches run nothing (the device kernels are tested on the
// GPU); the device header therefore keeps the clean state the deep copy wrote.
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <set>
#include <thread>

#include "dc_internal.h"

struct EventState {
  std::mutex mu;
  std::condition_variable cv;
  uint64_t recorded = 0;  // generation of the last record call
  uint64_t done = 0;      // generation its stream has reached
};
// queued operations hold the state, so an event may be destroyed while a
// record or a wait on it is still queued, as HIP allows
struct ihipEvent_t {
  std::shared_ptr<EventState> st = std::make_shared<EventState>();
};

struct ihipStream_t {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::function<void()>> q;
  bool running = false, stop = false;
  std::thread th;

  ihipStream_t() {
    th = std::thread([this] {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        cv.wait(lk, [&] { return stop || !q.empty(); });
        if (q.empty()) return;
        std::function<void()> op = std::move(q.front());
        q.pop_front();
        running = true;
        lk.unlock();
        op();
        lk.lock();
        running = false;
        cv.notify_all();
      }
    });
  }
  void push(std::function<void()> op) {
    std::lock_guard<std::mutex> lk(mu);
    q.push_back(std::move(op));
    cv.notify_all();
  }
  void drain() {
    std::unique_lock<std::mutex> lk(mu);
    cv.wait(lk, [&] { return q.empty() && !running; });
  }
  ~ihipStream_t() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
      cv.notify_all();
    }
    th.join();
  }
};

namespace {
std::mutex g_mu;
std::set<ihipStream_t*> g_streams;
ihipStream_t* null_stream() {
  static ihipStream_t* s = [] {
    ihipStream_t* n = new ihipStream_t();  // lives until the process ends
    std::lock_guard<std::mutex> lk(g_mu);
    g_streams.insert(n);
    return n;
  }();
  return s;
}
ihipStream_t* pick(hipStream_t s) { return s ? s : null_stream(); }
void* alloc256(size_t n) {
  void* p = nullptr;
  if (posix_memalign(&p, 256, n ? n : 1)) return nullptr;
  return p;
}
}  // namespace

extern "C" {

const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "mock HIP error"; }
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600* p, int) {
  memset(p, 0, sizeof(*p));
  strcpy(p->gcnArchName, "mock");
  p->multiProcessorCount = 256;
  return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t n) {
  *p = alloc256(n);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) { return hipMalloc(p, n); }
hipError_t hipFree(void* p) {
  free(p);
  return hipSuccess;
}
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipDeviceSynchronize() {
  std::set<ihipStream_t*> all;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    all = g_streams;
  }
  for (ihipStream_t* s : all) s->drain();
  return hipSuccess;
}
hipError_t hipMemset(void* dst, int v, size_t n) {
  (void)hipDeviceSynchronize();
  memset(dst, v, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
  pick(s)->push([=] { memcpy(dst, src, n); });
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  *s = new ihipStream_t();
  std::lock_guard<std::mutex> lk(g_mu);
  g_streams.insert(*s);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  pick(s)->drain();
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  if (!s) return hipErrorInvalidValue;
  s->drain();
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_streams.erase(s);
  }
  delete s;
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = new ihipEvent_t();
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  std::shared_ptr<EventState> st = e->st;
  uint64_t gen;
  {
    std::lock_guard<std::mutex> lk(st->mu);
    gen = ++st->recorded;
  }
  pick(s)->push([st, gen] {
    std::lock_guard<std::mutex> lk(st->mu);
    if (st->done < gen) st->done = gen;
    st->cv.notify_all();
  });
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  std::lock_guard<std::mutex> lk(e->st->mu);
  return e->st->done >= e->st->recorded ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  std::shared_ptr<EventState> st = e->st;
  std::unique_lock<std::mutex> lk(st->mu);
  st->cv.wait(lk, [&] { return st->done >= st->recorded; });
  return hipSuccess;
}
// no host memory is page-locked here: buffers are treated as pageable
hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void*) {
  memset(a, 0, sizeof(*a));
  return hipErrorInvalidValue;
}
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.001f;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
  std::shared_ptr<EventState> st = e->st;
  uint64_t gen;
  {
    std::lock_guard<std::mutex> lk(st->mu);
    gen = st->recorded;
  }
  pick(s)->push([st, gen] {
    std::unique_lock<std::mutex> lk(st->mu);
    st->cv.wait(lk, [&] { return st->done >= gen; });
  });
  return hipSuccess;
}
// graphs are not exercised on the host
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  *g = nullptr;
  return hipErrorNotSupported;
}
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, hipGraphNode_t*, char*, size_t) {
  return hipErrorNotSupported;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }

}  // extern "C"

// The device-side entry points of the library: a launch is an empty
// operation on its stream (ordered like a kernel, computing nothing).
namespace dc {
static hipError_t launch(hipStream_t s) {
  pick(s)->push([] {});
  return hipSuccess;
}
int device_cu_count() { return 256; }
dc_status noalloc_setup(int) { return DC_OK; }
void noalloc_release(int) {}
hipError_t launch_relocate(const Tables&, bool, hipStream_t s) { return launch(s); }
hipError_t launch_scalar(const Tables&, const DevScalar*, const DevScalarHop*, uint32_t, uint64_t*, int,
                         hipStream_t s) {
  return launch(s);
}
hipError_t launch_kick_drift(const Tables&, const KickDriftArgs&, hipStream_t s) { return launch(s); }
hipError_t launch_resolve_chain(const Tables&, const ChainArgs&, hipStream_t s) { return launch(s); }
hipError_t launch_leaf_tiles(const Tables&, const LeafArgs&, uint64_t, uint32_t, bool, hipStream_t s) {
  return launch(s);
}
hipError_t launch_stream_resolved(const Tables&, uint64_t, uint64_t, uint32_t, const LeafArgs&, hipStream_t s) {
  return launch(s);
}
hipError_t launch_stream_deref(const Tables&, const HopArgs&, uint64_t, uint32_t, const LeafArgs&, hipStream_t s) {
  return launch(s);
}
hipError_t launch_batch(const Tables&, const LeafArgs&, uint32_t, uint32_t, uint32_t, uint64_t, uint32_t,
                        hipStream_t s) {
  return launch(s);
}
hipError_t launch_batch_units(const Tables&, const LeafArgs&, uint32_t, uint32_t, uint32_t, hipStream_t s) {
  return launch(s);
}
hipError_t launch_reset_counters(DevHeader*, hipStream_t s) { return launch(s); }
hipError_t launch_leaf_prefix(const uint64_t*, uint64_t, uint64_t*, uint64_t*, hipStream_t s) { return launch(s); }
hipError_t launch_fused(const Tables&, const LeafArgs&, uint64_t, uint32_t, uint32_t, hipStream_t s) { return launch(s); }
hipError_t launch_fused_persistent(const Tables&, const LeafArgs&, uint64_t, uint32_t, uint32_t, uint32_t, hipStream_t s) {
  return launch(s);
}
}  // namespace dc
