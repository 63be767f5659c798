// libdc's deep copy for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): the relocation tables and the device header live in one fixed
// array per device instead of a caller-owned scratch buffer.
#include <mutex>

#include "dc_host.h"

namespace dc {

// The no-allocation deep copy's scratch. Each device holds its own copy from
// the library's load until the process ends. Host code never passes this name
// to a kernel or a copy: it uses the device address looked up per device
// below (in host code the name only stands for the symbol).
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices];   // the array's address on each device (null until looked up)
bool g_held[kMaxDevices];   // a tree made by the no-allocation copy is alive on that device
}  // namespace

dc_status noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(DC_E_INVAL, "device %d (at most %d devices)", device, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return DC_OK;
  void* ptr = nullptr;
  // `device` is current: the address is that device's copy of the array
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(DC_E_HIP, "no-allocation scratch on device %d: %s", device, hipGetErrorString(e));
  g_ptr[device] = ptr;
  return DC_OK;
}

void noalloc_release(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (device >= 0 && device < kMaxDevices) g_held[device] = false;
}

}  // namespace dc

using namespace dc;

extern "C" {

dc_status dc_deep_copy_to_device_noalloc(dc_ctx ctx, dc_plan plan, void* d_arena, uint64_t arena_bytes, void* stream,
                                         dc_tree* out) {
  if (!out) return fail(DC_E_INVAL, "out is null");
  *out = nullptr;
  if (!ctx || !plan) return fail(DC_E_INVAL, "null context or plan");
  if (plan->sl.total > kNoAllocScratchBytes)
    return fail(DC_E_RANGE, "the plan's tables need %llu bytes; the fixed scratch holds %llu",
                (unsigned long long)plan->sl.total, (unsigned long long)kNoAllocScratchBytes);
  const int dev = ctx->device;
  void* ptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    ptr = g_ptr[dev];  // set when the context was created
    if (!ptr) return fail(DC_E_STATE, "no-allocation scratch not set up on device %d", dev);
    if (g_held[dev])
      return fail(DC_E_STATE, "a tree from the no-allocation copy is still alive on device %d: release it first", dev);
    g_held[dev] = true;
  }
  const dc_status st = deep_copy(ctx, plan, d_arena, arena_bytes, ptr, kNoAllocScratchBytes, stream, true, out);
  if (st != DC_OK) {
    // copies into the array may still be queued: let them finish before
    // another call may overwrite it
    (void)hipDeviceSynchronize();
    noalloc_release(dev);
    return st;
  }
  (*out)->noalloc_dev = dev;
  return DC_OK;
}

}  // extern "C"
