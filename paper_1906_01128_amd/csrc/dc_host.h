// Host-side objects of libdc (C++17). Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <condition_variable>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "dc.h"
#include "dc_internal.h"

namespace dc {

// ---- errors -----------------------------------------------------------------------
dc_status fail(dc_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define DC_HIP(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return ::dc::fail(DC_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define DC_TRY(expr)              \
  do {                            \
    dc_status s_ = (expr);        \
    if (s_ != DC_OK) return s_;   \
  } while (0)

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Allocator whose resize leaves new elements default-initialised (no zero
// fill), for the planner's large tables that are written in parallel right
// after they are sized.
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept {
    ::new ((void*)p) U;
  }
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    ::new ((void*)p) U(std::forward<A>(a)...);
  }
};
template <class T>
using bigvec = std::vector<T, NoInitAlloc<T>>;

// ---- a small fork-join pool -------------------------------------------------------------
class Pool {
 public:
  explicit Pool(int nthreads);
  ~Pool();
  int size() const { return (int)workers_.size() + 1; }
  // runs fn(i) for every i in [0, n); the caller takes part; returns when all are done
  void run(int n, const std::function<void(int)>& fn);

 private:
  void loop();
  void work(uint64_t g, const std::function<void(int)>* fn, int n);
  std::vector<std::thread> workers_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(int)>* fn_ = nullptr;
  int n_ = 0;
  std::atomic<uint64_t> ticket_{0};  // (generation << 32) | next item
  std::atomic<int> done_{0};         // items of the current generation finished
  uint64_t gen_ = 0;
  bool stop_ = false;
};

// host threads a pool should use: the CPUs this process may run on, capped
// by OMP_NUM_THREADS and at 32
int host_threads();

// ---- staging: pinned ring of chunks between pageable host memory and the device ---------------
// A "piece" is a run of bytes at a fixed destination offset; gaps between
// pieces are written as zeros.
struct Piece {
  uint64_t off;       // destination offset
  const void* src;    // host bytes
  uint64_t bytes;
};

struct dc_ctx_impl;

}  // namespace dc

struct dc_ctx_s {
  int device = 0;
  int ncu = 256;
  // pinned staging: 8 chunks of 32 MiB, so that packing one chunk overlaps
  // the transfer of the previous ones. Each copy costs about 10 us of DMA
  // setup: the 134 MB Linear tree moved at 51.6 GB/s each way with 32 MiB
  // chunks against 49.9 / 49.3 with 16 MiB (57.3 for one pinned 1 GiB copy).
  static constexpr int kRing = 8;
  uint64_t chunk_bytes = 32ull << 20;
  uint8_t* ring[kRing] = {};
  hipEvent_t ev[kRing] = {};
  bool pending[kRing] = {};
  int next = 0;
  uint8_t* small = nullptr;  // pinned scratch for header reads
  dc::DevHeader* dev_hdr = nullptr;  // device header for kernels outside a tree
  uint8_t* aux = nullptr;            // device buffer for per-call descriptors (grows)
  uint64_t aux_bytes = 0;
  dc::Pool* pool = nullptr;
};

namespace dc {

// Copies `pieces` (sorted by off, non-overlapping) into device memory
// [0, total) at `dst`: packed through the pinned ring by the pool, zeros
// between pieces, each chunk sent with hipMemcpyAsync on `s` while the next
// one is packed.
dc_status upload_pieces(dc_ctx ctx, uint8_t* dst, uint64_t total, const std::vector<Piece>& pieces, hipStream_t s);
// Same, with pieces given by a callback for the objects of a plan (used for
// the arena: millions of objects, described without building a vector).
struct PieceSource {
  uint64_t n;
  std::function<Piece(uint64_t)> at;  // pieces in offset order
  std::function<uint64_t(uint64_t)> first_ending_after;  // first piece with off + bytes > x
};
dc_status upload_source(dc_ctx ctx, uint8_t* dst, uint64_t total, const PieceSource& src, hipStream_t s);
// memcpy for bulk data: non-temporal stores above 4 KiB (see dc_host.cpp)
void copy_stream(void* dst, const void* src, uint64_t n);
// Chunk boundaries of a staged transfer of [lo, hi): with ramp_up 1 MiB
// first, doubling up to max_chunk; with ramp_down halving again over the last
// chunks; max_chunk in between.
std::vector<uint64_t> chunk_bounds(uint64_t lo, uint64_t hi, uint64_t max_chunk, bool ramp_up, bool ramp_down);
// Transfers device [lo, hi) back through the ring; consume(buf, clo, chi)
// is called, in order, for each chunk [clo, chi) as it lands.
dc_status download(dc_ctx ctx, const uint8_t* src, uint64_t lo, uint64_t hi, hipStream_t s,
                   const std::function<void(const uint8_t*, uint64_t, uint64_t)>& consume);
dc_status ctx_wait_ring(dc_ctx ctx);

// ---- schema -----------------------------------------------------------------------
struct TypeDesc {
  std::string name;
  uint32_t size = 0, align = 1;
  bool described = false;
  std::vector<dc_field> fields;   // as given
  std::vector<uint32_t> order;    // field indices by ascending offset
  std::vector<uint32_t> pos;      // position of field i in `order`
  std::vector<std::pair<uint32_t, uint32_t>> plain_runs;  // [lo, hi) byte runs that are not pointers
  uint32_t follow = 0xFFFFFFFFu;  // per field (list order): followed by the walk
};

}  // namespace dc

struct dc_schema_s {
  std::vector<dc::TypeDesc> types;
};

namespace dc {

// ---- plan -------------------------------------------------------------------------
struct Obj {
  uint64_t host;
  uint64_t off;
  uint64_t bytes;
  uint64_t count;
  uint32_t kind;
  uint32_t type;
  uint32_t parent;      // first discoverer, kNone for a root
  uint32_t sobj;        // index among slotted struct arrays, kNone otherwise
  uint64_t parent_rel;  // offset of the discovering slot inside the parent
  uint64_t slot;        // index of the discovering slot in the slot enumeration (roots: ~0)
  uint32_t depth;       // pointer hops from the root
  uint32_t pad;
};

class FlatMap {  // host address -> object index
 public:
  void reserve(uint64_t n);
  uint32_t find(uint64_t key) const;
  void insert(uint64_t key, uint32_t val);

 private:
  void grow();
  std::vector<uint64_t> keys_;
  std::vector<uint32_t> vals_;
  uint64_t mask_ = 0, n_ = 0;
};

}  // namespace dc

struct dc_plan_s {
  std::vector<dc::TypeDesc> types;
  std::vector<dc::DevType> dev_types;
  uint32_t root_type = 0;
  uint64_t align = 64;
  std::vector<uint64_t> roots;  // host addresses as given
  std::vector<uint32_t> root_obj;
  dc::bigvec<dc::Obj> objs;
  // slotted struct arrays (arena order) and their slot prefix
  std::vector<dc::DevSObj> sobj;
  std::vector<uint64_t> sobj_pre;
  dc::bigvec<uint32_t> slot_target;  // per slot: target object or kNone
  // relocation units
  std::vector<dc::DevSeg> segs;
  std::vector<dc::DevTarget> tgts;
  dc::bigvec<uint16_t> slot_tix;  // per slot: index of its target in its unit's targets
  // leaves (FP32/FP64 arrays with >= 1 element), arena order
  dc::bigvec<uint32_t> leaves;
  dc::bigvec<uint64_t> leaf_pre, leaf_info, leaf_slot, leaf_out;
  dc::bigvec<uint64_t> leaf_dev;       // per leaf: its planned arena offset
  dc::bigvec<uint32_t> leaf_tgt;       // per leaf: global index of its parent slot's target entry
  std::vector<dc::DevResid> resid;     // slots that are no leaf's discovering slot
  uint64_t out_bytes = 0, total_chunks = 0, total_hops = 0;
  // every relocation unit's slots discover a contiguous run of leaves (in
  // leaf order), recorded in its DevSeg: the persistent launch can then run
  // each unit's attach, its leaves and its detach as one work item
  bool unit_leaves = false;
  uint64_t max_unit_leaf_chunks = 0;
  dc::ScratchLayout sl{};
  uint64_t arena_bytes = 0, payload_bytes = 0, leaf_bytes = 0, nslots_nonnull = 0;
};

namespace dc {
struct KdTables;
}

struct dc_tree_s {
  dc_ctx ctx = nullptr;
  dc_plan plan = nullptr;
  uint8_t* arena = nullptr;
  uint8_t* scratch = nullptr;
  dc::Tables tab{};
  bool attached = false;
  bool released = false;
  bool paths_uploaded = false;
  uint32_t tile_T = 0;              // tile size of the tile list in scratch
  uint64_t ntiles = 0;
  hipEvent_t tiles_ev = nullptr;    // recorded after the tile index was built
  dc::KdTables* kd = nullptr;       // element list of the kick-drift kernel (device)
  std::vector<std::pair<dc_tune, double>> tune_table;  // the last autotune: shape, median us
  int noalloc_dev = -1;             // device whose fixed scratch array this tree holds (-1: caller scratch)
};

namespace dc {
// The deep copy into caller (or fixed) device buffers; attach: relocate too.
dc_status deep_copy(dc_ctx ctx, dc_plan p, void* d_arena, uint64_t arena_bytes, void* d_scratch,
                    uint64_t scratch_bytes, void* stream, bool attach, dc_tree* out);
// Size of the fixed per-device scratch of dc_deep_copy_to_device_noalloc.
constexpr uint64_t kNoAllocScratchBytes = DC_NOALLOC_SCRATCH_BYTES;
// Looks up the fixed scratch array on `device` (current); once per device.
dc_status noalloc_setup(int device);
// A tree holding the device's fixed scratch was released.
void noalloc_release(int device);
dc_status plan_build(dc_plan p, const dc_schema_s* schema, uint32_t root_type, const void* const* roots,
                     uint64_t nroots, uint64_t align, const uint32_t* follow = nullptr, uint32_t nfollow = 0);
// Uploads the tile list for tiles of T chunks if scratch holds another size,
// and makes stream s wait until that upload is complete (it may have been
// made on another stream).
dc_status tree_ensure_tiles(dc_tree t, uint32_t T, hipStream_t s);
dc_status tree_check(dc_tree t, hipStream_t s);
// Frees the kick-drift tables of a tree.
void kd_free(dc_tree t);
// The tile list dc_run_kernel uses for every-leaf kernels.
dc_status tree_prepare_leaf_tiles(dc_tree t, hipStream_t s);
// Compute tiles of at most T chunks and kTileMaxLeaves leaves, in order.
std::vector<DevTile> build_tiles(const dc_plan_s* p, uint32_t T);
}  // namespace dc
