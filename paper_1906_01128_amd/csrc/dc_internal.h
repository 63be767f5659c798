// Internal layouts shared by the host core and the HIP kernels of libdc.
// Everything a kernel reads lives in the caller's scratch buffer at offsets
// fixed by the plan (ScratchLayout); the arena holds only the copied objects.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dc.h"

namespace dc {

constexpr uint32_t kMaxFields = 16;   // pointer members per struct type
constexpr uint32_t kMaxTypes = 64;
constexpr uint32_t kMaxChainSteps = 32;
constexpr uint32_t kNone = 0xFFFFFFFFu;

// Relocation work units ("segments"): a contiguous range of the global slot
// enumeration (struct objects in arena order, elements in index order,
// pointer members in ascending offset order) and the distinct objects its
// non-null slots point to. Every slot carries the index of its target in its
// unit's target list; a workgroup stages the unit's targets (address before
// and after the translation) in LDS and translates every slot of the range.
constexpr uint32_t kSegMaxSObjs = 256;     // struct objects spanned per unit
constexpr uint64_t kSegMaxSlots = 2048;    // slots per unit (so at most 2048 targets)
constexpr uint16_t kNoTarget = 0xFFFF;     // slot index of a null (or unfollowed) slot

constexpr uint32_t kChunk = 16;             // bytes per vector access of the leaf kernels

// Compute tiles: a contiguous range of the 16-byte chunks of the leaves laid
// end to end, at most kTileMaxLeaves leaves (their table sits in LDS) and at
// most the requested number of chunks. Built on the host per tile size.
constexpr uint32_t kTileMinChunks = 512;      // smallest tile size the scratch is sized for
constexpr uint32_t kTileMaxChunks = 1u << 20;
constexpr uint32_t kTileMaxLeaves = 256;
// Work queues of the persistent fused launch: queue q hands out the items
// q, q + kFusedQueues, ... to the workgroups whose index is q modulo it.
constexpr uint32_t kFusedQueues = 8;
// The device scan of the leaves' chunk prefix: blocks of kScanLeaves leaves.
constexpr uint32_t kScanBlock = 256, kScanPer = 4, kScanLeaves = kScanBlock * kScanPer;

struct DevTile {
  uint64_t c_lo, c_hi;  // chunk range
  uint32_t l_lo, l_hi;  // first and last leaf it touches
  uint64_t pad;
};

// Struct type as the kernels see it: pointer members sorted by offset.
struct DevType {
  uint32_t size;
  uint32_t nptr;
  uint32_t follow;  // bit k: pointer member k (offset order) is followed
  uint32_t pad;
  uint32_t ptr_off[kMaxFields];
  uint32_t kind[kMaxFields];
  uint32_t ptype[kMaxFields];
  int32_t cnt_off[kMaxFields];
  uint32_t cnt_bytes[kMaxFields];
  uint32_t cnt_mult[kMaxFields];
  uint64_t fixed[kMaxFields];
};

struct DevSObj {  // one struct array placed in the arena
  uint64_t off;
  uint64_t count;
  uint32_t type;
  uint32_t obj;
};

// One target of a relocation unit: the object's host address and arena offset.
struct DevTarget {
  uint64_t host, off;
};

struct DevSeg {
  uint64_t slot_lo, slot_hi;  // slot range [lo, hi)
  uint64_t tgt_lo, tgt_hi;    // range in the target table
  uint32_t sobj_lo, sobj_hi;  // struct objects overlapping the slot range
  // leaves [leaf_lo, leaf_hi) (leaf order) whose discovering slot lies in the
  // range; meaningful when every unit's leaves are contiguous (the plan says so)
  uint32_t leaf_lo, leaf_hi;
};

// Leaf (FP32/FP64 array with >= 1 element) records for the compute kernels.
// info = bytes | kind << 56.
constexpr int kLeafKindShift = 56;

// A pointer slot the fused relocate-and-compute launch translates on its own:
// one that is not the discovering slot of a leaf (null, unfollowed, reaching
// a struct, integer or empty array, or a second reach of any array).
struct DevResid {
  uint64_t slot_off;  // arena offset of the slot
  uint32_t tgt;       // global index of its target entry, kNone for a null slot
  uint32_t follow;    // 0: a member left out of a selective copy (zeroed)
};

struct DevPath {  // pointer path by which the walk first reached a leaf
  uint64_t root_off;
  uint32_t hop_lo, nhops;
};

// Header at offset 0 of scratch.
struct DevHeader {
  uint64_t arena;  // device address of the arena (B)
  uint64_t nobj, nsobj, nseg, nleaves, nslots;
  uint64_t total_chunks;
  // device-side error reporting (sticky until the host clears it)
  uint32_t err_count;
  uint32_t err_code;
  uint64_t err_slot;  // arena offset of the first bad slot
  uint32_t spin_fail;
  uint32_t pad0;
  // chain resolution result
  uint64_t chain_addr, chain_count;
  uint32_t chain_kind, chain_status;
  uint64_t pad1[4];
  // persistent kernel work queue and phase counters, one 128-byte cache line
  // each so that waiting workgroups do not slow the queue down
  uint32_t queue;
  uint32_t pad_q[31];
  uint32_t doneA;
  uint32_t pad_a[31];
  uint32_t doneB;
  uint32_t pad_b[31];
  // the persistent fused launch's work queues, one 128-byte line each
  uint32_t fq[kFusedQueues * 32];
};
// the host reads the header back into a 4 KiB pinned buffer
static_assert(sizeof(DevHeader) <= 4096, "device header larger than its host read buffer");

enum DevErr : uint32_t {
  kErrNone = 0,
  kErrUnknownPtr = 1,  // a slot value that is not a planned array start
  kErrNullChain = 2,
  kErrIndex = 3,
  kErrKind = 4,
  kErrSpin = 5,        // persistent kernel wait bound hit
  kErrWild = 6,        // a pointer followed by a kernel lies outside the arena
  kErrChain = 7        // the relocated chain does not lead where the plan says
};

struct ScratchLayout {
  uint64_t header, types, sobj, sobj_pre, segs, tgts, slot_tix;
  uint64_t leaf_slot, leaf_pre, leaf_info, leaf_out, leaf_tgt, leaf_dev, resid;
  uint64_t leaf_pre_scan;  // per block of kScanLeaves leaves: its chunk sum, then its offset
  uint64_t tiles, paths, hops;
  uint64_t static_end;  // [0, static_end) is uploaded with every deep copy
  uint64_t total;
};

// Arguments of the compute kernels. A pass reads each leaf from the arena
// (or, when src_out is set, from its place in the out image) and writes it
// to the arena (out == null) or to the out image.
struct LeafArgs {
  double a, b;
  float af, bf;
  uint8_t* out;
  uint32_t src_out;
  uint32_t pad;
};

// One chain for the device resolver: per step the byte offset of the pointer
// member, where its count lives, the element size of the array it points to
// and the index to continue at.
struct ChainArgs {
  uint64_t root_off;
  uint64_t expect_addr;  // where the plan says the chain ends (0: no check)
  uint32_t nsteps;
  uint32_t pad;
  uint32_t field_off[kMaxChainSteps];
  int32_t cnt_off[kMaxChainSteps];
  uint32_t cnt_bytes[kMaxChainSteps];
  uint32_t cnt_mult[kMaxChainSteps];
  uint32_t elem_size[kMaxChainSteps];
  uint32_t kind[kMaxChainSteps];
  uint64_t fixed[kMaxChainSteps];
  uint64_t index[kMaxChainSteps];
};

// Per-access chain walk: p = root; for each hop p = *(p + hop_off[h]).
struct HopArgs {
  uint64_t root_off;
  uint32_t nhops;
  uint32_t pad;
  uint64_t hop_off[kMaxChainSteps];
};

// A scalar member reached through a chain of struct steps.
struct DevScalar {
  uint64_t root_off;    // arena offset of the root struct
  uint64_t expect_off;  // arena offset of the scalar according to the plan
  uint32_t hop_lo, nhops;
  uint32_t offset, bytes;
};
struct DevScalarHop {
  uint32_t field_off;  // pointer member in the current element
  uint32_t elem_size;  // element size of the struct array it points to
  uint64_t index;      // element to move to
};

// One element of the molecular-dynamics update: where its x, v and f slots
// are and how many doubles each array holds.
struct DevTriple {
  uint64_t elem_off;  // arena offset of the struct element
  uint64_t count;     // doubles per array
};
struct KickDriftArgs {
  const DevTriple* tri;
  const uint64_t* pre;  // ntri + 1 entries: prefix of 16-byte chunks
  const DevTile* tiles;
  uint64_t ntiles;
  uint32_t x_off, v_off, f_off, pad;
  double dt, dt_over_m;
};

// ---- launchers (dc_kernels.hip) ------------------------------------------------
struct Tables {  // device addresses of the scratch tables
  DevHeader* hdr;
  const DevType* types;
  const DevSObj* sobj;
  const uint64_t* sobj_pre;  // nsobj + 1 entries (slot prefix)
  const DevSeg* segs;
  const DevTarget* tgts;  // every unit's targets, unit after unit
  const uint16_t* slot_tix;  // per slot: its target's index in its unit's list, or kNoTarget
  const uint64_t* leaf_slot;
  const uint64_t* leaf_pre;  // nleaves + 1 entries (16-byte chunk prefix)
  const uint64_t* leaf_info;
  const uint64_t* leaf_out;
  const uint32_t* leaf_tgt;  // per leaf: global index of its parent slot's target entry
  const uint64_t* leaf_dev;  // per leaf: its planned arena offset
  const DevResid* resid;     // the slots no leaf was first reached through
  const DevTile* tiles;
  const DevPath* paths;
  const uint64_t* hops;
  uint8_t* arena;
  uint64_t arena_bytes;
  uint64_t nseg, nleaves, total_chunks, nresid;
  uint32_t ntypes, pad;
};

hipError_t launch_relocate(const Tables& t, bool attach, hipStream_t s);
// update 0: temps[i] = the scalar (zero-extended); 1: the scalar = low bytes of temps[i]
hipError_t launch_scalar(const Tables& t, const DevScalar* refs, const DevScalarHop* hops, uint32_t n,
                         uint64_t* temps, int update, hipStream_t s);
hipError_t launch_kick_drift(const Tables& t, const KickDriftArgs& k, hipStream_t s);
hipError_t launch_resolve_chain(const Tables& t, const ChainArgs& c, hipStream_t s);
// every leaf, in the ntiles tiles of tile_chunks chunks listed in the tables
hipError_t launch_leaf_tiles(const Tables& t, const LeafArgs& la, uint64_t ntiles, uint32_t tile_chunks,
                             bool deref_each, hipStream_t s);
// one FP32/FP64 array at device address `base`, resolved once before the
// passes (the pointerchain extraction)
hipError_t launch_stream_resolved(const Tables& t, uint64_t base, uint64_t count, uint32_t kind, const LeafArgs& la,
                                  hipStream_t s);
hipError_t launch_stream_deref(const Tables& t, const HopArgs& h, uint64_t count, uint32_t kind,
                               const LeafArgs& la, hipStream_t s);
// spin_limit: polls of a workgroup's wait for a phase before it records kErrSpin
hipError_t launch_batch(const Tables& t, const LeafArgs& la, uint32_t flags, uint32_t block, uint32_t grid,
                        uint64_t ntiles, uint32_t spin_limit, hipStream_t s);
// one persistent launch, one queue item per relocation unit (attach, the
// unit's contiguous leaves, detach); needs the plan's per-unit leaf runs
hipError_t launch_batch_units(const Tables& t, const LeafArgs& la, uint32_t flags, uint32_t block, uint32_t grid,
                              hipStream_t s);
hipError_t launch_reset_counters(DevHeader* hdr, hipStream_t s);
// the fused launch's work in a persistent grid of `grid` 256-thread
// workgroups taking items from kFusedQueues device queues (reset first)
hipError_t launch_fused_persistent(const Tables& t, const LeafArgs& la, uint64_t ntiles, uint32_t tile_chunks,
                                   uint32_t flags, uint32_t grid, hipStream_t s);
// The leaves' 16-byte-chunk prefix (nl + 1 entries) from their size|kind
// words, on the device; scan holds (nl + kScanLeaves - 1) / kScanLeaves + 1 words.
hipError_t launch_leaf_prefix(const uint64_t* info, uint64_t nl, uint64_t* pre, uint64_t* scan, hipStream_t s);
// one launch that relocates and computes: every tile translates the parent
// slots of the leaves whose first chunk it holds (attach before its compute,
// detach after), extra workgroups translate the other slots; no workgroup
// waits for another
hipError_t launch_fused(const Tables& t, const LeafArgs& la, uint64_t ntiles, uint32_t tile_chunks, uint32_t flags,
                        hipStream_t s);
int device_cu_count();

}  // namespace dc
