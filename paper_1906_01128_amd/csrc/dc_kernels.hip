// Device kernels of libdc for gfx950 (CDNA4, 64-wide wavefronts).
//
// Nothing here is a dense contraction, so nothing uses MFMA: every kernel is
// bound by HBM bandwidth or memory latency. The leaf kernels stream 16-byte
// vector accesses, several per thread in flight; the relocation kernel stages
// each work unit's address-translation table in LDS.
#include <hip/hip_runtime.h>

#include "dc_internal.h"

namespace dc {

namespace {

constexpr int kRelocBlock = 512;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Global-memory accesses through addresses held as integers. Without the
// address-space cast the compiler would emit flat instructions, which also
// count against the LDS wait counter and cost more to issue.
typedef __attribute__((address_space(1))) u32x4 g_u32x4;
typedef __attribute__((address_space(1))) double g_double;
typedef __attribute__((address_space(1))) float g_float;
typedef __attribute__((address_space(1))) uint64_t g_u64;

__device__ __forceinline__ u32x4 gload16(uint64_t a) { return *(const g_u32x4*)a; }
__device__ __forceinline__ void gstore16(uint64_t a, u32x4 v) { *(g_u32x4*)a = v; }

// Leaf data streamed once per pass. NT: non-temporal loads and stores, which
// (both together; either alone changed nothing) ran a flat 12 GiB in-place
// fma stream at 6.5 TB/s against 5.96 with plain accesses, and the MD
// kick-drift kernel's five streams 5% faster. They are not used where leaves
// are small: on the MD leaves (about 1.5 KB, so many 128-byte lines are
// shared by two leaves or written in part) the tiled leaf kernel ran 2-11%
// slower with them at every tile shape, and the per-unit persistent launch
// 16% slower. Streams that fit the Infinity Cache and are read again pass
// after pass keep plain accesses too (128 MiB: 6.66 TB/s plain, 6.38 NT).
template <bool NT>
__device__ __forceinline__ u32x4 sload16(uint64_t a) {
  if constexpr (NT) return __builtin_nontemporal_load((const g_u32x4*)a);
  else return *(const g_u32x4*)a;
}
template <bool NT>
__device__ __forceinline__ void sstore16(uint64_t a, u32x4 v) {
  if constexpr (NT) __builtin_nontemporal_store(v, (g_u32x4*)a);
  else *(g_u32x4*)a = v;
}
template <bool NT, typename T>
__device__ __forceinline__ T sload(uint64_t a) {
  typedef __attribute__((address_space(1))) T gT;
  if constexpr (NT) return __builtin_nontemporal_load((const gT*)a);
  else return *(const gT*)a;
}
template <bool NT, typename T>
__device__ __forceinline__ void sstore(uint64_t a, T v) {
  typedef __attribute__((address_space(1))) T gT;
  if constexpr (NT) __builtin_nontemporal_store(v, (gT*)a);
  else *(gT*)a = v;
}

// Workgroup barrier that orders LDS accesses only. __syncthreads() also
// orders global memory, which on CDNA means waiting until every store of the
// wave has completed (one counter covers loads and stores): a loop that
// reuses LDS between rounds of streamed stores would pay a write round trip
// per round.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}


// What relocation needs of a struct type (the full DevType is 528 bytes).
struct RelocType {
  uint32_t size, nptr, follow, pad;
  uint32_t ptr_off[kMaxFields];
};

// LDS of one relocation unit: every target's address before and after the
// translation, indexed by the target index each slot carries, and the struct
// arrays the unit spans (their placement, and their slot prefix relative to
// the unit's first slot), then the types of the plan, so that a slot costs
// one global load (its value), one 2-byte load (its target index) and one
// store. About 35 KB plus 80 bytes per type: four 512-thread workgroups of a
// plan with up to a dozen types fit one CU's 160 KB.
struct RelocLds {
  uint64_t from[kSegMaxSlots];     // a target's address before the translation
  uint64_t to[kSegMaxSlots];       // and after it
  uint64_t sobj[kSegMaxSObjs];     // arena offset | type << 56
  uint32_t rel[kSegMaxSObjs + 4];  // slot prefix - first slot, clamped to [0, slots of the unit]
  // RelocType types[ntypes] follows
};
constexpr int kSObjTypeShift = 56;
static_assert(sizeof(RelocLds) % 16 == 0, "types start 16-byte aligned");

__host__ __device__ constexpr size_t reloc_lds_bytes(uint32_t ntypes) {
  return sizeof(RelocLds) + (size_t)ntypes * sizeof(RelocType);
}

__device__ __noinline__ void report_bad_slot(DevHeader* hdr, uint64_t slot_off) {
  atomicAdd(&hdr->err_count, 1u);
  atomicCAS(&hdr->err_code, 0u, (uint32_t)kErrUnknownPtr);
  atomicMin((unsigned long long*)&hdr->err_slot, (unsigned long long)slot_off);
}

// Every pointer a kernel follows is checked against the arena before use; a
// wild one is reported in the header and its work skipped, so that a damaged
// arena cannot make a kernel touch memory outside it.
__device__ __forceinline__ bool in_arena(const Tables& t, uint64_t p, uint64_t need) {
  const uint64_t B = (uint64_t)t.arena;
  return p >= B && p <= B + t.arena_bytes && need <= B + t.arena_bytes - p;
}

__device__ __noinline__ void report_wild(DevHeader* hdr) {
  atomicAdd(&hdr->err_count, 1u);
  atomicCAS(&hdr->err_code, 0u, (uint32_t)kErrWild);
}

// Translates every pointer slot of relocation unit `sg`. attach: host address
// -> arena address; detach: arena address -> host address. A slot must hold
// its planned target's address (or null): any other value is left alone and
// reported in the header. Three dependent rounds of global accesses: the
// unit's tables, targets and the slots' target indices; the slots' current
// values; the translated stores. A unit's at most 2048 slots are KS per
// thread (bs * KS >= 2048).

// A slot the unit translated, kept by a caller that restores it later: its
// arena offset (kKeepBad set when its value was not its planned target, ~0
// for none) and its value before the translation.
constexpr uint64_t kKeepBad = 1ull << 63;

template <bool KEEP, int KS>
__device__ void relocate_unit(const Tables& t, uint64_t sg, bool attach, uint8_t* lds, uint64_t* keep_off = nullptr,
                              uint64_t* keep_val = nullptr) {
  RelocLds* L = (RelocLds*)lds;
  RelocType* types = (RelocType*)(lds + sizeof(RelocLds));
  const int tid = threadIdx.x, bs = blockDim.x;
  const DevSeg seg = t.segs[sg];
  const uint64_t B = (uint64_t)t.arena;
  const uint64_t nslots = seg.slot_hi - seg.slot_lo;
  // slot prefix of the unit's first struct array, which may begin before the unit
  const uint64_t pre0 = t.sobj_pre[seg.sobj_lo];

  // the target index of each of the thread's slots, loaded with the tables
  uint32_t tx[KS];
#pragma unroll
  for (int k = 0; k < KS; k++) {
    const uint32_t jr = (uint32_t)k * bs + tid;
    tx[k] = jr < nslots ? t.slot_tix[seg.slot_lo + jr] : kNoTarget;
  }
  // stage: the targets' translations, the unit's struct arrays and slot
  // prefix, and the types
  const uint32_t ntgt = (uint32_t)(seg.tgt_hi - seg.tgt_lo);
  for (uint32_t i = tid; i < ntgt; i += bs) {
    const DevTarget tg = t.tgts[seg.tgt_lo + i];
    L->from[i] = attach ? tg.host : B + tg.off;
    L->to[i] = attach ? B + tg.off : tg.host;
  }
  const uint32_t nso = seg.sobj_hi - seg.sobj_lo;
  for (uint32_t i = tid; i <= nso; i += bs) {
    const uint64_t pr = t.sobj_pre[seg.sobj_lo + i];
    const uint64_t c = pr < seg.slot_lo ? seg.slot_lo : (pr > seg.slot_hi ? seg.slot_hi : pr);
    L->rel[i] = (uint32_t)(c - seg.slot_lo);
  }
  for (uint32_t i = tid; i < nso; i += bs) {
    const DevSObj so = t.sobj[seg.sobj_lo + i];
    L->sobj[i] = so.off | (uint64_t)so.type << kSObjTypeShift;
  }
  for (uint32_t i = tid; i < t.ntypes; i += bs) {
    const DevType* ty = &t.types[i];
    types[i].size = ty->size;
    types[i].nptr = ty->nptr;
    types[i].follow = ty->follow;
    for (uint32_t f = 0; f < kMaxFields; f++) types[i].ptr_off[f] = ty->ptr_off[f];
  }
  lds_barrier();

  // the thread's slots: their arena offsets and current values
  uint64_t soff[KS], val[KS];
  bool fol[KS];
#pragma unroll
  for (int k = 0; k < KS; k++) {
    const uint32_t jr = (uint32_t)k * bs + tid;  // slot - first slot
    soff[k] = ~0ull;
    val[k] = 0;
    fol[k] = true;
    if (jr >= nslots) continue;
    // struct array holding the slot: largest i with rel[i] <= jr
    uint32_t lo = 0, hi = nso;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (L->rel[mid] <= jr) lo = mid;
      else hi = mid;
    }
    const uint64_t so = L->sobj[lo];
    const RelocType& ty = types[so >> kSObjTypeShift];
    const uint64_t local = lo == 0 ? seg.slot_lo + jr - pre0 : (uint64_t)(jr - L->rel[lo]);
    const uint64_t e = local / ty.nptr;
    const uint32_t f = (uint32_t)(local - e * ty.nptr);
    soff[k] = (so & ((1ull << kSObjTypeShift) - 1)) + e * ty.size + ty.ptr_off[f];
    fol[k] = (ty.follow >> f) & 1u;
    val[k] = *(const g_u64*)(B + soff[k]);
  }

#pragma unroll
  for (int k = 0; k < KS; k++) {
    if (KEEP) keep_off[k] = ~0ull;
    if (soff[k] == ~0ull || val[k] == 0) continue;
    // a member left out of a selective copy reads as null on the device
    if (!fol[k]) {
      *(g_u64*)(B + soff[k]) = 0;
      continue;
    }
    if (tx[k] >= ntgt || L->from[tx[k]] != val[k]) {
      report_bad_slot(t.hdr, soff[k]);
      if (KEEP) keep_off[k] = soff[k] | kKeepBad;
      continue;
    }
    *(g_u64*)(B + soff[k]) = L->to[tx[k]];
    if (KEEP) {
      keep_off[k] = soff[k];
      keep_val[k] = val[k];
    }
  }
}

__global__ void __launch_bounds__(kRelocBlock, 4) k_relocate(Tables t, int attach) {
  extern __shared__ __align__(16) uint8_t lds[];
  for (uint64_t sg = blockIdx.x; sg < t.nseg; sg += gridDim.x) {
    relocate_unit<false, kSegMaxSlots / kRelocBlock>(t, sg, attach != 0, lds);
    lds_barrier();
  }
}

// ---- chain resolution (one thread) ---------------------------------------------------

__device__ __forceinline__ uint64_t read_count(const uint8_t* elem, int32_t cnt_off, uint32_t cnt_bytes,
                                               uint32_t mult, uint64_t fixed, bool* neg) {
  if (cnt_off < 0) return fixed;
  int64_t n;
  if (cnt_bytes == 4) n = *(const int32_t*)(elem + cnt_off);
  else n = *(const int64_t*)(elem + cnt_off);
  if (n < 0) {
    *neg = true;
    return 0;
  }
  return (uint64_t)n * mult;
}

__global__ void k_resolve_chain(Tables t, ChainArgs c) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  DevHeader* h = t.hdr;
  const uint8_t* elem = t.arena + c.root_off;
  for (uint32_t s = 0; s < c.nsteps; s++) {
    if (!in_arena(t, (uint64_t)elem + c.field_off[s], 8)) {
      h->chain_status = kErrKind;
      report_wild(h);
      return;
    }
    const uint64_t p = *(const uint64_t*)(elem + c.field_off[s]);
    bool neg = false;
    const uint64_t n = read_count(elem, c.cnt_off[s], c.cnt_bytes[s], c.cnt_mult[s], c.fixed[s], &neg);
    if (p == 0) {
      h->chain_status = kErrNullChain;
      return;
    }
    if (s + 1 == c.nsteps) {
      const uint64_t es = c.kind[s] == DC_KIND_F64 || c.kind[s] == DC_KIND_I64 ? 8
                          : c.kind[s] == DC_KIND_U8 ? 1
                          : c.kind[s] == DC_KIND_STRUCT ? c.elem_size[s] : 4;
      if (neg || !in_arena(t, p, n * es)) {
        h->chain_status = kErrKind;
        report_wild(h);
        return;
      }
      if (c.expect_addr && p != c.expect_addr) {
        atomicAdd(&h->err_count, 1u);
        atomicCAS(&h->err_code, 0u, (uint32_t)kErrChain);
      }
      h->chain_addr = p;
      h->chain_count = n;
      h->chain_kind = c.kind[s];
      h->chain_status = 0;
      return;
    }
    if (neg || c.index[s] >= n || c.kind[s] != DC_KIND_STRUCT) {
      h->chain_status = kErrIndex;
      return;
    }
    if (!in_arena(t, p, (c.index[s] + 1) * c.elem_size[s])) {
      h->chain_status = kErrKind;
      report_wild(h);
      return;
    }
    elem = (const uint8_t*)p + c.index[s] * c.elem_size[s];
  }
  h->chain_status = kErrNullChain;
}

// One thread per scalar chain: walk the chain through the relocated arena,
// check that it lands where the plan says, then read or write the scalar.
__global__ void __launch_bounds__(256) k_scalar(Tables t, const DevScalar* refs, const DevScalarHop* hops, uint32_t n,
                                                uint64_t* temps, int update) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const DevScalar r = refs[i];
  uint64_t elem = (uint64_t)t.arena + r.root_off;
  bool ok = true;
  for (uint32_t k = 0; k < r.nhops && ok; k++) {
    const DevScalarHop h = hops[r.hop_lo + k];
    if (!in_arena(t, elem + h.field_off, 8)) {
      ok = false;
      break;
    }
    const uint64_t p = *(const uint64_t*)(elem + h.field_off);
    ok = p != 0 && in_arena(t, p, (h.index + 1) * h.elem_size);
    elem = p + h.index * h.elem_size;
  }
  const uint64_t addr = elem + r.offset;
  if (!ok || addr != (uint64_t)t.arena + r.expect_off) {
    atomicAdd(&t.hdr->err_count, 1u);
    atomicCAS(&t.hdr->err_code, 0u, (uint32_t)kErrChain);
    return;
  }
  uint8_t* sp = (uint8_t*)addr;
  uint8_t* tp = (uint8_t*)&temps[i];
  if (update) {
    for (uint32_t b = 0; b < r.bytes; b++) sp[b] = tp[b];
  } else {
    uint64_t v = 0;
    for (uint32_t b = 0; b < r.bytes; b++) v |= (uint64_t)sp[b] << (8 * b);
    temps[i] = v;
  }
}

// ---- leaf arithmetic ------------------------------------------------------------------

union Vec16 {
  u32x4 u;
  double d[2];
  float f[4];
};

template <typename T>
__device__ __forceinline__ void fma_chunk_t(Vec16& v, const LeafArgs& la) {
  if constexpr (sizeof(T) == 8) {
    v.d[0] = __builtin_fma(v.d[0], la.a, la.b);
    v.d[1] = __builtin_fma(v.d[1], la.a, la.b);
  } else {
    v.f[0] = __builtin_fmaf(v.f[0], la.af, la.bf);
    v.f[1] = __builtin_fmaf(v.f[1], la.af, la.bf);
    v.f[2] = __builtin_fmaf(v.f[2], la.af, la.bf);
    v.f[3] = __builtin_fmaf(v.f[3], la.af, la.bf);
  }
}

// A chunk whose kind differs from lane to lane: both interpretations are
// computed and the right one kept, so that no lane diverges (the wrong one is
// discarded; GPU floating point does not trap).
__device__ __forceinline__ void fma_chunk_any(Vec16& v, bool f64, const LeafArgs& la) {
  Vec16 d = v, f = v;
  fma_chunk_t<double>(d, la);
  fma_chunk_t<float>(f, la);
  v.u = f64 ? d.u : f.u;
}

// the first `nbytes` (< 16) bytes of a chunk, element by element
__device__ __forceinline__ void fma_partial(uint64_t src, uint64_t dst, uint32_t nbytes, uint32_t kind,
                                            const LeafArgs& la) {
  if (kind == DC_KIND_F64) {
    for (uint32_t o = 0; o + 8 <= nbytes; o += 8)
      *(g_double*)(dst + o) = __builtin_fma(*(const g_double*)(src + o), la.a, la.b);
  } else {
    for (uint32_t o = 0; o + 4 <= nbytes; o += 4)
      *(g_float*)(dst + o) = __builtin_fmaf(*(const g_float*)(src + o), la.af, la.bf);
  }
}

// Makes a pointer opaque to the compiler, so that a load through it can be
// neither hoisted out of a loop nor merged with an earlier load of the same
// address: every chain walk really reads every pointer again.
__device__ __forceinline__ const uint8_t* opaque(const uint8_t* p) {
  asm volatile("" : "+v"(p));
  return p;
}

// ---- one array at the end of a resolved chain ----------------------------------------------

template <int U, typename T, bool NT>
__global__ void __launch_bounds__(256) k_stream_resolved(Tables t, uint64_t base, uint64_t count, LeafArgs la) {
  const uint64_t bytes = count * sizeof(T);
  if (!in_arena(t, base, bytes)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) report_wild(t.hdr);
    return;
  }
  const uint64_t src = la.src_out ? (uint64_t)la.out : base;
  const uint64_t dst = la.out ? (uint64_t)la.out : base;
  const uint64_t nfull = bytes / kChunk;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * U;
  for (uint64_t c0 = (uint64_t)blockIdx.x * blockDim.x * U + threadIdx.x; c0 < nfull; c0 += stride) {
    Vec16 v[U];
#pragma unroll
    for (int k = 0; k < U; k++) {
      const uint64_t c = c0 + (uint64_t)k * blockDim.x;
      if (c < nfull) v[k].u = sload16<NT>(src + c * kChunk);
    }
#pragma unroll
    for (int k = 0; k < U; k++) {
      const uint64_t c = c0 + (uint64_t)k * blockDim.x;
      if (c < nfull) {
        fma_chunk_t<T>(v[k], la);
        sstore16<NT>(dst + c * kChunk, v[k].u);
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && nfull * kChunk < bytes)
    fma_partial(src + nfull * kChunk, dst + nfull * kChunk, (uint32_t)(bytes - nfull * kChunk),
                sizeof(T) == 8 ? DC_KIND_F64 : DC_KIND_F32, la);
}

// Reads the pointer at `addr` through the scalar data cache. The chain a
// wavefront walks is the same for all its lanes, so on CDNA the walk is one
// scalar load per hop per wavefront, kept apart from the vector caches that the
// streamed leaf data flows through. The address passes through an opaque
// register move first, so the compiler can neither hoist the load out of the
// element loop nor reuse the value of an earlier walk: every element access
// really reads every pointer of the chain again.
__device__ __forceinline__ uint64_t walk_load(uint64_t addr) {
  asm volatile("" : "+s"(addr));
  return *(const __attribute__((address_space(4))) uint64_t*)addr;
}

// Every element access walks the chain from the root (Section 3: the cost
// the pointerchain directive removes). Each thread handles U elements with one
// walk each; a wavefront's 64 lanes access 64 consecutive elements per walk.
// The U walks of a wavefront advance hop by hop together, so their scalar
// loads overlap; the hop offsets (at most MAXH) are held in scalar registers.
//
// Bounds: a wavefront first walks the chain once with every slot checked
// against the arena (a slot outside it is replaced by the arena base before
// it is read; the wavefront then reports and stops). The U per-access walks
// that follow read the same slots, which no kernel of this library writes
// while the walk runs, and must land on the checked address. Checking every
// hop of every walk instead puts a vector compare on the scalar load chain
// and costs about a fifth of the bandwidth.
template <int U, int MAXH, typename T, bool NT>
__global__ void __launch_bounds__(256) k_stream_deref(Tables t, HopArgs h, uint64_t count, LeafArgs la) {
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t i0 = wave * 64 * U + lane;
  const uint64_t B = (uint64_t)t.arena, size = t.arena_bytes;
  uint64_t off[MAXH];
#pragma unroll
  for (int j = 0; j < MAXH; j++) off[j] = j < (int)h.nhops ? h.hop_off[j] : 0;
  bool ok = size >= 8;
  uint64_t q = B + h.root_off;
#pragma unroll
  for (int j = 0; j < MAXH; j++) {
    if (j < (int)h.nhops) {
      uint64_t slot = q + off[j];
      const bool in = slot - B <= size - 8;
      ok = ok && in;
      slot = in ? slot : B;
      q = walk_load(slot);
    }
  }
  const uint64_t need = count * sizeof(T);
  ok = ok && q - B <= size && need <= size - (q - B);
  if (!ok) {
    if (lane == 0) report_wild(t.hdr);
    return;
  }
  uint64_t p[U];
#pragma unroll
  for (int k = 0; k < U; k++) p[k] = B + h.root_off;
#pragma unroll
  for (int j = 0; j < MAXH; j++)
    if (j < (int)h.nhops)
#pragma unroll
      for (int k = 0; k < U; k++) p[k] = walk_load(p[k] + off[j]);
#pragma unroll
  for (int k = 0; k < U; k++) ok = ok && p[k] == q;
  if (!ok) {
    if (lane == 0) report_wild(t.hdr);
    return;
  }
  T x[U];
#pragma unroll
  for (int k = 0; k < U; k++) {
    const uint64_t i = i0 + (uint64_t)k * 64;
    const uint64_t src = la.src_out ? (uint64_t)la.out : p[k];
    if (i < count) x[k] = sload<NT, T>(src + i * sizeof(T));
  }
#pragma unroll
  for (int k = 0; k < U; k++) {
    const uint64_t i = i0 + (uint64_t)k * 64;
    const uint64_t dst = (la.out ? (uint64_t)la.out : p[k]) + i * sizeof(T);
    if (i < count) {
      if constexpr (sizeof(T) == 8) sstore<NT, double>(dst, __builtin_fma(x[k], la.a, la.b));
      else sstore<NT, float>(dst, __builtin_fmaf(x[k], la.af, la.bf));
    }
  }
}

// ---- every leaf: 16-byte chunks of the concatenated leaves, in tiles ---------------------

__device__ __forceinline__ uint32_t find_leaf(const uint64_t* pre, uint32_t nl, uint64_t c) {
  uint32_t lo = 0, hi = nl;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (pre[mid] <= c) lo = mid;
    else hi = mid;
  }
  return lo;
}

// LDS of one compute tile: prefix, followed address, size|kind, image offset
// and planned address of up to kTileMaxLeaves leaves (and one more prefix entry)
constexpr size_t kTileLds = (size_t)(kTileMaxLeaves + 2) * 5 * 8;
// a RESOLVED tile gives each of its leaves a thread of its own (launches have 256, 512 or 1024)
static_assert(kTileMaxLeaves <= 256, "one leaf per thread in the tile prologue");

// One round of a RESOLVED tile: chunk c_lo + k * bs + tid for k < U, each
// read from its leaf at base[i] (or from the image) when whole.
struct TileRound {
  Vec16 v;
  uint64_t byte;
  uint32_t i, nb;
};

template <int U>
__device__ __forceinline__ void tile_round_load(const LeafArgs& la, const uint64_t* pre, const uint64_t* base,
                                                const uint64_t* info, const uint64_t* outo, uint32_t nl,
                                                uint64_t c_lo, uint64_t c_hi, TileRound (&r)[U]) {
  const int tid = threadIdx.x, bs = blockDim.x;
#pragma unroll
  for (int k = 0; k < U; k++) {
    const uint64_t c = c_lo + (uint64_t)k * bs + tid;
    r[k].nb = 0;
    r[k].i = 0;
    r[k].byte = 0;
    if (c < c_hi) {
      const uint32_t i = find_leaf(pre, nl, c);
      const uint64_t byte = (c - pre[i]) * kChunk;
      const uint64_t lb = info[i] & ((1ull << kLeafKindShift) - 1);
      r[k].i = i;
      r[k].byte = byte;
      r[k].nb = base[i] == 0 ? 0 : (uint32_t)(lb - byte < kChunk ? lb - byte : kChunk);
      const uint64_t src = (la.src_out ? (uint64_t)la.out + outo[i] : base[i]) + byte;
      if (r[k].nb == kChunk) r[k].v.u = gload16(src);
    }
  }
}

template <int U>
__device__ __forceinline__ void tile_round_store(const LeafArgs& la, const uint64_t* addr, const uint64_t* info,
                                                 const uint64_t* outo, TileRound (&r)[U]) {
#pragma unroll
  for (int k = 0; k < U; k++) {
    if (r[k].nb == kChunk) {
      const uint32_t i = r[k].i;
      fma_chunk_any(r[k].v, (info[i] >> kLeafKindShift) == DC_KIND_F64, la);
      gstore16((la.out ? (uint64_t)la.out + outo[i] : addr[i]) + r[k].byte, r[k].v.u);
    }
  }
  // the last, shorter chunk of a leaf, element by element
#pragma unroll
  for (int k = 0; k < U; k++) {
    if (r[k].nb != 0 && r[k].nb != kChunk) {
      const uint32_t i = r[k].i;
      const uint64_t src = (la.src_out ? (uint64_t)la.out + outo[i] : addr[i]) + r[k].byte;
      const uint64_t dst = (la.out ? (uint64_t)la.out + outo[i] : addr[i]) + r[k].byte;
      fma_partial(src, dst, r[k].nb, (uint32_t)(info[i] >> kLeafKindShift), la);
    }
  }
}

// One compute tile: its chunk range of the leaves laid end to end, processed
// in rounds of U chunks per thread. RESOLVED: each leaf's address is read
// once per tile from its relocated parent slot; the first round's loads are
// issued at the leaf's planned address together with that slot read, and a
// chunk whose slot turns out to hold another address is read again from
// there before anything is stored, so the result is that of following the
// slot. DEREF: each element access walks the leaf's whole path from its root.
template <int U, bool DEREF>
__device__ void leaf_tile(const Tables& t, const LeafArgs& la, uint64_t tile, uint8_t* lds) {
  constexpr uint32_t N = kTileMaxLeaves + 2;
  uint64_t* pre = (uint64_t*)lds;
  uint64_t* addr = pre + N;   // RESOLVED: the address the parent slot holds (0: wild)
  uint64_t* info = addr + N;
  uint64_t* outo = info + N;
  uint64_t* plan = outo + N;  // RESOLVED: the planned address (0: outside the arena)
  const int tid = threadIdx.x, bs = blockDim.x;
  const uint64_t B = (uint64_t)t.arena;
  const DevTile tl = t.tiles[tile];
  const uint32_t l0 = tl.l_lo, l1 = tl.l_hi;
  const uint32_t nl = l1 - l0 + 1;
  if (!DEREF) {
    // one leaf per thread: every launch has at least kTileMaxLeaves threads
    uint64_t so = 0, lb = 0;
    if (tid < (int)nl) {
      const uint32_t l = l0 + tid;
      pre[tid] = t.leaf_pre[l];
      const uint64_t inf = t.leaf_info[l];
      info[tid] = inf;
      // image offsets only for a pass that reads or writes the image
      outo[tid] = la.out || la.src_out ? t.leaf_out[l] : 0;
      so = t.leaf_slot[l];
      lb = inf & ((1ull << kLeafKindShift) - 1);
      const uint64_t pl = B + t.leaf_dev[l];
      plan[tid] = in_arena(t, pl, lb) ? pl : 0;
    }
    if (tid == 0) pre[nl] = t.leaf_pre[l1 + 1];
    lds_barrier();
    TileRound r[U];
    tile_round_load<U>(la, pre, plan, info, outo, nl, tl.c_lo, tl.c_hi, r);
    // the parent slots, read while those loads are in flight
    if (tid < (int)nl) {
      const uint64_t a = *(const g_u64*)(B + so);
      if (in_arena(t, a, lb)) {
        addr[tid] = a;
      } else {
        addr[tid] = 0;
        report_wild(t.hdr);
      }
    }
    lds_barrier();
    // a chunk loaded from anywhere but its slot's address is loaded again
#pragma unroll
    for (int k = 0; k < U; k++) {
      const uint64_t c = tl.c_lo + (uint64_t)k * bs + tid;
      if (c < tl.c_hi && addr[r[k].i] != plan[r[k].i]) {
        const uint32_t i = r[k].i;
        const uint64_t lb2 = info[i] & ((1ull << kLeafKindShift) - 1);
        r[k].nb = addr[i] == 0 ? 0 : (uint32_t)(lb2 - r[k].byte < kChunk ? lb2 - r[k].byte : kChunk);
        const uint64_t src = (la.src_out ? (uint64_t)la.out + outo[i] : addr[i]) + r[k].byte;
        if (r[k].nb == kChunk) r[k].v.u = gload16(src);
      }
    }
    tile_round_store<U>(la, addr, info, outo, r);
    for (uint64_t c_lo = tl.c_lo + (uint64_t)bs * U; c_lo < tl.c_hi; c_lo += (uint64_t)bs * U) {
      tile_round_load<U>(la, pre, addr, info, outo, nl, c_lo, tl.c_hi, r);
      tile_round_store<U>(la, addr, info, outo, r);
    }
    // the next tile's prologue rewrites the tables; no wait for this tile's stores
    lds_barrier();
    return;
  }
  for (uint32_t i = tid; i < nl; i += bs) {
    const uint32_t l = l0 + i;
    pre[i] = t.leaf_pre[l];
    info[i] = t.leaf_info[l];
    outo[i] = t.leaf_out[l];
  }
  if (tid == 0) pre[nl] = t.leaf_pre[l1 + 1];
  // LDS only: nothing global written here is read by another thread
  lds_barrier();
  for (uint64_t c_lo = tl.c_lo; c_lo < tl.c_hi; c_lo += (uint64_t)bs * U) {
    const uint64_t c_hi = tl.c_hi;
#pragma unroll 1
    for (int k = 0; k < U; k++) {
      const uint64_t c = c_lo + (uint64_t)k * bs + tid;
      if (c >= c_hi) continue;
      const uint32_t i = find_leaf(pre, nl, c);
      const uint64_t byte = (c - pre[i]) * kChunk;
      const uint64_t lb = info[i] & ((1ull << kLeafKindShift) - 1);
      const uint32_t kind = (uint32_t)(info[i] >> kLeafKindShift);
      const uint32_t n = (uint32_t)(lb - byte < kChunk ? lb - byte : kChunk);
      const DevPath path = t.paths[l0 + i];
      const uint32_t es = kind == DC_KIND_F64 ? 8 : 4;
      for (uint32_t o = 0; o + es <= n; o += es) {
        const uint8_t* p = t.arena + path.root_off;
        bool ok = true;
        for (uint32_t hp = 0; hp < path.nhops && ok; hp++) {
          const uint8_t* slot = opaque(p) + t.hops[path.hop_lo + hp];
          ok = in_arena(t, (uint64_t)slot, 8);
          if (ok) p = (const uint8_t*)*(const g_u64*)(uint64_t)slot;
        }
        if (!ok || !in_arena(t, (uint64_t)p, lb)) {
          report_wild(t.hdr);
          break;
        }
        const uint64_t src = (la.src_out ? (uint64_t)la.out + outo[i] : (uint64_t)p) + byte + o;
        const uint64_t d = (la.out ? (uint64_t)la.out + outo[i] : (uint64_t)p) + byte + o;
        if (kind == DC_KIND_F64) *(g_double*)d = __builtin_fma(*(const g_double*)src, la.a, la.b);
        else *(g_float*)d = __builtin_fmaf(*(const g_float*)src, la.af, la.bf);
      }
    }
  }
  lds_barrier();
}

template <int U, bool DEREF>
__global__ void __launch_bounds__(256) k_leaf_tiles(Tables t, LeafArgs la, uint64_t ntiles) {
  __shared__ __align__(16) uint8_t lds[kTileLds];
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) leaf_tile<U, DEREF>(t, la, tile, lds);
}

// ---- relocation and compute fused, tile by tile ------------------------------------------
//
// Every leaf is reached through one slot, its discovering slot, which only
// the leaf's kernel reads. So a tile can translate the slots of its own
// leaves: the tile holding a leaf's first chunk checks the slot and, after
// its compute, writes the leaf's arena address into it (attach) and then the
// host address back (detach), as the flags ask; another tile holding later
// chunks of the same leaf accepts either value, since that first tile may run
// before, during or after it. Each leaf is computed at its planned arena
// address, the value the attach writes. Workgroups past the tiles translate every other slot (a
// second reach of an array, a slot reaching a struct, integer or empty
// array, null and unfollowed members). Nothing waits for anything: one launch
// relocates and computes every structure.

constexpr size_t kFusedLds = (size_t)(kTileMaxLeaves + 2) * 7 * 8;
constexpr uint64_t kFirstBit = 1ull << 63;  // in the slot-offset table: this tile holds the leaf's first chunk

// Q: run by the persistent form, whose thread 0 publishes the workgroup's
// next ticket (*tick_src, taken before this tile's first load) in *tick_dst
// once the first round's loads have returned, so that the ticket's return
// never holds up a load or a barrier. Only thread 0 reads *tick_src.
template <int U, bool Q = false>
__device__ void fused_tile(const Tables& t, const LeafArgs& la, uint64_t tile, uint32_t flags, uint8_t* lds,
                           uint32_t* tick_dst = nullptr, const uint32_t* tick_src = nullptr) {
  constexpr uint32_t N = kTileMaxLeaves + 2;
  uint64_t* pre = (uint64_t*)lds;
  uint64_t* addr = pre + N;  // the planned address, or 0: the leaf is not computed
  uint64_t* info = addr + N;
  uint64_t* outo = info + N;
  uint64_t* soff = outo + N;
  uint64_t* host = soff + N;
  uint64_t* plan = host + N;  // the planned address (0: outside the arena)
  const bool att = (flags & DC_BATCH_ATTACH) != 0, det = (flags & DC_BATCH_DETACH) != 0;
  const int tid = threadIdx.x, bs = blockDim.x;
  const uint64_t B = (uint64_t)t.arena;
  const DevTile tl = t.tiles[tile];
  const uint32_t l0 = tl.l_lo, l1 = tl.l_hi;
  const uint32_t nl = l1 - l0 + 1;
  // one leaf per thread (launches have 256 threads); until the check below,
  // soff and host hold the slot offset and the target index
  if (tid < (int)nl) {
    const uint32_t l = l0 + tid;
    const uint64_t inf = t.leaf_info[l];
    const uint64_t dev = B + t.leaf_dev[l];
    pre[tid] = t.leaf_pre[l];
    info[tid] = inf;
    outo[tid] = la.out || la.src_out ? t.leaf_out[l] : 0;
    soff[tid] = t.leaf_slot[l];
    host[tid] = t.leaf_tgt[l];
    plan[tid] = in_arena(t, dev, inf & ((1ull << kLeafKindShift) - 1)) ? dev : 0;
  }
  if (tid == 0) pre[nl] = t.leaf_pre[l1 + 1];
  lds_barrier();
  // the first round's loads at the planned addresses, the only ones a leaf is computed at
  TileRound r[U];
  tile_round_load<U>(la, pre, plan, info, outo, nl, tl.c_lo, tl.c_hi, r);
  // the slot's value and the leaf's target entry, while those loads are in flight
  if (tid < (int)nl) {
    const uint64_t so = soff[tid], dev = plan[tid];
    const bool first = pre[tid] >= tl.c_lo;
    const bool sok = in_arena(t, B + so, 8);
    const uint64_t v = sok ? *(const g_u64*)(B + so) : 0;
    const DevTarget tg = t.tgts[(uint32_t)host[tid]];
    uint64_t a = 0;
    if (sok && dev != 0 && B + tg.off == dev) {
      // the value the slot holds before this launch touches it, and the one
      // a first tile elsewhere may already have left in it
      const uint64_t before = att ? tg.host : dev;
      const uint64_t other = att ? dev : tg.host;
      if (v == before || (!first && (att || det) && v == other)) a = dev;
      else report_bad_slot(t.hdr, so);
    } else {
      report_wild(t.hdr);
    }
    addr[tid] = a;
    soff[tid] = so | (first && a ? kFirstBit : 0);
    host[tid] = tg.host;
  }
  // LDS only: the attach stores need not complete before the compute
  lds_barrier();
#pragma unroll
  for (int k = 0; k < U; k++)
    if (addr[r[k].i] == 0) r[k].nb = 0;
  tile_round_store<U>(la, addr, info, outo, r);
  if (Q && tid == 0) *tick_dst = *tick_src;
  for (uint64_t c_lo = tl.c_lo + (uint64_t)bs * U; c_lo < tl.c_hi; c_lo += (uint64_t)bs * U) {
    tile_round_load<U>(la, pre, addr, info, outo, nl, c_lo, tl.c_hi, r);
    tile_round_store<U>(la, addr, info, outo, r);
  }
  // the first tile of each leaf writes the slot: the arena address (attach)
  // or the host address (detach), after the compute, by the thread that read
  // it. Nothing in this launch needs the attached value (every tile computes
  // at the planned address), and attach and detach together leave the slot
  // holding the host address it was checked to hold: nothing to write
  if (att != det && tid < (int)nl && (soff[tid] & kFirstBit))
    *(g_u64*)(B + (soff[tid] & ~kFirstBit)) = att ? addr[tid] : host[tid];
  lds_barrier();
}

// bs of the other slots: translated as the relocation kernel would (attach,
// then detach when both are asked for)
__device__ void fused_resid(const Tables& t, uint64_t blk, uint32_t flags) {
  const uint64_t k = blk * blockDim.x + threadIdx.x;
  if (k >= t.nresid) return;
  const bool att = (flags & DC_BATCH_ATTACH) != 0, det = (flags & DC_BATCH_DETACH) != 0;
  const uint64_t B = (uint64_t)t.arena;
  const DevResid r = t.resid[k];
  if (!in_arena(t, B + r.slot_off, 8)) {
    report_wild(t.hdr);
    return;
  }
  g_u64* slot = (g_u64*)(B + r.slot_off);
  const uint64_t v = *slot;
  if (v == 0) return;
  // a member left out of a selective copy reads as null on the device (the
  // zero is made here: the compiler would otherwise hold it from the
  // kernel's start, spilled to scratch by every thread of the launch)
  if (!r.follow) {
    uint64_t zero = 0;
    asm volatile("" : "+v"(zero));
    *slot = zero;
    return;
  }
  if (r.tgt == kNone) {
    report_bad_slot(t.hdr, r.slot_off);
    return;
  }
  const DevTarget tg = t.tgts[r.tgt];
  const uint64_t dev = B + tg.off;
  if (v != (att ? tg.host : dev)) {
    report_bad_slot(t.hdr, r.slot_off);
    return;
  }
  // attach and detach together leave the checked host address in place
  if (att != det) *slot = att ? dev : tg.host;
}

template <int U>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) k_fused(Tables t, LeafArgs la, uint64_t ntiles, uint64_t nitems,
                                               uint32_t flags) {
  __shared__ __align__(16) uint8_t lds[kFusedLds];
  for (uint64_t item = blockIdx.x; item < nitems; item += gridDim.x) {
    if (item < ntiles) fused_tile<U>(t, la, item, flags, lds);
    else fused_resid(t, item - ntiles, flags);
  }
}

// The same items in a persistent grid. A grid-stride loop lets the
// workgroups drift apart over the arena, which HBM serves more slowly than
// the compact, advancing window of one item per workgroup in dispatch order;
// taking items from a queue keeps that window. One queue is bound by its
// atomic's throughput (on a flat 12 GiB stream of 16 KB tiles, 2.8 TB/s), so
// there are kFusedQueues of them, interleaved: the workgroup with index b
// takes tickets from queue q = b mod kFusedQueues, and ticket k names item
// k * kFusedQueues + q (the items the dispatcher would send to the same
// XCD). Every item is taken exactly once and no workgroup waits for another,
// so the launch ends whatever the order. The queues are reset before each
// launch (launch_reset_counters).
// One ticket from a queue: an atomic increment (wrapping at 2^32), which,
// unlike an atomic add, the compiler leaves as it is written; for an add to
// a wave-uniform address it would combine the wave's atomics into one and
// wait for its return at once to share it out. A global (not generic)
// address, so that the atomic does not hold up waits for LDS.
typedef __attribute__((address_space(1))) uint32_t g_u32;
__device__ __forceinline__ uint32_t ticket(DevHeader* hdr, uint32_t q) {
  // the queue's offset passes through an empty asm where it is used, so that
  // its address is formed there in scalar registers: hoisted out of the item
  // loop, the compiler keeps a vector copy of it spilled to scratch, whose
  // reload waits for every store the wave has in flight
  uint32_t w = q * 32;  // the queue's first word in hdr->fq
  asm volatile("" : "+s"(w));
  return __builtin_amdgcn_atomic_inc32((g_u32*)(hdr->fq + w), 0xffffffffu, __ATOMIC_RELAXED, "agent");
}

template <int U>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_fused_persistent(Tables t, LeafArgs la, uint64_t ntiles, uint64_t nitems, uint32_t flags) {
  __shared__ __align__(16) uint8_t lds[kFusedLds];
  __shared__ uint32_t tick[2];
  const uint32_t q = blockIdx.x % kFusedQueues;
  if (threadIdx.x == 0) tick[0] = ticket(t.hdr, q);
  lds_barrier();
  for (uint32_t cur = 0;; cur ^= 1) {
    // the same for every thread: taken as a scalar, so the item's descriptor
    // is a scalar load, which no earlier vector store holds up
    const uint64_t item = (uint64_t)__builtin_amdgcn_readfirstlane(tick[cur]) * kFusedQueues + q;
    if (item >= nitems) break;
    // Set and read by thread 0 only. Setting it in the other threads too would
    // make the whole wave wait, before every item, for the register the last
    // ticket returned into, and with it for every store the wave has in flight.
    uint32_t next;
    if (threadIdx.x == 0) next = ticket(t.hdr, q);
    if (item < ntiles) {
      fused_tile<U, true>(t, la, item, flags, lds, &tick[cur ^ 1], &next);
    } else {
      fused_resid(t, item - ntiles, flags);
      if (threadIdx.x == 0) tick[cur ^ 1] = next;
      lds_barrier();
    }
  }
}

// ---- molecular dynamics: kick then drift on sibling leaves ------------------------------
//
// One tile: a range of 16-byte chunks of the elements' arrays laid end to
// end (each element contributes ceil(count / 2) chunks; 256 per tile), at
// most kTileMaxLeaves elements. The element's three array addresses are read once
// per tile from its relocated slots (the resolved form of Section 3) and
// checked against the arena; per chunk: v = fma(f, dt/m, v), x = fma(v, dt, x).
constexpr size_t kKdLds = (size_t)(kTileMaxLeaves + 2) * 5 * 8;

template <int U, bool NT>
__global__ void __launch_bounds__(256) k_kick_drift(Tables t, KickDriftArgs k) {
  __shared__ __align__(16) uint8_t lds[kKdLds];
  constexpr uint32_t N = kTileMaxLeaves + 2;
  uint64_t* pre = (uint64_t*)lds;
  uint64_t* xa = pre + N;
  uint64_t* va = xa + N;
  uint64_t* fa = va + N;
  uint64_t* cnt = fa + N;
  const int tid = threadIdx.x, bs = blockDim.x;
  for (uint64_t tile = blockIdx.x; tile < k.ntiles; tile += gridDim.x) {
    const DevTile tl = k.tiles[tile];
    const uint32_t e0 = tl.l_lo, nl = tl.l_hi - tl.l_lo + 1;
    for (uint32_t i = tid; i < nl; i += bs) {
      const DevTriple tr = k.tri[e0 + i];
      const uint64_t el = (uint64_t)t.arena + tr.elem_off;
      const uint64_t need = tr.count * 8;
      uint64_t x = *(const g_u64*)(el + k.x_off), v = *(const g_u64*)(el + k.v_off),
               f = *(const g_u64*)(el + k.f_off);
      if (!in_arena(t, x, need) || !in_arena(t, v, need) || !in_arena(t, f, need)) {
        report_wild(t.hdr);
        x = v = f = 0;
      }
      pre[i] = k.pre[e0 + i];
      xa[i] = x;
      va[i] = v;
      fa[i] = f;
      cnt[i] = tr.count;
    }
    if (tid == 0) pre[nl] = k.pre[tl.l_hi + 1];
    lds_barrier();  // the element table; no global memory is shared between threads
    for (uint64_t c_lo = tl.c_lo; c_lo < tl.c_hi; c_lo += (uint64_t)bs * U) {
      Vec16 X[U], V[U], F[U];
      uint64_t xd[U], vd[U];
      uint32_t ne[U];  // doubles in this chunk: 0, 1 or 2
#pragma unroll
      for (int u = 0; u < U; u++) {
        const uint64_t c = c_lo + (uint64_t)u * bs + tid;
        ne[u] = 0;
        xd[u] = vd[u] = 0;
        if (c < tl.c_hi) {
          const uint32_t i = find_leaf(pre, nl, c);
          const uint64_t e = (c - pre[i]) * 2;  // first double of the chunk
          ne[u] = xa[i] == 0 ? 0 : (cnt[i] - e >= 2 ? 2u : (uint32_t)(cnt[i] - e));
          xd[u] = xa[i] + e * 8;
          vd[u] = va[i] + e * 8;
          if (ne[u] == 2) {
            X[u].u = sload16<NT>(xd[u]);
            V[u].u = sload16<NT>(vd[u]);
            F[u].u = sload16<NT>(fa[i] + e * 8);
          } else if (ne[u] == 1) {
            X[u].d[0] = *(const g_double*)xd[u];
            V[u].d[0] = *(const g_double*)vd[u];
            F[u].d[0] = *(const g_double*)(fa[i] + e * 8);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        if (ne[u] == 2) {
          V[u].d[0] = __builtin_fma(F[u].d[0], k.dt_over_m, V[u].d[0]);
          V[u].d[1] = __builtin_fma(F[u].d[1], k.dt_over_m, V[u].d[1]);
          X[u].d[0] = __builtin_fma(V[u].d[0], k.dt, X[u].d[0]);
          X[u].d[1] = __builtin_fma(V[u].d[1], k.dt, X[u].d[1]);
          sstore16<NT>(vd[u], V[u].u);
          sstore16<NT>(xd[u], X[u].u);
        } else if (ne[u] == 1) {
          const double v1 = __builtin_fma(F[u].d[0], k.dt_over_m, V[u].d[0]);
          *(g_double*)vd[u] = v1;
          *(g_double*)xd[u] = __builtin_fma(v1, k.dt, X[u].d[0]);
        }
      }
    }
    lds_barrier();  // before the next tile rewrites the table; no wait for this tile's stores
  }
}

// ---- persistent relocate + compute ------------------------------------------------------------
//
// One launch, one device work queue. Items: [attach units][compute tile
// batches][detach units]. A workgroup takes items in queue order. The
// compute items read the slots that attach units write, and detach units
// overwrite slots that compute items read, so a workgroup waits before its
// first compute item until every attach unit is done and before its first
// detach unit until every compute item is done. Every item a workgroup waits
// on was taken earlier by a running workgroup, so the waits end; they are
// bounded anyway (past the bound the kernel records kErrSpin and proceeds, so
// every wave exits). A workgroup reports its finished items of a phase once,
// when it moves past that phase: one device-scope release per workgroup
// rather than one per item (a release writes back the XCD's L2).

// The poll is relaxed and one acquire fence follows the wait: an acquire
// load at device scope invalidates the XCD's L2 on every poll, which, from
// hundreds of waiting workgroups, keeps dropping the lines the working ones
// stream through.
__device__ __forceinline__ uint32_t ld_relaxed(uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ void wait_count(DevHeader* hdr, uint32_t* ctr, uint32_t target, uint32_t spin_limit) {
  if (threadIdx.x == 0) {
    uint32_t spins = 0;
    while (ld_relaxed(ctr) < target) {
      __builtin_amdgcn_s_sleep(32);
      if (++spins > spin_limit) {
        atomicCAS(&hdr->err_code, 0u, (uint32_t)kErrSpin);
        atomicAdd(&hdr->spin_fail, 1u);
        break;
      }
    }
    // synchronizes with the release of the increments the poll has read;
    // the barrier then orders the other threads after it
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// adds n finished items to a phase counter; release: publish this
// workgroup's stores (the relocated slots) before the count
__device__ __forceinline__ void report_done(uint32_t* ctr, uint32_t n, bool release) {
  if (release) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0 && n) {
    if (release) __hip_atomic_fetch_add(ctr, n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    else __hip_atomic_fetch_add(ctr, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// BS threads per workgroup; resources held to eight waves per SIMD, so that
// a CU runs 2048 threads of the loop at once, as it does for the leaf kernel
template <int U, int BS>
__global__ void __launch_bounds__(BS, 8) k_batch(Tables t, LeafArgs la, uint32_t flags, uint64_t ntiles,
                                                  uint32_t per_item, uint32_t spin_limit) {
  constexpr int KS = (int)((kSegMaxSlots + BS - 1) / BS);
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ uint32_t s_item;
  DevHeader* hdr = t.hdr;
  const uint32_t nA = (flags & DC_BATCH_ATTACH) ? (uint32_t)t.nseg : 0;
  const uint32_t nB = (uint32_t)((ntiles + per_item - 1) / per_item);
  const uint32_t nC = (flags & DC_BATCH_DETACH) ? (uint32_t)t.nseg : 0;
  const uint32_t total = nA + nB + nC;
  // forced error path: each wait waits for one item more than its phase has
  const uint32_t extra = (flags & DC_BATCH_FORCE_WAIT_BOUND) ? 1u : 0u;
  uint32_t myA = 0, myB = 0;  // items finished and not yet reported
  bool pastA = false, pastB = false, waitedB = false;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&hdr->queue, 1u);
    lds_barrier();
    const uint32_t item = s_item;
    lds_barrier();
    if (!pastA && item >= nA) {
      report_done(&hdr->doneA, myA, true);
      pastA = true;
    }
    if (!pastB && item >= nA + nB) {
      // compute items only read slots: their count needs no release
      report_done(&hdr->doneB, myB, false);
      pastB = true;
    }
    if (item >= total) break;
    if (item < nA) {
      relocate_unit<false, KS>(t, item, true, lds);
      lds_barrier();
      myA++;
    } else if (item < nA + nB) {
      if (myB == 0) wait_count(hdr, &hdr->doneA, nA + extra, spin_limit);
      const uint64_t tlo = (uint64_t)(item - nA) * per_item;
      const uint64_t thi = tlo + per_item < ntiles ? tlo + per_item : ntiles;
      for (uint64_t tile = tlo; tile < thi; tile++) leaf_tile<U, false>(t, la, tile, lds);
      myB++;
    } else {
      if (!waitedB) {
        wait_count(hdr, &hdr->doneB, nB + extra, spin_limit);
        waitedB = true;
      }
      relocate_unit<false, KS>(t, item - nA - nB, false, lds);
      lds_barrier();
    }
  }
}

// ---- persistent relocate + compute, one item per relocation unit ---------------------------
//
// When every relocation unit's slots are the first to reach one contiguous run
// of leaves (the plan records the run in the unit), a unit's attach, the
// kernel over its leaves and its detach depend on nothing another unit does:
// the leaves' addresses are read from slots of that unit alone, and its
// detach rewrites slots that only its own leaves were reached through. One
// workgroup then takes a whole unit as one item of the device queue, with
// workgroup-scope ordering only, and no workgroup ever waits for another.
// With ATTACH and DETACH both, the detach writes back the slot values the
// attach read, held in registers; alone, it translates through the unit's
// LDS table as the separate reverse relocation does.

// Every chunk of leaves [l0, l1) (at most kTileMaxLeaves of them), in rounds
// of U chunks per thread; each leaf's address is read once from its relocated
// parent slot. Ends with an LDS barrier: the next run may overwrite the tables.
template <int U>
__device__ void leaf_run(const Tables& t, const LeafArgs& la, uint32_t l0, uint32_t l1, uint8_t* lds) {
  constexpr uint32_t N = kTileMaxLeaves + 2;
  uint64_t* pre = (uint64_t*)lds;
  uint64_t* addr = pre + N;
  uint64_t* info = addr + N;
  uint64_t* outo = info + N;
  const int tid = threadIdx.x, bs = blockDim.x;
  const uint32_t nl = l1 - l0;
  for (uint32_t i = tid; i <= nl; i += bs) {
    const uint32_t l = l0 + i;
    pre[i] = t.leaf_pre[l];
    if (i == nl) continue;
    const uint64_t inf = t.leaf_info[l];
    info[i] = inf;
    outo[i] = t.leaf_out[l];
    const uint64_t a = *(const g_u64*)((uint64_t)t.arena + t.leaf_slot[l]);
    if (in_arena(t, a, inf & ((1ull << kLeafKindShift) - 1))) {
      addr[i] = a;
    } else {
      addr[i] = 0;
      report_wild(t.hdr);
    }
  }
  lds_barrier();
  const uint64_t c_end = pre[nl];
  for (uint64_t c_lo = pre[0]; c_lo < c_end; c_lo += (uint64_t)bs * U) {
    Vec16 v[U];
    uint64_t src[U], dst[U];
    uint32_t nb[U];
    bool f64[U];
#pragma unroll
    for (int k = 0; k < U; k++) {
      const uint64_t c = c_lo + (uint64_t)k * bs + tid;
      nb[k] = 0;
      f64[k] = false;
      src[k] = dst[k] = 0;
      if (c < c_end) {
        const uint32_t i = find_leaf(pre, nl, c);
        const uint64_t byte = (c - pre[i]) * kChunk;
        const uint64_t lb = info[i] & ((1ull << kLeafKindShift) - 1);
        f64[k] = (info[i] >> kLeafKindShift) == DC_KIND_F64;
        nb[k] = addr[i] == 0 ? 0 : (uint32_t)(lb - byte < kChunk ? lb - byte : kChunk);
        src[k] = (la.src_out ? (uint64_t)la.out + outo[i] : addr[i]) + byte;
        dst[k] = (la.out ? (uint64_t)la.out + outo[i] : addr[i]) + byte;
      }
      if (nb[k] == kChunk) v[k].u = gload16(src[k]);
    }
#pragma unroll
    for (int k = 0; k < U; k++) {
      if (nb[k] == kChunk) {
        fma_chunk_any(v[k], f64[k], la);
        gstore16(dst[k], v[k].u);
      }
    }
#pragma unroll
    for (int k = 0; k < U; k++)
      if (nb[k] != 0 && nb[k] != kChunk) fma_partial(src[k], dst[k], nb[k], f64[k] ? DC_KIND_F64 : DC_KIND_F32, la);
  }
  lds_barrier();
}

template <int U, int BS>
__global__ void __launch_bounds__(BS, 8) k_batch_units(Tables t, LeafArgs la, uint32_t flags) {
  constexpr int KS = (int)((kSegMaxSlots + BS - 1) / BS);
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ uint32_t s_item;
  const bool att = (flags & DC_BATCH_ATTACH) != 0, det = (flags & DC_BATCH_DETACH) != 0;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&t.hdr->queue, 1u);
    lds_barrier();
    const uint32_t u = s_item;
    lds_barrier();
    if (u >= t.nseg) break;
    uint64_t koff[KS], kval[KS];
    if (att) {
      relocate_unit<true, KS>(t, u, true, lds, koff, kval);
      // the translated slots (global stores of other threads) are read below
      __syncthreads();
    }
    const uint32_t lhi = t.segs[u].leaf_hi;
    for (uint32_t l = t.segs[u].leaf_lo; l < lhi; l += kTileMaxLeaves)
      leaf_run<U>(t, la, l, l + kTileMaxLeaves < lhi ? l + kTileMaxLeaves : lhi, lds);
    if (det) {
      if (att) {
        // every read of these slots completed before the last run's barrier
#pragma unroll
        for (int k = 0; k < KS; k++) {
          if (koff[k] == ~0ull) continue;
          if (koff[k] & kKeepBad) report_bad_slot(t.hdr, koff[k] & ~kKeepBad);
          else *(g_u64*)((uint64_t)t.arena + koff[k]) = kval[k];
        }
      } else {
        relocate_unit<false, KS>(t, u, false, lds);
      }
    }
    lds_barrier();
  }
}

__global__ void k_reset_counters(DevHeader* hdr) {
  if (threadIdx.x == 0) {
    hdr->queue = 0;
    hdr->doneA = 0;
    hdr->doneB = 0;
  }
  if (threadIdx.x < kFusedQueues) hdr->fq[threadIdx.x * 32] = 0;
}

}  // namespace

int device_cu_count() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
  return n;
}

hipError_t launch_relocate(const Tables& t, bool attach, hipStream_t s) {
  if (t.nseg == 0) return hipSuccess;
  const uint64_t grid = t.nseg < 65536 ? t.nseg : 65536;
  if (t.ntypes > kMaxTypes) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_relocate, dim3((uint32_t)grid), dim3(kRelocBlock), reloc_lds_bytes(t.ntypes), s, t,
                     attach ? 1 : 0);
  return hipGetLastError();
}

// Streams of at least this many bytes per pass use non-temporal accesses:
// larger than the 256 MB Infinity Cache, they are not read again from it.
#ifndef DC_STREAM_NT_BYTES
#define DC_STREAM_NT_BYTES (256ull << 20)
#endif
static bool stream_nt(uint64_t bytes) { return bytes >= (uint64_t)DC_STREAM_NT_BYTES; }

hipError_t launch_scalar(const Tables& t, const DevScalar* refs, const DevScalarHop* hops, uint32_t n,
                         uint64_t* temps, int update, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scalar, dim3((n + 255) / 256), dim3(256), 0, s, t, refs, hops, n, temps, update);
  return hipGetLastError();
}

hipError_t launch_kick_drift(const Tables& t, const KickDriftArgs& k, hipStream_t s) {
  if (k.ntiles == 0) return hipSuccess;
  const uint64_t grid = k.ntiles < (1u << 20) ? k.ntiles : (1u << 20);
  // one chunk per thread (256-chunk tiles), at full occupancy: measured on
  // 10,000 MD simulations (19.8 GB per step) 3.86 ms, against 4.07 ms with two
  // chunks per thread at five workgroups per CU (4.47 at eight) and 4.3-4.7 ms
  // with four
  // the three arrays of every element are leaves of the tree: its leaf bytes decide
  if (stream_nt(t.total_chunks * kChunk))
    hipLaunchKernelGGL((k_kick_drift<1, true>), dim3((uint32_t)grid), dim3(256), 0, s, t, k);
  else
    hipLaunchKernelGGL((k_kick_drift<1, false>), dim3((uint32_t)grid), dim3(256), 0, s, t, k);
  return hipGetLastError();
}

hipError_t launch_resolve_chain(const Tables& t, const ChainArgs& c, hipStream_t s) {
  hipLaunchKernelGGL(k_resolve_chain, dim3(1), dim3(64), 0, s, t, c);
  return hipGetLastError();
}

hipError_t launch_stream_resolved(const Tables& t, uint64_t base, uint64_t count, uint32_t kind, const LeafArgs& la,
                                  hipStream_t s) {
  // One 16-byte chunk per thread and a grid covering the array: on nonzero
  // data this measured fastest both for arrays resident in the 256 MB
  // Infinity Cache (7.1 TB/s on 128 MiB) and for HBM-sized ones (5.9 TB/s
  // on 2-12 GiB), ahead of grid-stride loops with more chunks per thread.
  const uint64_t bytes = count * (kind == DC_KIND_F64 ? 8 : 4);
  const uint64_t chunks = bytes / kChunk;
  constexpr int U = 1;
  uint64_t blocks = (chunks + 256ull * U - 1) / (256ull * U);
  if (blocks > (1ull << 31) - 1) blocks = (1ull << 31) - 1;
  if (blocks == 0) blocks = 1;
  const bool nt = stream_nt(bytes);
  if (kind == DC_KIND_F64 && nt)
    hipLaunchKernelGGL((k_stream_resolved<U, double, true>), dim3((uint32_t)blocks), dim3(256), 0, s, t, base, count, la);
  else if (kind == DC_KIND_F64)
    hipLaunchKernelGGL((k_stream_resolved<U, double, false>), dim3((uint32_t)blocks), dim3(256), 0, s, t, base, count, la);
  else if (nt)
    hipLaunchKernelGGL((k_stream_resolved<U, float, true>), dim3((uint32_t)blocks), dim3(256), 0, s, t, base, count, la);
  else
    hipLaunchKernelGGL((k_stream_resolved<U, float, false>), dim3((uint32_t)blocks), dim3(256), 0, s, t, base, count, la);
  return hipGetLastError();
}

hipError_t launch_stream_deref(const Tables& t, const HopArgs& h, uint64_t count, uint32_t kind,
                               const LeafArgs& la, hipStream_t s) {
  constexpr int U = 4;
  const uint64_t blocks = (count + 256ull * U - 1) / (256ull * U);
  if (blocks == 0) return hipSuccess;
  if (h.nhops > kMaxChainSteps) return hipErrorInvalidValue;
  const bool nt = stream_nt(count * (kind == DC_KIND_F64 ? 8 : 4));
#define DC_DEREF_T(MAXH, T)                                                                                          \
  if (nt)                                                                                                            \
    hipLaunchKernelGGL((k_stream_deref<U, MAXH, T, true>), dim3((uint32_t)blocks), dim3(256), 0, s, t, h, count, la);  \
  else                                                                                                               \
    hipLaunchKernelGGL((k_stream_deref<U, MAXH, T, false>), dim3((uint32_t)blocks), dim3(256), 0, s, t, h, count, la);
#define DC_DEREF(MAXH)       \
  if (kind == DC_KIND_F64) { \
    DC_DEREF_T(MAXH, double) \
  } else {                   \
    DC_DEREF_T(MAXH, float)  \
  }
  if (h.nhops <= 4) {
    DC_DEREF(4)
  } else if (h.nhops <= 8) {
    DC_DEREF(8)
  } else if (h.nhops <= 16) {
    DC_DEREF(16)
  } else {
    DC_DEREF(32)
  }
#undef DC_DEREF
#undef DC_DEREF_T
  return hipGetLastError();
}

hipError_t launch_leaf_tiles(const Tables& t, const LeafArgs& la, uint64_t ntiles, uint32_t tile_chunks,
                             bool deref_each, hipStream_t s) {
  if (ntiles == 0) return hipSuccess;
  const uint64_t grid = ntiles < (1u << 20) ? ntiles : (1u << 20);
  // RESOLVED: one round per tile for 512- and 1024-chunk tiles (two or four
  // chunks per thread), rounds of 1024 for larger ones
  // (the sweep of chunks per thread x non-temporal accesses on the MD leaves,
  // best tile size each: 1 chunk 4.46 ms, 2 4.44, 4 4.25; non-temporal 4.72-4.95)
  if (deref_each)
    hipLaunchKernelGGL((k_leaf_tiles<4, true>), dim3((uint32_t)grid), dim3(256), 0, s, t, la, ntiles);
  else if (tile_chunks <= 512)
    hipLaunchKernelGGL((k_leaf_tiles<2, false>), dim3((uint32_t)grid), dim3(256), 0, s, t, la, ntiles);
  else
    hipLaunchKernelGGL((k_leaf_tiles<4, false>), dim3((uint32_t)grid), dim3(256), 0, s, t, la, ntiles);
  return hipGetLastError();
}

hipError_t launch_batch(const Tables& t, const LeafArgs& la, uint32_t flags, uint32_t block, uint32_t grid,
                        uint64_t ntiles, uint32_t spin_limit, hipStream_t s) {
  if (t.ntypes > kMaxTypes) return hipErrorInvalidValue;
  const size_t rl = reloc_lds_bytes(t.ntypes);
  const size_t lds = kTileLds > rl ? kTileLds : rl;
  // compute tiles are taken a few at a time, so that the queue sees about 32
  // items per workgroup rather than one atomic per tile
  const uint64_t per = ntiles / ((uint64_t)grid * 32 + 1) + 1;
  const uint32_t per_item = (uint32_t)(per > 256 ? 256 : per);
  // chunks per thread per round: 1024 chunks per workgroup round (512 with
  // 256 threads: four chunks per thread would spill within the register
  // budget of eight waves per SIMD)
  switch (block) {
    case 256:
      hipLaunchKernelGGL((k_batch<2, 256>), dim3(grid), dim3(block), lds, s, t, la, flags, ntiles, per_item, spin_limit);
      break;
    case 512:
      hipLaunchKernelGGL((k_batch<2, 512>), dim3(grid), dim3(block), lds, s, t, la, flags, ntiles, per_item, spin_limit);
      break;
    case 1024:
      hipLaunchKernelGGL((k_batch<1, 1024>), dim3(grid), dim3(block), lds, s, t, la, flags, ntiles, per_item, spin_limit);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_units(const Tables& t, const LeafArgs& la, uint32_t flags, uint32_t block, uint32_t grid,
                              hipStream_t s) {
  if (t.ntypes > kMaxTypes) return hipErrorInvalidValue;
  const size_t rl = reloc_lds_bytes(t.ntypes);
  const size_t lds = kTileLds > rl ? kTileLds : rl;
  switch (block) {
    case 256:
      hipLaunchKernelGGL((k_batch_units<2, 256>), dim3(grid), dim3(block), lds, s, t, la, flags);
      break;
    case 512:
      hipLaunchKernelGGL((k_batch_units<2, 512>), dim3(grid), dim3(block), lds, s, t, la, flags);
      break;
    case 1024:
      hipLaunchKernelGGL((k_batch_units<1, 1024>), dim3(grid), dim3(block), lds, s, t, la, flags);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fused(const Tables& t, const LeafArgs& la, uint64_t ntiles, uint32_t tile_chunks, uint32_t flags,
                        hipStream_t s) {
  const uint64_t nitems = ntiles + (t.nresid + 255) / 256;
  if (nitems == 0) return hipSuccess;
  const uint64_t grid = nitems < (1u << 20) ? nitems : (1u << 20);
  if (tile_chunks <= 512)
    hipLaunchKernelGGL((k_fused<2>), dim3((uint32_t)grid), dim3(256), 0, s, t, la, ntiles, nitems, flags);
  else
    hipLaunchKernelGGL((k_fused<4>), dim3((uint32_t)grid), dim3(256), 0, s, t, la, ntiles, nitems, flags);
  return hipGetLastError();
}

hipError_t launch_fused_persistent(const Tables& t, const LeafArgs& la, uint64_t ntiles, uint32_t tile_chunks,
                                   uint32_t flags, uint32_t grid, hipStream_t s) {
  const uint64_t nitems = ntiles + (t.nresid + 255) / 256;
  if (nitems == 0) return hipSuccess;
  // every queue needs a workgroup: its items are taken by no other
  if (grid < kFusedQueues) grid = kFusedQueues;
  // tickets are 32-bit
  if (nitems / kFusedQueues >= 0xffffffffull - grid) return hipErrorInvalidValue;
  if (tile_chunks <= 512)
    hipLaunchKernelGGL((k_fused_persistent<2>), dim3(grid), dim3(256), 0, s, t, la, ntiles, nitems, flags);
  else
    hipLaunchKernelGGL((k_fused_persistent<4>), dim3(grid), dim3(256), 0, s, t, la, ntiles, nitems, flags);
  return hipGetLastError();
}

hipError_t launch_reset_counters(DevHeader* hdr, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, hdr);
  return hipGetLastError();
}

}  // namespace dc
