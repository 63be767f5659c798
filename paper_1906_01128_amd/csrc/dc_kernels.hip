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

constexpr int kRelocBlock = 256;

// LDS of one relocation unit: open-addressing hash of (key -> object) and
// the slot prefix of the struct arrays the unit spans.
constexpr size_t kRelocLds = kSegHashSlots * 8 + kSegHashSlots * 4 + (kSegMaxSObjs + 1) * 8;

__device__ __forceinline__ uint32_t hash_slot(uint64_t key) {
  // multiplicative hashing; keys are 16-byte aligned addresses
  return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - 11)) & (kSegHashSlots - 1);
}
static_assert(kSegHashSlots == 2048, "hash_slot assumes 2^11 slots");

__device__ __forceinline__ void hash_insert(uint64_t* keys, uint32_t* vals, uint64_t key, uint32_t val) {
  uint32_t h = hash_slot(key);
  for (uint32_t probe = 0; probe < kSegHashSlots; probe++) {
    unsigned long long prev = atomicCAS((unsigned long long*)&keys[h], 0ull, (unsigned long long)key);
    if (prev == 0ull || prev == key) {
      vals[h] = val;
      return;
    }
    h = (h + 1) & (kSegHashSlots - 1);
  }
}

__device__ __forceinline__ uint32_t hash_find(const uint64_t* keys, const uint32_t* vals, uint64_t key) {
  uint32_t h = hash_slot(key);
  for (uint32_t probe = 0; probe < kSegHashSlots; probe++) {
    uint64_t k = keys[h];
    if (k == key) return vals[h];
    if (k == 0) return kNone;
    h = (h + 1) & (kSegHashSlots - 1);
  }
  return kNone;
}

__device__ __forceinline__ void report_bad_slot(DevHeader* hdr, uint64_t slot_off) {
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
// -> arena address; detach: arena address -> host address. A slot holding a
// value that is not one of the unit's planned targets is left alone and
// reported in the header.
__device__ void relocate_unit(const Tables& t, uint64_t sg, bool attach, uint8_t* lds) {
  uint64_t* keys = (uint64_t*)lds;
  uint32_t* vals = (uint32_t*)(keys + kSegHashSlots);
  uint64_t* pre = (uint64_t*)(vals + kSegHashSlots);
  const int tid = threadIdx.x, bs = blockDim.x;
  const DevSeg seg = t.segs[sg];
  const uint64_t B = (uint64_t)t.arena;

  for (uint32_t i = tid; i < kSegHashSlots; i += bs) keys[i] = 0;
  const uint32_t nso = seg.sobj_hi - seg.sobj_lo;
  for (uint32_t i = tid; i <= nso; i += bs) pre[i] = t.sobj_pre[seg.sobj_lo + i];
  __syncthreads();
  const uint32_t ntgt = (uint32_t)(seg.tgt_hi - seg.tgt_lo);
  for (uint32_t i = tid; i < ntgt; i += bs) {
    uint32_t obj = t.targets[seg.tgt_lo + i];
    uint64_t key = attach ? t.obj_host[obj] : B + t.obj_off[obj];
    hash_insert(keys, vals, key, obj);
  }
  __syncthreads();

  for (uint64_t j = seg.slot_lo + tid; j < seg.slot_hi; j += bs) {
    // struct array holding slot j: largest i with pre[i] <= j
    uint32_t lo = 0, hi = nso;
    while (hi - lo > 1) {
      uint32_t mid = (lo + hi) >> 1;
      if (pre[mid] <= j) lo = mid;
      else hi = mid;
    }
    const DevSObj so = t.sobj[seg.sobj_lo + lo];
    const DevType* ty = &t.types[so.type];
    const uint32_t nptr = ty->nptr;
    const uint64_t local = j - pre[lo];
    const uint64_t e = local / nptr;
    const uint32_t f = (uint32_t)(local - e * nptr);
    const uint64_t slot_off = so.off + e * ty->size + ty->ptr_off[f];
    uint64_t* slot = (uint64_t*)(t.arena + slot_off);
    const uint64_t p = *slot;
    if (p == 0) continue;
    const uint32_t obj = hash_find(keys, vals, p);
    if (obj == kNone) {
      report_bad_slot(t.hdr, slot_off);
      continue;
    }
    *slot = attach ? B + t.obj_off[obj] : t.obj_host[obj];
  }
}

__global__ void __launch_bounds__(kRelocBlock) k_relocate(Tables t, int attach) {
  __shared__ __align__(16) uint8_t lds[kRelocLds];
  for (uint64_t sg = blockIdx.x; sg < t.nseg; sg += gridDim.x) {
    relocate_unit(t, sg, attach != 0, lds);
    __syncthreads();
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

// ---- leaf arithmetic ------------------------------------------------------------------

union Vec16 {
  uint4 u;
  double d[2];
  float f[4];
};

__device__ __forceinline__ void fma_chunk(Vec16& v, uint32_t kind, const LeafArgs& la) {
  if (kind == DC_KIND_F64) {
    v.d[0] = __builtin_fma(v.d[0], la.a, la.b);
    v.d[1] = __builtin_fma(v.d[1], la.a, la.b);
  } else {
    v.f[0] = __builtin_fmaf(v.f[0], la.af, la.bf);
    v.f[1] = __builtin_fmaf(v.f[1], la.af, la.bf);
    v.f[2] = __builtin_fmaf(v.f[2], la.af, la.bf);
    v.f[3] = __builtin_fmaf(v.f[3], la.af, la.bf);
  }
}

// the first `nbytes` (< 16) bytes of a chunk, element by element
__device__ __forceinline__ void fma_partial(const uint8_t* src, uint8_t* dst, uint32_t nbytes, uint32_t kind,
                                            const LeafArgs& la) {
  if (kind == DC_KIND_F64) {
    for (uint32_t o = 0; o + 8 <= nbytes; o += 8)
      *(double*)(dst + o) = __builtin_fma(*(const double*)(src + o), la.a, la.b);
  } else {
    for (uint32_t o = 0; o + 4 <= nbytes; o += 4)
      *(float*)(dst + o) = __builtin_fmaf(*(const float*)(src + o), la.af, la.bf);
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

template <int U>
__global__ void __launch_bounds__(256) k_stream_resolved(Tables t, uint64_t count, uint32_t kind, LeafArgs la) {
  if (t.hdr->chain_status != 0) return;
  uint8_t* base = (uint8_t*)t.hdr->chain_addr;  // resolved once, before the region
  if (!in_arena(t, (uint64_t)base, count * (kind == DC_KIND_F64 ? 8 : 4))) return;  // reported by the resolver
  const uint8_t* src = la.src_out ? la.out : base;
  uint8_t* dst = la.out ? la.out : base;
  const uint32_t es = kind == DC_KIND_F64 ? 8 : 4;
  const uint64_t bytes = count * es;
  const uint64_t nfull = bytes / kChunk;
  const uint64_t c0 = (uint64_t)blockIdx.x * blockDim.x * U + threadIdx.x;
  Vec16 v[U];
#pragma unroll
  for (int k = 0; k < U; k++) {
    const uint64_t c = c0 + (uint64_t)k * blockDim.x;
    if (c < nfull) v[k].u = *(const uint4*)(src + c * kChunk);
  }
#pragma unroll
  for (int k = 0; k < U; k++) {
    const uint64_t c = c0 + (uint64_t)k * blockDim.x;
    if (c < nfull) {
      fma_chunk(v[k], kind, la);
      *(uint4*)(dst + c * kChunk) = v[k].u;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && nfull * kChunk < bytes)
    fma_partial(src + nfull * kChunk, dst + nfull * kChunk, (uint32_t)(bytes - nfull * kChunk), kind, la);
}

// Every element access walks the chain from the root (Section 3: the cost
// the pointerchain directive removes). U independent elements per thread keep
// several walks in flight.
template <int U, typename T>
__global__ void __launch_bounds__(256) k_stream_deref(Tables t, HopArgs h, uint64_t count, LeafArgs la) {
  const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x * U + threadIdx.x;
  const uint8_t* p[U];
#pragma unroll
  for (int k = 0; k < U; k++) p[k] = t.arena + h.root_off;
  bool ok = true;
  for (uint32_t hop = 0; hop < h.nhops; hop++) {
    const uint64_t off = h.hop_off[hop];
#pragma unroll
    for (int k = 0; k < U; k++) {
      const uint8_t* slot = opaque(p[k]) + off;
      if (!in_arena(t, (uint64_t)slot, 8)) {
        ok = false;
        p[k] = t.arena;
      } else {
        p[k] = *(const uint8_t* const*)slot;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < U; k++) ok = ok && in_arena(t, (uint64_t)p[k], count * sizeof(T));
  if (!ok) {
    report_wild(t.hdr);
    return;
  }
  T x[U];
#pragma unroll
  for (int k = 0; k < U; k++) {
    const uint64_t i = i0 + (uint64_t)k * blockDim.x;
    const T* src = la.src_out ? (const T*)la.out : (const T*)p[k];
    if (i < count) x[k] = src[i];
  }
#pragma unroll
  for (int k = 0; k < U; k++) {
    const uint64_t i = i0 + (uint64_t)k * blockDim.x;
    T* dst = la.out ? (T*)la.out : (T*)p[k];
    if (i < count) {
      if constexpr (sizeof(T) == 8) dst[i] = __builtin_fma(x[k], la.a, la.b);
      else dst[i] = __builtin_fmaf(x[k], la.af, la.bf);
    }
  }
}

// ---- every leaf: 16-byte chunks of the concatenated leaves, in tiles ---------------------

__global__ void k_tile_index(Tables t, uint32_t T, uint64_t ntiles) {
  const uint64_t tile = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tile > ntiles) return;
  if (tile == ntiles) {
    t.tile_first[tile] = (uint32_t)(t.nleaves - 1);
    return;
  }
  const uint64_t c = tile * T;
  uint64_t lo = 0, hi = t.nleaves;  // largest l with leaf_pre[l] <= c
  while (hi - lo > 1) {
    uint64_t mid = (lo + hi) >> 1;
    if (t.leaf_pre[mid] <= c) lo = mid;
    else hi = mid;
  }
  t.tile_first[tile] = (uint32_t)lo;
}

__device__ __forceinline__ uint32_t find_leaf(const uint64_t* pre, uint32_t nl, uint64_t c) {
  uint32_t lo = 0, hi = nl;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (pre[mid] <= c) lo = mid;
    else hi = mid;
  }
  return lo;
}

__host__ __device__ constexpr size_t tile_lds_bytes(uint32_t T) { return (size_t)(T + 2) * 4 * 8; }

// One compute tile: chunks [tile*T, tile*T + T) of the leaf concatenation.
// RESOLVED: each leaf's address is read once per tile from its relocated
// parent slot. DEREF: each element access walks the leaf's whole path.
template <int U, bool DEREF>
__device__ void leaf_tile(const Tables& t, const LeafArgs& la, uint64_t tile, uint32_t T, uint8_t* lds) {
  uint64_t* pre = (uint64_t*)lds;
  uint64_t* addr = pre + (T + 2);
  uint64_t* info = addr + (T + 2);
  uint64_t* outo = info + (T + 2);
  const int tid = threadIdx.x, bs = blockDim.x;
  const uint32_t l0 = t.tile_first[tile], l1 = t.tile_first[tile + 1];
  const uint32_t nl = l1 - l0 + 1;
  for (uint32_t i = tid; i < nl; i += bs) {
    const uint32_t l = l0 + i;
    pre[i] = t.leaf_pre[l];
    info[i] = t.leaf_info[l];
    outo[i] = t.leaf_out[l];
    if (!DEREF) {
      const uint64_t a = *(const uint64_t*)(t.arena + t.leaf_slot[l]);
      const uint64_t lb = t.leaf_info[l] & ((1ull << kLeafKindShift) - 1);
      if (in_arena(t, a, lb)) {
        addr[i] = a;
      } else {
        addr[i] = 0;
        report_wild(t.hdr);
      }
    }
  }
  if (tid == 0) pre[nl] = t.leaf_pre[l1 + 1];
  __syncthreads();
  const uint64_t c_lo = tile * T;
  const uint64_t c_hi = c_lo + T < t.total_chunks ? c_lo + T : t.total_chunks;

  if (!DEREF) {
    Vec16 v[U];
    uint8_t* dst[U];
    uint32_t nb[U], kd[U];
#pragma unroll
    for (int k = 0; k < U; k++) {
      const uint64_t c = c_lo + (uint64_t)k * bs + tid;
      nb[k] = 0;
      if (c < c_hi) {
        const uint32_t i = find_leaf(pre, nl, c);
        if (addr[i] == 0) continue;
        const uint64_t byte = (c - pre[i]) * kChunk;
        const uint64_t lb = info[i] & ((1ull << kLeafKindShift) - 1);
        kd[k] = (uint32_t)(info[i] >> kLeafKindShift);
        nb[k] = (uint32_t)(lb - byte < kChunk ? lb - byte : kChunk);
        const uint8_t* src = (la.src_out ? la.out + outo[i] : (const uint8_t*)addr[i]) + byte;
        dst[k] = (la.out ? la.out + outo[i] : (uint8_t*)addr[i]) + byte;
        if (nb[k] == kChunk) v[k].u = *(const uint4*)src;
        else fma_partial(src, dst[k], nb[k], kd[k], la);
      }
    }
#pragma unroll
    for (int k = 0; k < U; k++) {
      if (nb[k] == kChunk) {
        fma_chunk(v[k], kd[k], la);
        *(uint4*)dst[k] = v[k].u;
      }
    }
  } else {
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
          if (ok) p = *(const uint8_t* const*)slot;
        }
        if (!ok || !in_arena(t, (uint64_t)p, lb)) {
          report_wild(t.hdr);
          break;
        }
        const uint8_t* src = (la.src_out ? la.out + outo[i] : p) + byte + o;
        uint8_t* d = (la.out ? la.out + outo[i] : (uint8_t*)p) + byte + o;
        if (kind == DC_KIND_F64) *(double*)d = __builtin_fma(*(const double*)src, la.a, la.b);
        else *(float*)d = __builtin_fmaf(*(const float*)src, la.af, la.bf);
      }
    }
  }
  __syncthreads();
}

template <int U, bool DEREF>
__global__ void __launch_bounds__(256) k_leaf_tiles(Tables t, LeafArgs la, uint32_t T, uint64_t ntiles) {
  extern __shared__ __align__(16) uint8_t lds[];
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) leaf_tile<U, DEREF>(t, la, tile, T, lds);
}

// ---- persistent relocate + compute ------------------------------------------------------------
//
// One launch, one device work queue. Items: [attach units][compute tile
// batches][detach units]. A workgroup takes items in queue order; before its
// first compute item it waits until every attach unit is done (they were all
// taken earlier, by running workgroups, so the wait ends), and before its
// first detach unit until every compute batch is done. The waits are bounded:
// past the bound the kernel records kErrSpin and proceeds, so every wave exits.

__device__ __forceinline__ uint32_t ld_acquire(uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ void wait_count(DevHeader* hdr, uint32_t* ctr, uint32_t target) {
  if (threadIdx.x == 0) {
    uint32_t spins = 0;
    while (ld_acquire(ctr) < target) {
      __builtin_amdgcn_s_sleep(4);
      if (++spins > (1u << 26)) {
        atomicCAS(&hdr->err_code, 0u, (uint32_t)kErrSpin);
        atomicAdd(&hdr->spin_fail, 1u);
        break;
      }
    }
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// every thread releases its own stores at device scope, then one thread
// counts the item as done
__device__ __forceinline__ void signal_done(uint32_t* ctr) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int U>
__global__ void k_batch(Tables t, LeafArgs la, uint32_t flags, uint32_t T, uint64_t ntiles, uint32_t per_item) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ uint32_t s_item;
  DevHeader* hdr = t.hdr;
  const uint32_t nA = (flags & DC_BATCH_ATTACH) ? (uint32_t)t.nseg : 0;
  const uint32_t nB = (uint32_t)((ntiles + per_item - 1) / per_item);
  const uint32_t nC = (flags & DC_BATCH_DETACH) ? (uint32_t)t.nseg : 0;
  const uint32_t total = nA + nB + nC;
  bool waitedA = false, waitedB = false;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&hdr->queue, 1u);
    __syncthreads();
    const uint32_t item = s_item;
    __syncthreads();
    if (item >= total) break;
    if (item < nA) {
      relocate_unit(t, item, true, lds);
      signal_done(&hdr->doneA);
    } else if (item < nA + nB) {
      if (!waitedA) {
        wait_count(hdr, &hdr->doneA, nA);
        waitedA = true;
      }
      const uint64_t b = item - nA;
      const uint64_t tlo = b * per_item;
      const uint64_t thi = tlo + per_item < ntiles ? tlo + per_item : ntiles;
      for (uint64_t tile = tlo; tile < thi; tile++) leaf_tile<U, false>(t, la, tile, T, lds);
      signal_done(&hdr->doneB);
    } else {
      if (!waitedB) {
        wait_count(hdr, &hdr->doneB, nB);
        waitedB = true;
      }
      relocate_unit(t, item - nA - nB, false, lds);
      __syncthreads();
    }
  }
}

__global__ void k_reset_counters(DevHeader* hdr) {
  if (threadIdx.x == 0) {
    hdr->queue = 0;
    hdr->doneA = 0;
    hdr->doneB = 0;
    hdr->doneC = 0;
  }
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
  hipLaunchKernelGGL(k_relocate, dim3((uint32_t)grid), dim3(kRelocBlock), 0, s, t, attach ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_resolve_chain(const Tables& t, const ChainArgs& c, hipStream_t s) {
  hipLaunchKernelGGL(k_resolve_chain, dim3(1), dim3(64), 0, s, t, c);
  return hipGetLastError();
}

hipError_t launch_stream_resolved(const Tables& t, uint64_t count, uint32_t kind, const LeafArgs& la,
                                  hipStream_t s) {
  constexpr int U = 4;
  const uint64_t bytes = count * (kind == DC_KIND_F64 ? 8 : 4);
  const uint64_t chunks = bytes / kChunk;
  uint64_t blocks = (chunks + 256ull * U - 1) / (256ull * U);
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_stream_resolved<U>, dim3((uint32_t)blocks), dim3(256), 0, s, t, count, kind, la);
  return hipGetLastError();
}

hipError_t launch_stream_deref(const Tables& t, const HopArgs& h, uint64_t count, uint32_t kind,
                               const LeafArgs& la, hipStream_t s) {
  constexpr int U = 4;
  uint64_t blocks = (count + 256ull * U - 1) / (256ull * U);
  if (blocks == 0) return hipSuccess;
  if (kind == DC_KIND_F64)
    hipLaunchKernelGGL((k_stream_deref<U, double>), dim3((uint32_t)blocks), dim3(256), 0, s, t, h, count, la);
  else
    hipLaunchKernelGGL((k_stream_deref<U, float>), dim3((uint32_t)blocks), dim3(256), 0, s, t, h, count, la);
  return hipGetLastError();
}

hipError_t launch_tile_index(const Tables& t, uint32_t T, uint64_t ntiles, hipStream_t s) {
  const uint64_t n = ntiles + 1;
  hipLaunchKernelGGL(k_tile_index, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, t, T, ntiles);
  return hipGetLastError();
}

hipError_t launch_leaf_tiles(const Tables& t, const LeafArgs& la, uint32_t T, uint64_t ntiles, bool deref_each,
                             hipStream_t s) {
  if (ntiles == 0) return hipSuccess;
  const size_t lds = tile_lds_bytes(T);
  const uint64_t grid = ntiles < (1u << 20) ? ntiles : (1u << 20);
  if (T == 1024) {
    if (deref_each)
      hipLaunchKernelGGL((k_leaf_tiles<4, true>), dim3((uint32_t)grid), dim3(256), lds, s, t, la, T, ntiles);
    else
      hipLaunchKernelGGL((k_leaf_tiles<4, false>), dim3((uint32_t)grid), dim3(256), lds, s, t, la, T, ntiles);
  } else if (T == 2048) {
    if (deref_each)
      hipLaunchKernelGGL((k_leaf_tiles<8, true>), dim3((uint32_t)grid), dim3(256), lds, s, t, la, T, ntiles);
    else
      hipLaunchKernelGGL((k_leaf_tiles<8, false>), dim3((uint32_t)grid), dim3(256), lds, s, t, la, T, ntiles);
  } else if (T == 512) {
    if (deref_each)
      hipLaunchKernelGGL((k_leaf_tiles<2, true>), dim3((uint32_t)grid), dim3(256), lds, s, t, la, T, ntiles);
    else
      hipLaunchKernelGGL((k_leaf_tiles<2, false>), dim3((uint32_t)grid), dim3(256), lds, s, t, la, T, ntiles);
  } else if (T == 256) {
    if (deref_each)
      hipLaunchKernelGGL((k_leaf_tiles<1, true>), dim3((uint32_t)grid), dim3(256), lds, s, t, la, T, ntiles);
    else
      hipLaunchKernelGGL((k_leaf_tiles<1, false>), dim3((uint32_t)grid), dim3(256), lds, s, t, la, T, ntiles);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch(const Tables& t, const LeafArgs& la, uint32_t flags, uint32_t block, uint32_t grid,
                        uint32_t T, uint64_t ntiles, hipStream_t s) {
  // chunks per thread per tile: T / block, one of 1, 2, 4, 8
  const uint32_t U = T / block;
  size_t lds = tile_lds_bytes(T);
  if (lds < kRelocLds) lds = kRelocLds;
  // compute tiles are taken in batches so that the queue sees about 16
  // items per workgroup
  uint64_t per = ntiles / ((uint64_t)grid * 16 + 1) + 1;
  const uint32_t per_item = (uint32_t)(per > 64 ? 64 : per);
#define DC_BATCH_CASE(UU)                                                                                  \
  case UU:                                                                                                 \
    hipLaunchKernelGGL(k_batch<UU>, dim3(grid), dim3(block), lds, s, t, la, flags, T, ntiles, per_item); \
    break;
  switch (U) {
    DC_BATCH_CASE(1)
    DC_BATCH_CASE(2)
    DC_BATCH_CASE(4)
    DC_BATCH_CASE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef DC_BATCH_CASE
  return hipGetLastError();
}

hipError_t launch_reset_counters(DevHeader* hdr, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, hdr);
  return hipGetLastError();
}

}  // namespace dc
