// libdc planner: the host walk that sizes and lays out the tree (the sizing
// step of Algorithm 1, with space handed out in the order the walk requests
// it), the relocation work units, the leaf tables and the scratch layout the
// kernels read.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <numeric>

#include "dc_host.h"

namespace dc {

// ---- FlatMap -------------------------------------------------------------------------

static inline uint64_t mix(uint64_t k) { return (k >> 3) * 0x9E3779B97F4A7C15ull; }

void FlatMap::reserve(uint64_t n) {
  uint64_t cap = 64;
  while (cap < 2 * n) cap <<= 1;
  keys_.assign(cap, 0);
  vals_.assign(cap, 0);
  mask_ = cap - 1;
  n_ = 0;
}

uint32_t FlatMap::find(uint64_t key) const {
  if (keys_.empty()) return kNone;
  uint64_t i = (mix(key) >> 20) & mask_;
  for (;;) {
    const uint64_t k = keys_[i];
    if (k == key) return vals_[i];
    if (k == 0) return kNone;
    i = (i + 1) & mask_;
  }
}

void FlatMap::grow() {
  std::vector<uint64_t> ok = std::move(keys_);
  std::vector<uint32_t> ov = std::move(vals_);
  const uint64_t cap = ok.empty() ? 64 : ok.size() * 2;
  keys_.assign(cap, 0);
  vals_.assign(cap, 0);
  mask_ = cap - 1;
  for (size_t j = 0; j < ok.size(); j++) {
    if (!ok[j]) continue;
    uint64_t i = (mix(ok[j]) >> 20) & mask_;
    while (keys_[i]) i = (i + 1) & mask_;
    keys_[i] = ok[j];
    vals_[i] = ov[j];
  }
}

void FlatMap::insert(uint64_t key, uint32_t val) {
  if (keys_.empty() || 2 * (n_ + 1) > keys_.size()) grow();
  uint64_t i = (mix(key) >> 20) & mask_;
  while (keys_[i]) i = (i + 1) & mask_;
  keys_[i] = key;
  vals_[i] = val;
  n_++;
}

// ---- walk --------------------------------------------------------------------------

static uint64_t elem_size(const std::vector<TypeDesc>& types, uint32_t kind, uint32_t type) {
  switch (kind) {
    case DC_KIND_STRUCT: return types[type].size;
    case DC_KIND_F32: return 4;
    case DC_KIND_F64: return 8;
    case DC_KIND_I32: return 4;
    case DC_KIND_I64: return 8;
    case DC_KIND_U8: return 1;
  }
  return 0;
}

// element count of the array a pointer member refers to
static dc_status field_count(const dc_field& f, const uint8_t* elem, uint64_t* count) {
  if (f.count_offset < 0) {
    *count = f.fixed_count;
    return DC_OK;
  }
  int64_t n;
  if (f.count_bytes == 4) {
    int32_t v;
    memcpy(&v, elem + f.count_offset, 4);
    n = v;
  } else {
    memcpy(&n, elem + f.count_offset, 8);
  }
  if (n < 0) return fail(DC_E_INVAL, "negative element count %lld", (long long)n);
  *count = (uint64_t)n * f.count_mult;
  return DC_OK;
}

namespace {

// What a walk produces: objects in placement order with their struct arrays,
// slot prefix and slot targets (indices local to the walk).
struct WalkOut {
  bigvec<Obj> objs;
  std::vector<DevSObj> sobj;
  std::vector<uint64_t> sobj_pre;
  bigvec<uint32_t> slot_target;  // per slot: target object or kNone
  std::vector<uint32_t> root_obj;
  uint64_t nslots = 0, nonnull = 0;
  FlatMap map;
};

struct Walker {
  const std::vector<TypeDesc>& types;
  uint32_t root_type;
  WalkOut& w;

  dc_status emit(uint64_t host, uint32_t kind, uint32_t type, uint64_t count, uint32_t parent, uint64_t rel,
                 uint64_t slot, uint32_t* out) {
    if (w.objs.size() >= kNone - 1) return fail(DC_E_RANGE, "more than 2^32-2 objects");
    Obj o{};
    o.host = host;
    o.kind = kind;
    o.type = type;
    o.count = count;
    o.bytes = count * elem_size(types, kind, type);
    o.parent = parent;
    o.parent_rel = rel;
    o.slot = slot;
    o.depth = parent == kNone ? 0 : w.objs[parent].depth + 1;
    o.sobj = kNone;
    const uint32_t idx = (uint32_t)w.objs.size();
    if (kind == DC_KIND_STRUCT && count > 0 && !types[type].order.empty()) {
      o.sobj = (uint32_t)w.sobj.size();
      DevSObj so{};
      so.count = count;
      so.type = type;
      so.obj = idx;
      w.sobj.push_back(so);
      w.sobj_pre.push_back(w.nslots);
      w.nslots += count * types[type].order.size();
      w.slot_target.resize(w.nslots, kNone);
    }
    w.objs.push_back(o);
    w.map.insert(host, idx);
    *out = idx;
    return DC_OK;
  }

  struct Frame {
    uint32_t obj;
    uint32_t k;
    uint64_t e;
  };

  // Depth-first pre-order from one root: an array is placed when first
  // reached; then, element by element and member by member in ascending
  // offset order, each non-null pointer not seen before is followed at once.
  dc_status walk_root(uint64_t root) {
    uint32_t idx = w.map.find(root);
    if (idx != kNone) {
      const Obj& o = w.objs[idx];
      if (o.kind != DC_KIND_STRUCT || o.type != root_type || o.count != 1)
        return fail(DC_E_CONFLICT, "root %#llx was reached before as a different array", (unsigned long long)root);
      w.root_obj.push_back(idx);
      return DC_OK;
    }
    DC_TRY(emit(root, DC_KIND_STRUCT, root_type, 1, kNone, 0, ~0ull, &idx));
    w.root_obj.push_back(idx);
    std::vector<Frame> stack;
    if (w.objs[idx].sobj != kNone) stack.push_back({idx, 0, 0});
    while (!stack.empty()) {
      Frame& fr = stack.back();
      const Obj& o = w.objs[fr.obj];
      const TypeDesc& t = types[o.type];
      if (fr.e == o.count) {
        stack.pop_back();
        continue;
      }
      const uint32_t nptr = (uint32_t)t.order.size();
      const uint32_t fi = t.order[fr.k];
      const dc_field& fd = t.fields[fi];
      const uint8_t* elem = (const uint8_t*)(uintptr_t)o.host + fr.e * t.size;
      const uint64_t slot = w.sobj_pre[o.sobj] + fr.e * nptr + fr.k;
      const uint64_t rel = fr.e * t.size + fd.offset;
      const uint32_t from = fr.obj;
      if (++fr.k == nptr) {
        fr.k = 0;
        fr.e++;
      }
      if (!((t.follow >> fi) & 1u)) continue;  // not part of a selective copy
      uint64_t ptr;
      memcpy(&ptr, elem + fd.offset, 8);
      if (ptr == 0) continue;
      uint64_t count;
      DC_TRY(field_count(fd, elem, &count));
      const uint32_t ptype = fd.kind == DC_KIND_STRUCT ? fd.type_id : 0;
      const uint32_t seen = w.map.find(ptr);
      if (seen != kNone) {
        const Obj& s = w.objs[seen];
        if (s.kind != fd.kind || s.type != ptype || s.count != count)
          return fail(DC_E_CONFLICT, "address %#llx reached as %llu elements of kind %u/type %u and as %llu of %u/%u",
                      (unsigned long long)ptr, (unsigned long long)s.count, s.kind, s.type,
                      (unsigned long long)count, fd.kind, ptype);
        w.slot_target[slot] = seen;
        w.nonnull++;
        continue;
      }
      uint32_t child;
      DC_TRY(emit(ptr, fd.kind, ptype, count, from, rel, slot, &child));
      w.slot_target[slot] = child;
      w.nonnull++;
      if (w.objs[child].sobj != kNone) stack.push_back({child, 0, 0});
    }
    return DC_OK;
  }
};

// The planner's worker threads: one pool per process, used by one plan at a
// time (a plan made while another is being made walks on its caller's thread).
std::mutex g_plan_pool_mu;
Pool* plan_pool() {
  static Pool* pool = new Pool(host_threads());  // lives until the process ends
  return pool;
}

// A plan over at least this many roots is walked in parallel, in chunks of
// consecutive roots (independent structures, as in a batch).
constexpr uint64_t kParallelMinRoots = 64;
constexpr uint64_t kMaxChunks = 256;

// Sorted-order check of the walked arrays' host ranges: no two may overlap
// (a pointer into the middle of another array, or, for a chunked walk, an
// array reached from two chunks). Returns false on the first overlap; `msg`
// gets the sequential planner's wording.
bool ranges_disjoint_sorted(std::vector<std::pair<uint64_t, uint64_t>>& r, uint64_t lo, uint64_t hi, char* msg,
                            size_t cap) {
  std::sort(r.begin() + lo, r.begin() + hi);
  for (uint64_t i = lo; i + 1 < hi; i++)
    if (r[i].first + r[i].second > r[i + 1].first) {
      if (msg) snprintf(msg, cap, "address %#llx lies inside the array at %#llx", (unsigned long long)r[i + 1].first,
                        (unsigned long long)r[i].first);
      return false;
    }
  return true;
}

}  // namespace

// Bucketed by address range across the pool, each bucket sorted on its own:
// the same answer as one sort of every (host, extent) pair.
static bool objects_disjoint_parallel(const bigvec<Obj>& objs, Pool* pool, int nparts) {
  const uint64_t n = objs.size();
  if (n < 2) return true;
  // splitters at quantiles of a sample of the addresses, so that every
  // bucket gets a similar share however the addresses cluster
  const uint64_t nb = 4096;
  std::vector<uint64_t> split;
  {
    const uint64_t ns = std::min<uint64_t>(n, 64 * nb);
    std::vector<uint64_t> sample(ns);
    for (uint64_t i = 0; i < ns; i++) sample[i] = objs[i * n / ns].host;
    std::sort(sample.begin(), sample.end());
    for (uint64_t b = 1; b < nb; b++) split.push_back(sample[b * ns / nb]);
  }
  auto bucket = [&](uint64_t h) { return (uint64_t)(std::upper_bound(split.begin(), split.end(), h) - split.begin()); };
  std::vector<uint64_t> cnt((size_t)nparts * nb, 0);
  pool->run(nparts, [&](int k) {
    uint64_t* c = &cnt[(size_t)k * nb];
    for (uint64_t i = n * k / nparts; i < n * (k + 1) / nparts; i++) c[bucket(objs[i].host)]++;
  });
  // bucket-major, part-minor prefix: every part writes its own run of each bucket
  std::vector<uint64_t> bstart(nb + 1, 0);
  uint64_t at = 0;
  for (uint64_t b = 0; b < nb; b++) {
    bstart[b] = at;
    for (int k = 0; k < nparts; k++) {
      const uint64_t c = cnt[(size_t)k * nb + b];
      cnt[(size_t)k * nb + b] = at;
      at += c;
    }
  }
  bstart[nb] = at;
  std::vector<std::pair<uint64_t, uint64_t>> r(n);
  pool->run(nparts, [&](int k) {
    uint64_t* c = &cnt[(size_t)k * nb];
    for (uint64_t i = n * k / nparts; i < n * (k + 1) / nparts; i++)
      r[c[bucket(objs[i].host)]++] = {objs[i].host, std::max<uint64_t>(objs[i].bytes, 1)};
  });
  std::atomic<bool> ok{true};
  pool->run((int)std::min<uint64_t>(nb, 512), [&](int k) {
    for (uint64_t b = nb * k / 512; b < nb * (k + 1) / 512 && ok.load(std::memory_order_relaxed); b++)
      if (!ranges_disjoint_sorted(r, bstart[b], bstart[b + 1], nullptr, 0)) ok = false;
  });
  if (!ok) return false;
  // across bucket boundaries: the last range of a bucket and the first of the next non-empty one
  uint64_t prev = ~0ull;
  for (uint64_t b = 0; b < nb; b++) {
    if (bstart[b] == bstart[b + 1]) continue;
    if (prev != ~0ull && r[prev].first + r[prev].second > r[bstart[b]].first) return false;
    prev = bstart[b + 1] - 1;
  }
  return true;
}

// The walk of nch chunks of consecutive roots, each chunk walked on its own
// (its own visited map) on the pool, then laid end to end. Equal to the walk
// in root order exactly when no array is reached from two chunks and no two
// arrays overlap: checked, and cobj is left empty (the caller then walks in
// root order) otherwise, or when any chunk fails. On success cobj holds the
// chunks' object index bounds and the plan its objects, struct arrays, slot
// prefix (with the total at the end), slot targets and root objects.
static void walk_chunks(dc_plan p, const void* const* roots, uint64_t nroots, uint64_t nch, Pool* pool,
                        std::vector<uint64_t>& cobj) {
  std::vector<WalkOut> outs(nch);
  std::atomic<bool> ok{true};
  pool->run((int)nch, [&](int c) {
    WalkOut& w = outs[c];
    w.map.reserve(1024);
    Walker wk{p->types, p->root_type, w};
    for (uint64_t r = nroots * c / nch; r < nroots * (c + 1) / nch && ok.load(std::memory_order_relaxed); r++)
      if (wk.walk_root((uint64_t)(uintptr_t)roots[r]) != DC_OK) ok = false;
    w.map = FlatMap();
  });
  if (!ok) return;
  std::vector<uint64_t> ob(nch + 1, 0), sb(nch + 1, 0), lb(nch + 1, 0), rb(nch + 1, 0);
  uint64_t nonnull = 0;
  for (uint64_t c = 0; c < nch; c++) {
    ob[c + 1] = ob[c] + outs[c].objs.size();
    sb[c + 1] = sb[c] + outs[c].sobj.size();
    lb[c + 1] = lb[c] + outs[c].nslots;
    rb[c + 1] = rb[c] + outs[c].root_obj.size();
    nonnull += outs[c].nonnull;
  }
  if (ob[nch] >= kNone - 1) return;
  p->objs.resize(ob[nch]);
  p->sobj.resize(sb[nch]);
  p->sobj_pre.resize(sb[nch] + 1);
  p->slot_target.resize(lb[nch]);
  p->root_obj.resize(rb[nch]);
  pool->run((int)nch, [&](int c) {
    WalkOut& w = outs[c];
    const uint32_t o0 = (uint32_t)ob[c], s0 = (uint32_t)sb[c];
    for (size_t i = 0; i < w.objs.size(); i++) {
      Obj o = w.objs[i];
      if (o.parent != kNone) o.parent += o0;
      if (o.sobj != kNone) o.sobj += s0;
      if (o.slot != ~0ull) o.slot += lb[c];
      p->objs[o0 + i] = o;
    }
    for (size_t i = 0; i < w.sobj.size(); i++) {
      DevSObj so = w.sobj[i];
      so.obj += o0;
      p->sobj[s0 + i] = so;
      p->sobj_pre[s0 + i] = w.sobj_pre[i] + lb[c];
    }
    for (size_t i = 0; i < w.slot_target.size(); i++)
      p->slot_target[lb[c] + i] = w.slot_target[i] == kNone ? kNone : w.slot_target[i] + o0;
    for (size_t i = 0; i < w.root_obj.size(); i++) p->root_obj[rb[c] + i] = w.root_obj[i] + o0;
    bigvec<Obj>().swap(w.objs);
    bigvec<uint32_t>().swap(w.slot_target);
  });
  p->sobj_pre[sb[nch]] = lb[nch];
  if (!objects_disjoint_parallel(p->objs, pool, (int)std::min<uint64_t>(nch, 64))) {
    // an array reached from two chunks (or a pointer into an array): the walk in root order decides
    p->objs.clear();
    p->sobj.clear();
    p->sobj_pre.clear();
    p->slot_target.clear();
    p->root_obj.clear();
    return;
  }
  p->nslots_nonnull = nonnull;
  cobj = ob;
}

std::vector<DevTile> build_tiles(const dc_plan_s* p, uint32_t T) {
  std::vector<DevTile> tiles;
  const uint64_t nl = p->leaves.size();
  const uint64_t total = p->total_chunks;
  uint64_t l = 0;
  for (uint64_t c = 0; c < total;) {
    while (p->leaf_pre[l + 1] <= c) l++;  // the leaf holding chunk c
    uint64_t hi = std::min<uint64_t>(c + T, total);
    hi = std::min<uint64_t>(hi, p->leaf_pre[std::min<uint64_t>(l + kTileMaxLeaves, nl)]);
    uint64_t lh = l;
    while (p->leaf_pre[lh + 1] < hi) lh++;  // the leaf holding chunk hi - 1
    DevTile tl{};
    tl.c_lo = c;
    tl.c_hi = hi;
    tl.l_lo = (uint32_t)l;
    tl.l_hi = (uint32_t)lh;
    tiles.push_back(tl);
    c = hi;
  }
  return tiles;
}

dc_status plan_build(dc_plan p, const dc_schema_s* schema, uint32_t root_type, const void* const* roots,
                     uint64_t nroots, uint64_t align, const uint32_t* follow, uint32_t nfollow) {
  p->types = schema->types;
  if (nfollow > p->types.size()) return fail(DC_E_INVAL, "%u follow masks for %zu types", nfollow, p->types.size());
  for (uint32_t i = 0; i < nfollow; i++) {
    const size_t nf = p->types[i].fields.size();
    if (nf < 32 && (follow[i] >> nf) != 0)
      return fail(DC_E_INVAL, "follow mask 0x%x of type %u sets bits past its %zu fields", follow[i], i, nf);
    p->types[i].follow = follow[i];
  }
  if (root_type >= p->types.size()) return fail(DC_E_INVAL, "root type %u not described", root_type);
  for (size_t i = 0; i < p->types.size(); i++)
    for (const dc_field& f : p->types[i].fields)
      if (f.kind == DC_KIND_STRUCT && f.type_id >= p->types.size())
        return fail(DC_E_INVAL, "type %zu (%s) points to undescribed type %u", i, p->types[i].name.c_str(), f.type_id);
  p->root_type = root_type;
  p->align = align;

  // the walk: chunks of consecutive roots in parallel when there are many
  // roots and the planner's threads are free; otherwise (or when a chunked
  // walk finds anything but disjoint, valid structures) one walk in root
  // order, whose result and errors are the definition
  std::vector<uint64_t> cobj;  // object index bounds of the chunks
  bool nulls = false;
  for (uint64_t r = 0; r < nroots; r++) nulls = nulls || !roots[r];
  {
    std::unique_lock<std::mutex> lk(g_plan_pool_mu, std::defer_lock);
    if (nroots >= kParallelMinRoots && !nulls && lk.try_lock() && plan_pool()->size() > 1)
      walk_chunks(p, roots, nroots, std::min<uint64_t>(nroots, kMaxChunks), plan_pool(), cobj);
  }
  if (cobj.empty()) {
    WalkOut w;
    w.map.reserve(1024);
    Walker wk{p->types, root_type, w};
    for (uint64_t r = 0; r < nroots; r++) {
      const uint64_t addr = (uint64_t)(uintptr_t)roots[r];
      if (!addr) return fail(DC_E_INVAL, "root %llu is null", (unsigned long long)r);
      DC_TRY(wk.walk_root(addr));
    }
    p->objs = std::move(w.objs);
    p->sobj = std::move(w.sobj);
    p->sobj_pre = std::move(w.sobj_pre);
    p->slot_target = std::move(w.slot_target);
    p->root_obj = std::move(w.root_obj);
    p->nslots_nonnull = w.nonnull;
    p->sobj_pre.push_back(w.nslots);
    // a pointer into the middle of another array shows as overlapping ranges
    const uint64_t nobj = p->objs.size();
    std::vector<uint32_t> by_host(nobj);
    std::iota(by_host.begin(), by_host.end(), 0u);
    std::sort(by_host.begin(), by_host.end(), [&](uint32_t a, uint32_t b) { return p->objs[a].host < p->objs[b].host; });
    for (uint64_t i = 0; i + 1 < nobj; i++) {
      const Obj& a = p->objs[by_host[i]];
      const Obj& b = p->objs[by_host[i + 1]];
      if (a.host + std::max<uint64_t>(a.bytes, 1) > b.host)
        return fail(DC_E_RANGE, "address %#llx lies inside the array at %#llx (%llu bytes)", (unsigned long long)b.host,
                    (unsigned long long)a.host, (unsigned long long)a.bytes);
    }
    cobj = {0, nobj};
  }
  for (uint64_t r = 0; r < nroots; r++) p->roots.push_back((uint64_t)(uintptr_t)roots[r]);
  const uint64_t nobj = p->objs.size();
  const uint64_t nch = cobj.size() - 1;
  // chunk bounds in the struct-array and slot enumerations
  std::vector<uint64_t> csobj(nch + 1), cslot(nch + 1);
  for (uint64_t c = 0; c <= nch; c++) {
    uint64_t so = c == nch ? p->sobj.size() : 0;
    if (c < nch) {
      // the first struct array placed at or after the chunk's first object
      uint64_t lo = 0, hi = p->sobj.size();
      while (lo < hi) {
        const uint64_t mid = (lo + hi) / 2;
        if (p->sobj[mid].obj < cobj[c]) lo = mid + 1;
        else hi = mid;
      }
      so = lo;
    }
    csobj[c] = so;
    cslot[c] = p->sobj_pre[so];
  }
  std::unique_lock<std::mutex> lk(g_plan_pool_mu, std::defer_lock);
  Pool* pool = nch > 1 && lk.try_lock() ? plan_pool() : nullptr;
  auto each_chunk = [&](const std::function<void(int)>& fn) {
    if (pool) pool->run((int)nch, fn);
    else
      for (uint64_t c = 0; c < nch; c++) fn((int)c);
  };

  // layout in walk order: each chunk from 0, then shifted by the aligned sizes
  // of the chunks before it (an aligned shift does not change the rounding)
  {
    std::vector<uint64_t> csize(nch + 1, 0), cpay(nch, 0);
    each_chunk([&](int c) {
      uint64_t end = 0, pay = 0;
      for (uint64_t i = cobj[c]; i < cobj[c + 1]; i++) {
        Obj& o = p->objs[i];
        o.off = i == cobj[c] ? 0 : align_up(end, align);
        end = o.off + std::max<uint64_t>(o.bytes, 1);
        pay += o.bytes;
      }
      csize[c] = cobj[c + 1] > cobj[c] ? align_up(end, align) : 0;
      cpay[c] = pay;
    });
    uint64_t at = 0;
    for (uint64_t c = 0; c < nch; c++) {
      const uint64_t sz = csize[c];
      csize[c] = at;
      at += sz;
      p->payload_bytes += cpay[c];
    }
    p->arena_bytes = nobj ? at : 0;
    // the relocation kernel packs an arena offset and a type into 64 bits
    if (p->arena_bytes >= (1ull << 48))
      return fail(DC_E_RANGE, "arena of %llu bytes (limit 2^48)", (unsigned long long)p->arena_bytes);
    each_chunk([&](int c) {
      if (csize[c])
        for (uint64_t i = cobj[c]; i < cobj[c + 1]; i++) p->objs[i].off += csize[c];
      for (uint64_t so = csobj[c]; so < csobj[c + 1]; so++) p->sobj[so].off = p->objs[p->sobj[so].obj].off;
    });
  }

  std::vector<uint64_t> sbase, lbase;  // the chunks' units and leaves
  // relocation units over the slot enumeration, cut greedily within each
  // chunk. A small tree is cut into smaller units so that its relocation
  // spreads over more workgroups (it is latency-bound); a large one uses
  // full units.
  {
    const uint64_t nslots = p->sobj_pre.back();
    uint64_t unit_slots = 128;
    while (unit_slots < kSegMaxSlots && nslots / unit_slots > 256) unit_slots *= 2;
    bigvec<uint32_t> mark(nobj);
    bigvec<uint16_t> tix(nobj);  // index of an object in the current unit's targets
    p->slot_tix.resize(nslots);
    std::vector<std::vector<DevSeg>> csegs(nch);
    std::vector<std::vector<DevTarget>> ctgts(nch);
    each_chunk([&](int c) {
      for (uint64_t i = cobj[c]; i < cobj[c + 1]; i++) mark[i] = kNone;
      std::vector<DevSeg>& segs = csegs[c];
      std::vector<DevTarget>& tgts = ctgts[c];
      uint32_t seg_id = 0, ntgt = 0;
      DevSeg cur{};
      auto open = [&](uint64_t slot, uint64_t so) {
        cur = DevSeg{};
        cur.slot_lo = slot;
        cur.tgt_lo = tgts.size();
        cur.sobj_lo = (uint32_t)so;
        ntgt = 0;
      };
      auto close = [&](uint64_t hi, uint64_t so_hi) {
        cur.slot_hi = hi;
        cur.tgt_hi = tgts.size();
        cur.sobj_hi = (uint32_t)so_hi;
        if (cur.slot_hi > cur.slot_lo) {
          segs.push_back(cur);
          seg_id++;
        }
      };
      open(cslot[c], csobj[c]);
      for (uint64_t so = csobj[c]; so < csobj[c + 1]; so++) {
        if (so - cur.sobj_lo >= kSegMaxSObjs) {
          close(p->sobj_pre[so], so);
          open(p->sobj_pre[so], so);
        }
        for (uint64_t j = p->sobj_pre[so]; j < p->sobj_pre[so + 1]; j++) {
          // a unit's distinct targets never outnumber its slots: the slot
          // count alone bounds the target list and its 16-bit indices
          if (j - cur.slot_lo >= unit_slots) {
            close(j, so + 1);
            open(j, so);
          }
          const uint32_t t = p->slot_target[j];
          if (t == kNone) {
            p->slot_tix[j] = kNoTarget;
            continue;
          }
          if (mark[t] != seg_id) {
            mark[t] = seg_id;
            tix[t] = (uint16_t)ntgt;
            tgts.push_back(DevTarget{p->objs[t].host, p->objs[t].off});
            ntgt++;
          }
          p->slot_tix[j] = tix[t];
        }
      }
      close(cslot[c + 1], csobj[c + 1]);
    });
    uint64_t nseg = 0, ntg = 0;
    std::vector<uint64_t> tbase(nch);
    sbase.assign(nch + 1, 0);
    for (uint64_t c = 0; c < nch; c++) {
      sbase[c] = nseg;
      tbase[c] = ntg;
      nseg += csegs[c].size();
      ntg += ctgts[c].size();
    }
    sbase[nch] = nseg;
    p->segs.resize(nseg);
    p->tgts.resize(ntg);
    each_chunk([&](int c) {
      for (size_t k = 0; k < csegs[c].size(); k++) {
        DevSeg g = csegs[c][k];
        g.tgt_lo += tbase[c];
        g.tgt_hi += tbase[c];
        p->segs[sbase[c] + k] = g;
      }
      std::copy(ctgts[c].begin(), ctgts[c].end(), p->tgts.begin() + tbase[c]);
      std::vector<DevSeg>().swap(csegs[c]);
      std::vector<DevTarget>().swap(ctgts[c]);
    });
  }

  // leaves and the out-of-place leaf image, per chunk: counts, then the
  // tables at each chunk's place (the out image shifted like the layout)
  {
    std::vector<uint64_t> cnl(nch + 1, 0), cchunks(nch + 1, 0), cout(nch + 1, 0), chops(nch, 0), clb(nch, 0);
    each_chunk([&](int c) {
      uint64_t nl = 0, chunks = 0, oend = 0, hops = 0, lb = 0;
      bool first = true;
      for (uint64_t i = cobj[c]; i < cobj[c + 1]; i++) {
        const Obj& o = p->objs[i];
        if (o.kind != DC_KIND_F32 && o.kind != DC_KIND_F64) continue;
        const uint64_t ooff = first ? 0 : align_up(oend, align);
        first = false;
        oend = ooff + std::max<uint64_t>(o.bytes, 1);
        lb += o.bytes;
        if (o.count == 0) continue;
        nl++;
        chunks += (o.bytes + kChunk - 1) / kChunk;
        hops += o.depth;
      }
      cnl[c] = nl;
      cchunks[c] = chunks;
      cout[c] = first ? 0 : align_up(oend, align);
      chops[c] = hops;
      clb[c] = lb;
    });
    uint64_t nl = 0, chunks = 0, out = 0;
    for (uint64_t c = 0; c < nch; c++) {
      const uint64_t a = cnl[c], b = cchunks[c], o = cout[c];
      cnl[c] = nl;
      cchunks[c] = chunks;
      cout[c] = out;
      nl += a;
      chunks += b;
      out += o;
      p->total_hops += chops[c];
      p->leaf_bytes += clb[c];
    }
    p->leaves.resize(nl);
    p->leaf_pre.resize(nl + 1);
    p->leaf_info.resize(nl);
    p->leaf_slot.resize(nl);
    p->leaf_out.resize(nl);
    p->leaf_dev.resize(nl);
    each_chunk([&](int c) {
      uint64_t l = cnl[c], ch = cchunks[c], oend = 0;
      bool first = true;
      for (uint64_t i = cobj[c]; i < cobj[c + 1]; i++) {
        const Obj& o = p->objs[i];
        if (o.kind != DC_KIND_F32 && o.kind != DC_KIND_F64) continue;
        const uint64_t ooff = first ? 0 : align_up(oend, align);
        first = false;
        oend = ooff + std::max<uint64_t>(o.bytes, 1);
        if (o.count == 0) continue;
        p->leaves[l] = (uint32_t)i;
        p->leaf_pre[l] = ch;
        p->leaf_info[l] = o.bytes | ((uint64_t)o.kind << kLeafKindShift);
        p->leaf_slot[l] = p->objs[o.parent].off + o.parent_rel;
        p->leaf_out[l] = cout[c] + ooff;
        p->leaf_dev[l] = o.off;
        ch += (o.bytes + kChunk - 1) / kChunk;
        l++;
      }
    });
    p->leaf_pre[nl] = chunks;
    p->total_chunks = chunks;
    p->out_bytes = out;
    cnl[nch] = nl;
    lbase = cnl;
  }
  // the leaves each relocation unit's slots discover: a leaf belongs to the
  // unit holding the slot that first reached it. When the owning units never
  // decrease along the leaf order (a depth-first layout whose struct arrays
  // list their leaf members before deeper struct members, as every workload
  // here does), every unit owns one contiguous run of leaves. A leaf's slot
  // lies in its own chunk, so each chunk is checked on its own
  {
    const uint64_t nl = p->leaves.size(), ns = p->segs.size();
    std::vector<uint64_t> cmax(nch, 0);
    std::atomic<bool> mono{ns > 0 && ns < kNone && nl > 0 && nl < kNone};
    each_chunk([&](int c) {
      const uint64_t s0 = sbase[c], s1 = sbase[c + 1];
      for (uint64_t s = s0; s < s1; s++) p->segs[s].leaf_lo = p->segs[s].leaf_hi = 0;
      uint64_t u = s0;
      for (uint64_t l = lbase[c]; l < lbase[c + 1] && mono.load(std::memory_order_relaxed); l++) {
        const uint64_t slot = p->objs[p->leaves[l]].slot;
        while (u + 1 < s1 && p->segs[u].slot_hi <= slot) u++;
        if (u >= s1 || slot < p->segs[u].slot_lo || slot >= p->segs[u].slot_hi) mono = false;  // an earlier unit
        else if (p->segs[u].leaf_hi == 0) p->segs[u].leaf_lo = (uint32_t)l, p->segs[u].leaf_hi = (uint32_t)l + 1;
        else p->segs[u].leaf_hi = (uint32_t)l + 1;
      }
      // units without leaves get the empty run where the next leaves start
      uint32_t at = (uint32_t)lbase[c + 1];
      for (uint64_t s = s1; s-- > s0;) {
        if (p->segs[s].leaf_hi == 0) p->segs[s].leaf_lo = p->segs[s].leaf_hi = at;
        else at = p->segs[s].leaf_lo;
        cmax[c] = std::max<uint64_t>(cmax[c], p->leaf_pre[p->segs[s].leaf_hi] - p->leaf_pre[p->segs[s].leaf_lo]);
      }
    });
    p->unit_leaves = mono.load();
    if (p->unit_leaves)
      for (uint64_t c = 0; c < nch; c++) p->max_unit_leaf_chunks = std::max(p->max_unit_leaf_chunks, cmax[c]);
  }
  // the fused relocate-and-compute launch: each leaf's parent slot's target
  // entry, and every other slot with its arena offset (slots, units and
  // leaves of a chunk stay within the chunk)
  {
    p->leaf_tgt.resize(p->leaves.size());
    std::vector<std::vector<DevResid>> cres(nch);
    each_chunk([&](int c) {
      const uint64_t s0 = sbase[c], s1 = sbase[c + 1];
      auto unit_of = [&](uint64_t slot) {  // last unit of the chunk starting at or before slot
        uint64_t lo = s0, hi = s1;
        while (hi - lo > 1) {
          const uint64_t mid = (lo + hi) / 2;
          if (p->segs[mid].slot_lo <= slot) lo = mid;
          else hi = mid;
        }
        return lo;
      };
      for (uint64_t l = lbase[c]; l < lbase[c + 1]; l++) {
        const uint64_t slot = p->objs[p->leaves[l]].slot;
        p->leaf_tgt[l] = (uint32_t)(p->segs[unit_of(slot)].tgt_lo + p->slot_tix[slot]);
      }
      uint64_t u = s0;
      for (uint64_t so = csobj[c]; so < csobj[c + 1]; so++) {
        const DevSObj& sob = p->sobj[so];
        const TypeDesc& ty = p->types[sob.type];
        const uint64_t nptr = ty.order.size();
        for (uint64_t j = p->sobj_pre[so]; j < p->sobj_pre[so + 1]; j++) {
          while (u + 1 < s1 && p->segs[u + 1].slot_lo <= j) u++;
          const uint32_t t = p->slot_target[j];
          if (t != kNone) {
            const Obj& o = p->objs[t];
            if ((o.kind == DC_KIND_F32 || o.kind == DC_KIND_F64) && o.count && o.slot == j) continue;  // a leaf's
          }
          const uint64_t local = j - p->sobj_pre[so], e = local / nptr, f = local % nptr;
          DevResid r;
          r.slot_off = sob.off + e * ty.size + ty.fields[ty.order[f]].offset;
          r.tgt = t == kNone ? kNone : (uint32_t)(p->segs[u].tgt_lo + p->slot_tix[j]);
          r.follow = (ty.follow >> ty.order[f]) & 1u;
          cres[c].push_back(r);
        }
      }
    });
    for (uint64_t c = 0; c < nch; c++) p->resid.insert(p->resid.end(), cres[c].begin(), cres[c].end());
  }
  lk = std::unique_lock<std::mutex>();  // the pool is free for other plans

  // device types
  p->dev_types.resize(p->types.size());
  for (size_t i = 0; i < p->types.size(); i++) {
    const TypeDesc& t = p->types[i];
    DevType& d = p->dev_types[i];
    memset(&d, 0, sizeof(d));
    d.size = t.size;
    d.nptr = (uint32_t)t.order.size();
    for (uint32_t k = 0; k < d.nptr; k++) {
      if ((t.follow >> t.order[k]) & 1u) d.follow |= 1u << k;
      const dc_field& f = t.fields[t.order[k]];
      d.ptr_off[k] = f.offset;
      d.kind[k] = f.kind;
      d.ptype[k] = f.type_id;
      d.cnt_off[k] = f.count_offset;
      d.cnt_bytes[k] = f.count_bytes;
      d.cnt_mult[k] = f.count_mult;
      d.fixed[k] = f.fixed_count;
    }
  }

  // scratch layout
  {
    ScratchLayout& s = p->sl;
    uint64_t at = 0;
    auto take = [&](uint64_t bytes) {
      const uint64_t o = at;
      at = align_up(at + bytes, 256);
      return o;
    };
    const uint64_t nl = p->leaves.size();
    s.header = take(sizeof(DevHeader));
    s.types = take(sizeof(DevType) * p->dev_types.size());
    s.sobj = take(sizeof(DevSObj) * p->sobj.size());
    s.sobj_pre = take(8 * p->sobj_pre.size());
    s.segs = take(sizeof(DevSeg) * p->segs.size());
    s.tgts = take(sizeof(DevTarget) * p->tgts.size());
    s.slot_tix = take(2 * p->slot_tix.size());
    s.leaf_slot = take(8 * nl);
    s.leaf_info = take(8 * nl);
    s.leaf_out = take(8 * nl);
    s.leaf_tgt = take(4 * nl);
    s.leaf_dev = take(8 * nl);
    s.resid = take(sizeof(DevResid) * p->resid.size());
    s.static_end = at;
    // computed on the device from the leaf sizes after each upload
    s.leaf_pre = take(8 * (nl + 1));
    s.leaf_pre_scan = take(8 * ((nl + kScanLeaves - 1) / kScanLeaves + 1));
    const uint64_t max_tiles = (p->total_chunks + kTileMinChunks - 1) / kTileMinChunks +
                               p->leaves.size() / (kTileMaxLeaves - 1) + 2;
    s.tiles = take(sizeof(DevTile) * max_tiles);
    s.paths = take(sizeof(DevPath) * nl);
    s.hops = take(8 * (p->total_hops + 1));
    s.total = at;
  }
  return DC_OK;
}

}  // namespace dc

using namespace dc;

extern "C" {

dc_status dc_plan_create(dc_ctx ctx, dc_schema schema, uint32_t root_type, const void* const* roots, uint64_t nroots,
                         uint64_t align, dc_plan* out, uint64_t* arena_bytes, uint64_t* scratch_bytes) {
  return dc_plan_create_selective(ctx, schema, root_type, roots, nroots, align, nullptr, 0, out, arena_bytes,
                                  scratch_bytes);
}

dc_status dc_plan_create_selective(dc_ctx ctx, dc_schema schema, uint32_t root_type, const void* const* roots,
                                   uint64_t nroots, uint64_t align, const uint32_t* follow, uint32_t nfollow,
                                   dc_plan* out, uint64_t* arena_bytes, uint64_t* scratch_bytes) {
  (void)ctx;
  if (nfollow && !follow) return fail(DC_E_INVAL, "dc_plan_create_selective: null follow masks");
  if (!out) return fail(DC_E_INVAL, "dc_plan_create: out is null");
  *out = nullptr;
  if (!schema || (!roots && nroots)) return fail(DC_E_INVAL, "dc_plan_create: null schema or roots");
  if (align == 0) align = 64;
  if (align < 16 || align > 4096 || (align & (align - 1)))
    return fail(DC_E_INVAL, "dc_plan_create: align %llu (power of two in 16..4096)", (unsigned long long)align);
  dc_plan p = new dc_plan_s();
  dc_status st = plan_build(p, schema, root_type, roots, nroots, align, follow, nfollow);
  if (st != DC_OK) {
    delete p;
    return st;
  }
  *out = p;
  if (arena_bytes) *arena_bytes = p->arena_bytes;
  if (scratch_bytes) *scratch_bytes = p->sl.total;
  clear_error();
  return DC_OK;
}

dc_status dc_plan_destroy(dc_plan p) {
  if (!p) return fail(DC_E_INVAL, "dc_plan_destroy: null plan");
  delete p;
  return DC_OK;
}

dc_status dc_plan_query(dc_plan p, dc_plan_info* out) {
  if (!p || !out) return fail(DC_E_INVAL, "dc_plan_query: null argument");
  out->nobjects = p->objs.size();
  out->nslots = p->sobj_pre.empty() ? 0 : p->sobj_pre.back();
  out->nslots_nonnull = p->nslots_nonnull;
  out->nleaves = p->leaves.size();
  out->payload_bytes = p->payload_bytes;
  out->leaf_bytes = p->leaf_bytes;
  out->arena_bytes = p->arena_bytes;
  out->scratch_bytes = p->sl.total;
  out->out_bytes = p->out_bytes;
  out->nsegments = p->segs.size();
  out->nroots = p->roots.size();
  out->unit_leaves = p->unit_leaves ? 1 : 0;
  out->max_unit_leaf_bytes = p->max_unit_leaf_chunks * kChunk;
  out->leaf_prefix_offset = p->sl.leaf_pre;
  return DC_OK;
}

dc_status dc_plan_objects(dc_plan p, dc_object* out, uint64_t cap, uint64_t* n) {
  if (!p || (!out && cap)) return fail(DC_E_INVAL, "dc_plan_objects: null argument");
  const uint64_t m = std::min<uint64_t>(cap, p->objs.size());
  for (uint64_t i = 0; i < m; i++) {
    const Obj& o = p->objs[i];
    out[i].host_addr = o.host;
    out[i].offset = o.off;
    out[i].bytes = o.bytes;
    out[i].count = o.count;
    out[i].kind = o.kind;
    out[i].type_id = o.type;
  }
  if (n) *n = p->objs.size();
  return DC_OK;
}

}  // extern "C"
