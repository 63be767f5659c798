// libdc planner: the host walk that sizes and lays out the tree (the sizing
// step of Algorithm 1, with space handed out in the order the walk requests
// it), the relocation work units, the leaf tables and the scratch layout the
// kernels read.
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
struct Walker {
  dc_plan p;
  uint64_t nslots = 0;

  dc_status emit(uint64_t host, uint32_t kind, uint32_t type, uint64_t count, uint32_t parent, uint64_t rel,
                 uint64_t slot, uint32_t* out) {
    if (p->objs.size() >= kNone - 1) return fail(DC_E_RANGE, "more than 2^32-2 objects");
    Obj o{};
    o.host = host;
    o.kind = kind;
    o.type = type;
    o.count = count;
    o.bytes = count * elem_size(p->types, kind, type);
    o.parent = parent;
    o.parent_rel = rel;
    o.slot = slot;
    o.depth = parent == kNone ? 0 : p->objs[parent].depth + 1;
    o.sobj = kNone;
    const uint32_t idx = (uint32_t)p->objs.size();
    if (kind == DC_KIND_STRUCT && count > 0 && !p->types[type].order.empty()) {
      o.sobj = (uint32_t)p->sobj.size();
      DevSObj so{};
      so.count = count;
      so.type = type;
      so.obj = idx;
      p->sobj.push_back(so);
      p->sobj_pre.push_back(nslots);
      nslots += count * p->types[type].order.size();
      p->slot_target.resize(nslots, kNone);
    }
    p->objs.push_back(o);
    p->map.insert(host, idx);
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
    uint32_t idx = p->map.find(root);
    if (idx != kNone) {
      const Obj& o = p->objs[idx];
      if (o.kind != DC_KIND_STRUCT || o.type != p->root_type || o.count != 1)
        return fail(DC_E_CONFLICT, "root %#llx was reached before as a different array", (unsigned long long)root);
      p->root_obj.push_back(idx);
      return DC_OK;
    }
    DC_TRY(emit(root, DC_KIND_STRUCT, p->root_type, 1, kNone, 0, ~0ull, &idx));
    p->root_obj.push_back(idx);
    std::vector<Frame> stack;
    if (p->objs[idx].sobj != kNone) stack.push_back({idx, 0, 0});
    while (!stack.empty()) {
      Frame& fr = stack.back();
      const Obj& o = p->objs[fr.obj];
      const TypeDesc& t = p->types[o.type];
      if (fr.e == o.count) {
        stack.pop_back();
        continue;
      }
      const uint32_t nptr = (uint32_t)t.order.size();
      const uint32_t fi = t.order[fr.k];
      const dc_field& fd = t.fields[fi];
      const uint8_t* elem = (const uint8_t*)(uintptr_t)o.host + fr.e * t.size;
      const uint64_t slot = p->sobj_pre[o.sobj] + fr.e * nptr + fr.k;
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
      const uint32_t seen = p->map.find(ptr);
      if (seen != kNone) {
        const Obj& s = p->objs[seen];
        if (s.kind != fd.kind || s.type != ptype || s.count != count)
          return fail(DC_E_CONFLICT, "address %#llx reached as %llu elements of kind %u/type %u and as %llu of %u/%u",
                      (unsigned long long)ptr, (unsigned long long)s.count, s.kind, s.type,
                      (unsigned long long)count, fd.kind, ptype);
        p->slot_target[slot] = seen;
        p->nslots_nonnull++;
        continue;
      }
      uint32_t child;
      DC_TRY(emit(ptr, fd.kind, ptype, count, from, rel, slot, &child));
      p->slot_target[slot] = child;
      p->nslots_nonnull++;
      if (p->objs[child].sobj != kNone) stack.push_back({child, 0, 0});
    }
    return DC_OK;
  }
};
}  // namespace

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
  p->map.reserve(1024);
  Walker w{p};
  for (uint64_t r = 0; r < nroots; r++) {
    const uint64_t addr = (uint64_t)(uintptr_t)roots[r];
    if (!addr) return fail(DC_E_INVAL, "root %llu is null", (unsigned long long)r);
    p->roots.push_back(addr);
    DC_TRY(w.walk_root(addr));
  }
  p->sobj_pre.push_back(w.nslots);
  const uint64_t nobj = p->objs.size();

  // a pointer into the middle of another array shows as overlapping ranges
  {
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
  }

  // layout in walk order
  uint64_t end = 0;
  for (uint64_t i = 0; i < nobj; i++) {
    Obj& o = p->objs[i];
    o.off = i == 0 ? 0 : align_up(end, align);
    end = o.off + std::max<uint64_t>(o.bytes, 1);
    p->payload_bytes += o.bytes;
  }
  p->arena_bytes = nobj ? align_up(end, align) : 0;
  // the relocation kernel packs an arena offset and a type into 64 bits
  if (p->arena_bytes >= (1ull << 48))
    return fail(DC_E_RANGE, "arena of %llu bytes (limit 2^48)", (unsigned long long)p->arena_bytes);
  for (DevSObj& so : p->sobj) so.off = p->objs[so.obj].off;

  // relocation units over the slot enumeration. A small tree is cut into
  // smaller units so that its relocation spreads over more workgroups (it is
  // latency-bound); a large one uses full units.
  {
    const uint64_t nslots = w.nslots;
    uint64_t unit_slots = 128;
    while (unit_slots < kSegMaxSlots && nslots / unit_slots > 256) unit_slots *= 2;
    std::vector<uint32_t> mark(nobj, kNone);
    uint32_t seg_id = 0, ntgt = 0;
    DevSeg cur{};
    uint32_t so = 0;
    auto close = [&](uint64_t hi, uint32_t so_hi) {
      cur.slot_hi = hi;
      cur.tgt_hi = p->tgts.size();
      cur.sobj_hi = so_hi;
      if (cur.slot_hi > cur.slot_lo) {
        p->segs.push_back(cur);
        seg_id++;
      }
    };
    cur.slot_lo = 0;
    cur.tgt_lo = 0;
    cur.sobj_lo = 0;
    for (so = 0; so < p->sobj.size(); so++) {
      if (so - cur.sobj_lo >= kSegMaxSObjs) {
        close(p->sobj_pre[so], so);
        cur = DevSeg{};
        cur.slot_lo = p->sobj_pre[so];
        cur.tgt_lo = p->tgts.size();
        cur.sobj_lo = so;
        ntgt = 0;
      }
      for (uint64_t j = p->sobj_pre[so]; j < p->sobj_pre[so + 1]; j++) {
        const uint32_t t = p->slot_target[j];
        const bool new_tgt = t != kNone && mark[t] != seg_id;
        if (j - cur.slot_lo >= unit_slots || (new_tgt && ntgt == kSegMaxTargets)) {
          close(j, so + 1);
          cur = DevSeg{};
          cur.slot_lo = j;
          cur.tgt_lo = p->tgts.size();
          cur.sobj_lo = so;
          ntgt = 0;
        }
        if (t != kNone && mark[t] != seg_id) {
          mark[t] = seg_id;
          p->tgts.push_back(DevTarget{p->objs[t].host, p->objs[t].off});
          ntgt++;
        }
      }
    }
    close(nslots, (uint32_t)p->sobj.size());
  }

  // leaves and the out-of-place leaf image
  {
    uint64_t chunks = 0, oend = 0;
    bool first = true;
    for (uint64_t i = 0; i < nobj; i++) {
      const Obj& o = p->objs[i];
      if (o.kind != DC_KIND_F32 && o.kind != DC_KIND_F64) continue;
      const uint64_t ooff = first ? 0 : align_up(oend, align);
      first = false;
      oend = ooff + std::max<uint64_t>(o.bytes, 1);
      p->leaf_bytes += o.bytes;
      if (o.count == 0) continue;
      p->leaves.push_back((uint32_t)i);
      p->leaf_pre.push_back(chunks);
      p->leaf_info.push_back(o.bytes | ((uint64_t)o.kind << kLeafKindShift));
      p->leaf_slot.push_back(p->objs[o.parent].off + o.parent_rel);
      p->leaf_out.push_back(ooff);
      chunks += (o.bytes + kChunk - 1) / kChunk;
      p->total_hops += o.depth;
    }
    p->leaf_pre.push_back(chunks);
    p->total_chunks = chunks;
    p->out_bytes = first ? 0 : align_up(oend, align);
  }

  // the leaves each relocation unit's slots discover: a leaf belongs to the
  // unit holding the slot that first reached it. When the owning units never
  // decrease along the leaf order (a depth-first layout whose struct arrays
  // list their leaf members before deeper struct members, as every workload
  // here does), every unit owns one contiguous run of leaves
  {
    const uint64_t nl = p->leaves.size(), ns = p->segs.size();
    bool mono = ns > 0 && ns < kNone;
    uint64_t u = 0;
    for (uint64_t s = 0; s < ns; s++) p->segs[s].leaf_lo = p->segs[s].leaf_hi = 0;
    for (uint64_t l = 0; l < nl && mono; l++) {
      const uint64_t slot = p->objs[p->leaves[l]].slot;
      while (u + 1 < ns && p->segs[u].slot_hi <= slot) u++;
      if (slot < p->segs[u].slot_lo || slot >= p->segs[u].slot_hi) mono = false;  // an earlier unit
      else if (p->segs[u].leaf_hi == 0) p->segs[u].leaf_lo = (uint32_t)l, p->segs[u].leaf_hi = (uint32_t)l + 1;
      else p->segs[u].leaf_hi = (uint32_t)l + 1;
    }
    // units without leaves get the empty run where the next leaves start
    uint32_t at = (uint32_t)nl;
    for (uint64_t s = ns; s-- > 0;) {
      if (p->segs[s].leaf_hi == 0) p->segs[s].leaf_lo = p->segs[s].leaf_hi = at;
      else at = p->segs[s].leaf_lo;
    }
    p->unit_leaves = mono && nl > 0 && nl < kNone;
    for (uint64_t s = 0; s < ns && p->unit_leaves; s++)
      p->max_unit_leaf_chunks = std::max<uint64_t>(
          p->max_unit_leaf_chunks, p->leaf_pre[p->segs[s].leaf_hi] - p->leaf_pre[p->segs[s].leaf_lo]);
  }

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
    s.leaf_slot = take(8 * nl);
    s.leaf_pre = take(8 * (nl + 1));
    s.leaf_info = take(8 * nl);
    s.leaf_out = take(8 * nl);
    s.static_end = at;
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
