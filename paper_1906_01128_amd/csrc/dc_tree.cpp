// libdc tree operations: the deep copy (pack, transfer, relocate), chain
// resolution, the leaf kernels and the copy back.
#include <string.h>

#include <algorithm>

#include "dc_host.h"

namespace dc {

static Tables make_tables(dc_plan p, uint8_t* arena, uint8_t* scratch) {
  const ScratchLayout& s = p->sl;
  Tables t{};
  t.hdr = (DevHeader*)(scratch + s.header);
  t.types = (const DevType*)(scratch + s.types);
  t.sobj = (const DevSObj*)(scratch + s.sobj);
  t.sobj_pre = (const uint64_t*)(scratch + s.sobj_pre);
  t.segs = (const DevSeg*)(scratch + s.segs);
  t.tgts = (const DevTarget*)(scratch + s.tgts);
  t.slot_tix = (const uint16_t*)(scratch + s.slot_tix);
  t.leaf_slot = (const uint64_t*)(scratch + s.leaf_slot);
  t.leaf_pre = (const uint64_t*)(scratch + s.leaf_pre);
  t.leaf_info = (const uint64_t*)(scratch + s.leaf_info);
  t.leaf_out = (const uint64_t*)(scratch + s.leaf_out);
  t.leaf_tgt = (const uint32_t*)(scratch + s.leaf_tgt);
  t.leaf_dev = (const uint64_t*)(scratch + s.leaf_dev);
  t.resid = (const DevResid*)(scratch + s.resid);
  t.nresid = p->resid.size();
  t.tiles = (const DevTile*)(scratch + s.tiles);
  t.paths = (const DevPath*)(scratch + s.paths);
  t.hops = (const uint64_t*)(scratch + s.hops);
  t.arena = arena;
  t.arena_bytes = p->arena_bytes;
  t.nseg = p->segs.size();
  t.nleaves = p->leaves.size();
  t.total_chunks = p->total_chunks;
  t.ntypes = (uint32_t)p->dev_types.size();
  return t;
}

static dc_status check_buffers(dc_plan p, void* d_arena, uint64_t arena_bytes, void* d_scratch,
                               uint64_t scratch_bytes) {
  if (arena_bytes < p->arena_bytes)
    return fail(DC_E_RANGE, "arena of %llu bytes, plan needs %llu", (unsigned long long)arena_bytes,
                (unsigned long long)p->arena_bytes);
  if (scratch_bytes < p->sl.total)
    return fail(DC_E_RANGE, "scratch of %llu bytes, plan needs %llu", (unsigned long long)scratch_bytes,
                (unsigned long long)p->sl.total);
  if ((!d_arena && p->arena_bytes) || !d_scratch) return fail(DC_E_INVAL, "null device buffer");
  if (((uintptr_t)d_arena | (uintptr_t)d_scratch) & 255) return fail(DC_E_RANGE, "device buffers must be 256-byte aligned");
  return DC_OK;
}

// The plan's tables, with a fresh header, into scratch [0, static_end).
static dc_status upload_tables(dc_ctx ctx, dc_plan p, uint8_t* arena, uint8_t* scratch, hipStream_t s,
                               DevHeader* hdr_store) {
  DevHeader& h = *hdr_store;
  memset(&h, 0, sizeof(h));
  h.arena = (uint64_t)(uintptr_t)arena;
  h.nobj = p->objs.size();
  h.nsobj = p->sobj.size();
  h.nseg = p->segs.size();
  h.nleaves = p->leaves.size();
  h.nslots = p->sobj_pre.back();
  h.total_chunks = p->total_chunks;
  h.err_slot = ~0ull;
  h.chain_status = kErrNullChain;
  const ScratchLayout& sl = p->sl;
  std::vector<Piece> pcs;
  auto add = [&](uint64_t off, const void* src, uint64_t bytes) {
    if (bytes) pcs.push_back({off, src, bytes});
  };
  add(sl.header, &h, sizeof(h));
  add(sl.types, p->dev_types.data(), sizeof(DevType) * p->dev_types.size());
  add(sl.sobj, p->sobj.data(), sizeof(DevSObj) * p->sobj.size());
  add(sl.sobj_pre, p->sobj_pre.data(), 8 * p->sobj_pre.size());
  add(sl.segs, p->segs.data(), sizeof(DevSeg) * p->segs.size());
  add(sl.tgts, p->tgts.data(), sizeof(DevTarget) * p->tgts.size());
  add(sl.slot_tix, p->slot_tix.data(), 2 * p->slot_tix.size());
  add(sl.leaf_slot, p->leaf_slot.data(), 8 * p->leaf_slot.size());
  add(sl.leaf_info, p->leaf_info.data(), 8 * p->leaf_info.size());
  add(sl.leaf_out, p->leaf_out.data(), 8 * p->leaf_out.size());
  add(sl.leaf_tgt, p->leaf_tgt.data(), 4 * p->leaf_tgt.size());
  add(sl.leaf_dev, p->leaf_dev.data(), 8 * p->leaf_dev.size());
  add(sl.resid, p->resid.data(), sizeof(DevResid) * p->resid.size());
  // packing is synchronous, so the header copy may live on the stack
  return upload_pieces(ctx, scratch, sl.static_end, pcs, s);
}

static PieceSource arena_source(dc_plan p) {
  PieceSource src;
  src.n = p->objs.size();
  src.at = [p](uint64_t i) {
    const Obj& o = p->objs[i];
    return Piece{o.off, (const void*)(uintptr_t)o.host, o.bytes};
  };
  src.first_ending_after = [p](uint64_t x) {
    // objects are in increasing offset order; the first whose extent ends after x
    uint64_t lo = 0, hi = p->objs.size();
    while (lo < hi) {
      const uint64_t mid = (lo + hi) / 2;
      const Obj& o = p->objs[mid];
      if (o.off + std::max<uint64_t>(o.bytes, 1) <= x) lo = mid + 1;
      else hi = mid;
    }
    return lo;
  };
  return src;
}

dc_status deep_copy(dc_ctx ctx, dc_plan p, void* d_arena, uint64_t arena_bytes, void* d_scratch,
                    uint64_t scratch_bytes, void* stream, bool attach, dc_tree* out) {
  if (!out) return fail(DC_E_INVAL, "out is null");
  *out = nullptr;
  if (!ctx || !p) return fail(DC_E_INVAL, "null context or plan");
  DC_TRY(check_buffers(p, d_arena, arena_bytes, d_scratch, scratch_bytes));
  DC_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  uint8_t* arena = (uint8_t*)d_arena;
  uint8_t* scratch = (uint8_t*)d_scratch;
  DevHeader h;
  DC_TRY(upload_tables(ctx, p, arena, scratch, s, &h));
  {
    const ScratchLayout& sl = p->sl;
    const hipError_t e = launch_leaf_prefix((const uint64_t*)(scratch + sl.leaf_info), p->leaves.size(),
                                            (uint64_t*)(scratch + sl.leaf_pre), (uint64_t*)(scratch + sl.leaf_pre_scan), s);
    if (e != hipSuccess) return fail(DC_E_HIP, "leaf prefix launch: %s", hipGetErrorString(e));
  }
  DC_TRY(upload_source(ctx, arena, p->arena_bytes, arena_source(p), s));
  dc_tree t = new dc_tree_s();
  t->ctx = ctx;
  t->plan = p;
  t->arena = arena;
  t->scratch = scratch;
  t->tab = make_tables(p, arena, scratch);
  if (attach) {
    hipError_t e = launch_relocate(t->tab, true, s);
    if (e != hipSuccess) {
      delete t;
      return fail(DC_E_HIP, "relocate launch: %s", hipGetErrorString(e));
    }
    t->attached = true;
  }
  *out = t;
  clear_error();
  return DC_OK;
}

dc_status tree_check(dc_tree t, hipStream_t s) {
  DC_HIP(hipMemcpyAsync(t->ctx->small, t->tab.hdr, sizeof(DevHeader), hipMemcpyDeviceToHost, s));
  DC_HIP(hipStreamSynchronize(s));
  const DevHeader* h = (const DevHeader*)t->ctx->small;
  if (h->err_count || h->err_code)
    return fail(DC_E_STATE, "device check failed: code %u, %u bad pointer slot(s), first at arena offset %llu%s",
                h->err_code, h->err_count, (unsigned long long)h->err_slot,
                h->spin_fail ? " (persistent kernel wait bound hit)" : "");
  return DC_OK;
}

dc_status tree_ensure_tiles(dc_tree t, uint32_t T, hipStream_t s) {
  if (t->tile_T == T) {
    if (t->tiles_ev) DC_HIP(hipStreamWaitEvent(s, t->tiles_ev, 0));
    return DC_OK;
  }
  if (T < kTileMinChunks || T > kTileMaxChunks || (T & (T - 1))) return fail(DC_E_INVAL, "tile of %u chunks", T);
  if (t->plan->leaves.empty()) return DC_OK;
  // the list is rewritten in place: kernels on other streams may still read the old one
  if (t->tile_T != 0) DC_HIP(hipDeviceSynchronize());
  if (!t->tiles_ev) DC_HIP(hipEventCreateWithFlags(&t->tiles_ev, hipEventDisableTiming));
  const std::vector<DevTile> tiles = build_tiles(t->plan, T);
  const uint64_t bytes = sizeof(DevTile) * tiles.size();
  if (bytes > t->plan->sl.paths - t->plan->sl.tiles) return fail(DC_E_RANGE, "tile list exceeds its scratch space");
  std::vector<Piece> pcs{{0, tiles.data(), bytes}};
  DC_TRY(upload_pieces(t->ctx, t->scratch + t->plan->sl.tiles, bytes, pcs, s));
  DC_HIP(hipEventRecord(t->tiles_ev, s));
  t->tile_T = T;
  t->ntiles = tiles.size();
  return DC_OK;
}

// Pointer paths of every leaf, for per-access walks; uploaded on first use.
static dc_status ensure_paths(dc_tree t, hipStream_t s) {
  if (t->paths_uploaded) return DC_OK;
  dc_plan p = t->plan;
  std::vector<DevPath> paths(p->leaves.size());
  std::vector<uint64_t> hops(p->total_hops + 1, 0);
  uint64_t at = 0;
  for (size_t l = 0; l < p->leaves.size(); l++) {
    uint32_t o = p->leaves[l];
    const uint32_t d = p->objs[o].depth;
    paths[l].hop_lo = (uint32_t)at;
    paths[l].nhops = d;
    for (uint32_t k = d; k > 0; k--) {
      hops[at + k - 1] = p->objs[o].parent_rel;
      o = p->objs[o].parent;
    }
    paths[l].root_off = p->objs[o].off;
    at += d;
  }
  std::vector<Piece> pcs;
  if (!paths.empty()) pcs.push_back({0, paths.data(), sizeof(DevPath) * paths.size()});
  DC_TRY(upload_pieces(t->ctx, t->scratch + p->sl.paths, sizeof(DevPath) * paths.size(), pcs, s));
  std::vector<Piece> hp{{0, hops.data(), 8 * hops.size()}};
  DC_TRY(upload_pieces(t->ctx, t->scratch + p->sl.hops, 8 * hops.size(), hp, s));
  DC_TRY(ctx_wait_ring(t->ctx));  // complete before any stream uses them
  t->paths_uploaded = true;
  return DC_OK;
}

// Follows a chain through the plan (no device access): the target object of
// every step, checking fields, nulls and indices.
struct ChainPlan {
  uint32_t target;  // object at the end
  ChainArgs dev;    // for the device resolver
  HopArgs hops;     // for per-access walks
};

static dc_status plan_chain(dc_plan p, uint64_t root_index, const dc_step* steps, uint32_t nsteps, ChainPlan* out) {
  if (root_index >= p->root_obj.size())
    return fail(DC_E_INVAL, "root index %llu of %zu", (unsigned long long)root_index, p->root_obj.size());
  if (nsteps == 0 || nsteps > kMaxChainSteps || !steps) return fail(DC_E_INVAL, "chain of %u steps", nsteps);
  memset(out, 0, sizeof(*out));
  uint32_t cur = p->root_obj[root_index];
  uint64_t e = 0;
  out->dev.root_off = p->objs[cur].off;
  out->dev.nsteps = nsteps;
  out->hops.root_off = p->objs[cur].off;
  out->hops.nhops = nsteps;
  uint64_t carry = 0;  // index * element size of the previous step
  for (uint32_t s = 0; s < nsteps; s++) {
    const Obj& o = p->objs[cur];
    if (o.kind != DC_KIND_STRUCT) return fail(DC_E_INVAL, "chain step %u starts in a primitive array", s);
    const TypeDesc& ty = p->types[o.type];
    if (steps[s].field >= ty.fields.size())
      return fail(DC_E_INVAL, "chain step %u: field %u of type %s with %zu fields", s, steps[s].field,
                  ty.name.c_str(), ty.fields.size());
    const dc_field& f = ty.fields[steps[s].field];
    const uint64_t slot = p->sobj_pre[o.sobj] + e * ty.order.size() + ty.pos[steps[s].field];
    const uint32_t tgt = p->slot_target[slot];
    if (tgt == kNone) return fail(DC_E_RANGE, "chain step %u reads a null pointer", s);
    const Obj& to = p->objs[tgt];
    out->dev.field_off[s] = f.offset;
    out->dev.cnt_off[s] = f.count_offset;
    out->dev.cnt_bytes[s] = f.count_bytes;
    out->dev.cnt_mult[s] = f.count_mult;
    out->dev.fixed[s] = f.fixed_count;
    out->dev.kind[s] = f.kind;
    out->dev.elem_size[s] = f.kind == DC_KIND_STRUCT ? p->types[f.type_id].size : 0;
    out->dev.index[s] = steps[s].index;
    out->hops.hop_off[s] = carry + f.offset;
    if (s + 1 == nsteps) {
      out->target = tgt;
      return DC_OK;
    }
    if (to.kind != DC_KIND_STRUCT) return fail(DC_E_INVAL, "chain step %u leads to a primitive array", s);
    if (steps[s].index >= to.count)
      return fail(DC_E_RANGE, "chain step %u: index %llu of %llu elements", s, (unsigned long long)steps[s].index,
                  (unsigned long long)to.count);
    if (to.sobj == kNone && s + 1 < nsteps) return fail(DC_E_RANGE, "chain step %u leads to a struct without pointers", s);
    carry = steps[s].index * p->types[to.type].size;
    cur = tgt;
    e = steps[s].index;
  }
  return fail(DC_E_INVAL, "empty chain");
}

// Chunks per tile of the plain every-leaf kernel. Small tiles (1024 chunks,
// one round of four chunks per thread) measured fastest on gfx950 for both
// cache-resident and HBM-sized trees: many short workgroups keep more
// requests in flight than fewer long ones.
// Tile size of the every-leaf kernels: 512-chunk tiles (two chunks per
// thread) for large leaves streamed from HBM, 1024-chunk tiles (four per
// thread) otherwise. Measured: large leaves well beyond the 256 MB Infinity
// Cache (the 1 GB wide tree, ~230 KB per leaf) 5.5 TB/s with 512 against 5.0
// with 1024; the same shape at 0.28 GB, mostly cache-resident, 5.1 against
// 5.6; small leaves (the 12 GB MD cells' arrays, ~1.5 KB), whose leaf-table
// prologue then serves fewer chunks per tile, 4.60 ms against 4.27.
static uint32_t leaf_tile_for(dc_plan p, int ncu) {
  (void)ncu;
  const uint64_t nl = p->leaves.size();
  const bool large = nl && p->total_chunks / nl >= 2048;  // 32 KB per leaf on average
  return large && p->leaf_bytes >= (512ull << 20) ? 512u : 1024u;
}

static uint64_t chain_out_bytes(dc_plan p, uint32_t target) {
  return align_up(std::max<uint64_t>(p->objs[target].bytes, 1), p->align);
}

dc_status tree_prepare_leaf_tiles(dc_tree t, hipStream_t s) {
  return tree_ensure_tiles(t, leaf_tile_for(t->plan, t->ctx->ncu), s);
}

}  // namespace dc

using namespace dc;

extern "C" {

dc_status dc_deep_copy_to_device(dc_ctx ctx, dc_plan plan, void* d_arena, uint64_t arena_bytes, void* d_scratch,
                                 uint64_t scratch_bytes, void* stream, dc_tree* out) {
  return deep_copy(ctx, plan, d_arena, arena_bytes, d_scratch, scratch_bytes, stream, true, out);
}

dc_status dc_stage_to_device(dc_ctx ctx, dc_plan plan, void* d_arena, uint64_t arena_bytes, void* d_scratch,
                             uint64_t scratch_bytes, void* stream, dc_tree* out) {
  return deep_copy(ctx, plan, d_arena, arena_bytes, d_scratch, scratch_bytes, stream, false, out);
}

static dc_status relocate(dc_tree t, bool attach, void* stream) {
  if (!t || t->released) return fail(DC_E_INVAL, "null or released tree");
  if (t->attached == attach)
    return fail(DC_E_STATE, attach ? "tree is already attached" : "tree is not attached");
  DC_HIP(hipSetDevice(t->ctx->device));
  hipError_t e = launch_relocate(t->tab, attach, (hipStream_t)stream);
  if (e != hipSuccess) return fail(DC_E_HIP, "relocate launch: %s", hipGetErrorString(e));
  t->attached = attach;
  return DC_OK;
}

dc_status dc_attach(dc_tree t, void* stream) { return relocate(t, true, stream); }
dc_status dc_detach(dc_tree t, void* stream) { return relocate(t, false, stream); }

dc_status dc_resolve_chain(dc_tree t, uint64_t root_index, const dc_step* steps, uint32_t nsteps, void* stream,
                           dc_chain* out) {
  if (!t || t->released || !out) return fail(DC_E_INVAL, "dc_resolve_chain: null argument");
  if (!t->attached) return fail(DC_E_STATE, "dc_resolve_chain: tree is not attached");
  ChainPlan cp;
  DC_TRY(plan_chain(t->plan, root_index, steps, nsteps, &cp));
  DC_HIP(hipSetDevice(t->ctx->device));
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_resolve_chain(t->tab, cp.dev, s);
  if (e != hipSuccess) return fail(DC_E_HIP, "resolve launch: %s", hipGetErrorString(e));
  DC_TRY(tree_check(t, s));
  const DevHeader* h = (const DevHeader*)t->ctx->small;
  const Obj& o = t->plan->objs[cp.target];
  const uint64_t want = (uint64_t)(uintptr_t)t->arena + o.off;
  if (h->chain_status != 0 || h->chain_addr != want || h->chain_count != o.count || h->chain_kind != o.kind)
    return fail(DC_E_STATE, "device chain resolution (status %u, %#llx, %llu) disagrees with the plan (%#llx, %llu)",
                h->chain_status, (unsigned long long)h->chain_addr, (unsigned long long)h->chain_count,
                (unsigned long long)want, (unsigned long long)o.count);
  out->dev_addr = h->chain_addr;
  out->count = h->chain_count;
  out->kind = h->chain_kind;
  out->reserved = 0;
  return DC_OK;
}

dc_status dc_out_bytes(dc_tree t, const dc_kernel_args* a, uint64_t* out) {
  if (!t || !a || !out) return fail(DC_E_INVAL, "dc_out_bytes: null argument");
  if (a->select == DC_SELECT_ALL_LEAVES) {
    *out = t->plan->out_bytes;
    return DC_OK;
  }
  ChainPlan cp;
  DC_TRY(plan_chain(t->plan, a->root_index, a->chain, a->nsteps, &cp));
  *out = chain_out_bytes(t->plan, cp.target);
  return DC_OK;
}

dc_status dc_run_kernel(dc_tree t, const dc_kernel_args* a, void* stream) {
  if (!t || t->released || !a) return fail(DC_E_INVAL, "dc_run_kernel: null argument");
  if (!t->attached) return fail(DC_E_STATE, "dc_run_kernel: tree is not attached");
  if (a->mode != DC_MODE_RESOLVED && a->mode != DC_MODE_DEREF_EACH) return fail(DC_E_INVAL, "mode %u", a->mode);
  if (a->select != DC_SELECT_CHAIN && a->select != DC_SELECT_ALL_LEAVES) return fail(DC_E_INVAL, "select %u", a->select);
  dc_plan p = t->plan;
  DC_HIP(hipSetDevice(t->ctx->device));
  hipStream_t s = (hipStream_t)stream;
  LeafArgs la{};
  la.a = a->a;
  la.b = a->b;
  la.af = a->af;
  la.bf = a->bf;
  la.out = (uint8_t*)a->d_out;
  if (la.out && ((uintptr_t)la.out & 15)) return fail(DC_E_RANGE, "d_out must be 16-byte aligned");
  hipError_t e = hipSuccess;
  if (a->select == DC_SELECT_CHAIN) {
    ChainPlan cp;
    DC_TRY(plan_chain(p, a->root_index, a->chain, a->nsteps, &cp));
    const Obj& o = p->objs[cp.target];
    if (o.kind != DC_KIND_F32 && o.kind != DC_KIND_F64)
      return fail(DC_E_INVAL, "the chain ends in an array of kind %u, not FP32/FP64", o.kind);
    if (la.out && a->out_bytes < chain_out_bytes(p, cp.target))
      return fail(DC_E_RANGE, "d_out of %llu bytes, needs %llu", (unsigned long long)a->out_bytes,
                  (unsigned long long)chain_out_bytes(p, cp.target));
    if (a->mode == DC_MODE_RESOLVED) {
      // Resolve once, before the passes (Section 3): the effective address
      // comes from the plan, and one walk of the relocated chain on the
      // device checks that the copy leads there; every pass then indexes it.
      const uint64_t base = (uint64_t)(uintptr_t)t->arena + o.off;
      cp.dev.expect_addr = base;
      e = launch_resolve_chain(t->tab, cp.dev, s);
      for (uint32_t it = 0; it < a->iters && e == hipSuccess; it++) {
        la.src_out = (la.out && it > 0) ? 1 : 0;
        e = launch_stream_resolved(t->tab, base, o.count, o.kind, la, s);
      }
    } else {
      for (uint32_t it = 0; it < a->iters && e == hipSuccess; it++) {
        la.src_out = (la.out && it > 0) ? 1 : 0;
        e = launch_stream_deref(t->tab, cp.hops, o.count, o.kind, la, s);
      }
    }
  } else {
    if (la.out && a->out_bytes < p->out_bytes)
      return fail(DC_E_RANGE, "d_out of %llu bytes, needs %llu", (unsigned long long)a->out_bytes,
                  (unsigned long long)p->out_bytes);
    if (p->leaves.empty() || a->iters == 0) return DC_OK;
    DC_TRY(tree_ensure_tiles(t, leaf_tile_for(p, t->ctx->ncu), s));
    const bool deref = a->mode == DC_MODE_DEREF_EACH;
    if (deref) DC_TRY(ensure_paths(t, s));
    for (uint32_t it = 0; it < a->iters && e == hipSuccess; it++) {
      la.src_out = (la.out && it > 0) ? 1 : 0;
      e = launch_leaf_tiles(t->tab, la, t->ntiles, t->tile_T, deref, s);
    }
  }
  if (e != hipSuccess) return fail(DC_E_HIP, "kernel launch: %s", hipGetErrorString(e));
  return DC_OK;
}

dc_status dc_copy_back(dc_tree t, uint32_t flags, void* stream) {
  if (!t || t->released) return fail(DC_E_INVAL, "dc_copy_back: null or released tree");
  if (flags & ~(uint32_t)(DC_COPY_LEAVES | DC_COPY_SCALARS)) return fail(DC_E_INVAL, "flags %#x", flags);
  dc_plan p = t->plan;
  DC_HIP(hipSetDevice(t->ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const bool leaves = flags & DC_COPY_LEAVES, scalars = flags & DC_COPY_SCALARS;
  // the range of the arena holding anything to copy back
  uint64_t lo = ~0ull, hi = 0;
  for (const Obj& o : p->objs) {
    const bool want = (o.kind == DC_KIND_STRUCT) ? scalars : leaves;
    if (!want || o.bytes == 0) continue;
    lo = std::min(lo, o.off);
    hi = std::max(hi, o.off + o.bytes);
  }
  if (hi > lo) {
    const PieceSource src = arena_source(p);
    Pool* pool = t->ctx->pool;
    dc_status st = download(t->ctx, t->arena, lo, hi, s, [&](const uint8_t* buf, uint64_t clo, uint64_t chi) {
      const uint64_t part = 1ull << 20;
      const int nparts = (int)((chi - clo + part - 1) / part);
      pool->run(nparts, [&](int k) {
        const uint64_t plo = clo + (uint64_t)k * part, phi = std::min(chi, plo + part);
        for (uint64_t i = src.first_ending_after(plo); i < p->objs.size(); i++) {
          const Obj& o = p->objs[i];
          if (o.off >= phi) break;
          const uint64_t a = std::max(o.off, plo), b = std::min(o.off + o.bytes, phi);
          if (b <= a) continue;
          uint8_t* host = (uint8_t*)(uintptr_t)o.host;
          if (o.kind != DC_KIND_STRUCT) {
            if (leaves) copy_stream(host + (a - o.off), buf + (a - clo), b - a);
          } else if (scalars) {
            const TypeDesc& ty = p->types[o.type];
            for (uint64_t x = a; x < b;) {
              const uint64_t e = (x - o.off) / ty.size;
              const uint64_t ebase = o.off + e * ty.size;
              for (const auto& run : ty.plain_runs) {
                const uint64_t ra = std::max(ebase + run.first, x), rb = std::min(ebase + run.second, b);
                if (rb > ra) memcpy(host + (ra - o.off), buf + (ra - clo), rb - ra);
              }
              x = ebase + ty.size;
            }
          }
        }
      });
    });
    DC_TRY(st);
  }
  DC_TRY(tree_check(t, s));
  return DC_OK;
}

dc_status dc_tree_check(dc_tree t, void* stream) {
  if (!t || t->released) return fail(DC_E_INVAL, "dc_tree_check: null or released tree");
  DC_HIP(hipSetDevice(t->ctx->device));
  return tree_check(t, (hipStream_t)stream);
}

dc_status dc_tree_objects(dc_tree t, dc_object* out, uint64_t cap, uint64_t* n) {
  if (!t || t->released) return fail(DC_E_INVAL, "dc_tree_objects: null or released tree");
  DC_TRY(dc_plan_objects(t->plan, out, cap, n));
  const uint64_t m = std::min<uint64_t>(cap, t->plan->objs.size());
  for (uint64_t i = 0; i < m; i++) out[i].offset += (uint64_t)(uintptr_t)t->arena;
  return DC_OK;
}

dc_status dc_tree_release(dc_tree t) {
  if (!t) return fail(DC_E_INVAL, "dc_tree_release: null tree");
  t->released = true;
  if (t->tiles_ev) (void)hipEventDestroy(t->tiles_ev);
  kd_free(t);
  if (t->noalloc_dev >= 0) {
    // the device's fixed scratch is free for the next no-allocation copy once
    // nothing queued still reads this tree's tables from it
    (void)hipSetDevice(t->ctx->device);
    (void)hipDeviceSynchronize();
    noalloc_release(t->noalloc_dev);
  }
  delete t;
  return DC_OK;
}

}  // extern "C"
