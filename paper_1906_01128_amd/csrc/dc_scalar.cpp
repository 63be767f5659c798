// libdc scalar chains (Section 3, scalar variables): a scalar member reached
// by a chain is read into a temporary on the device and written back through
// the chain when the region that uses it ends.
#include <string.h>

#include "dc_host.h"

namespace dc {

// Follows one scalar chain through the plan: the device hops and the arena
// offset the scalar must be found at.
static dc_status plan_scalar(dc_plan p, const dc_scalar_ref& r, uint32_t idx, std::vector<DevScalarHop>& hops,
                             DevScalar* out) {
  if (r.root_index >= p->root_obj.size())
    return fail(DC_E_INVAL, "scalar %u: root index %llu of %zu", idx, (unsigned long long)r.root_index,
                p->root_obj.size());
  if (r.nsteps > kMaxChainSteps || (r.nsteps && !r.steps))
    return fail(DC_E_INVAL, "scalar %u: chain of %u steps", idx, r.nsteps);
  if (r.bytes != 1 && r.bytes != 4 && r.bytes != 8) return fail(DC_E_INVAL, "scalar %u: %u bytes", idx, r.bytes);
  uint32_t cur = p->root_obj[r.root_index];
  uint64_t e = 0;
  out->root_off = p->objs[cur].off;
  out->hop_lo = (uint32_t)hops.size();
  out->nhops = r.nsteps;
  for (uint32_t s = 0; s < r.nsteps; s++) {
    const Obj& o = p->objs[cur];
    const TypeDesc& ty = p->types[o.type];
    if (r.steps[s].field >= ty.fields.size())
      return fail(DC_E_INVAL, "scalar %u step %u: field %u of type %s", idx, s, r.steps[s].field, ty.name.c_str());
    const dc_field& f = ty.fields[r.steps[s].field];
    if (f.kind != DC_KIND_STRUCT) return fail(DC_E_INVAL, "scalar %u step %u leads to a primitive array", idx, s);
    if (o.sobj == kNone) return fail(DC_E_RANGE, "scalar %u step %u: element has no pointer members", idx, s);
    const uint64_t slot = p->sobj_pre[o.sobj] + e * ty.order.size() + ty.pos[r.steps[s].field];
    const uint32_t tgt = p->slot_target[slot];
    if (tgt == kNone) return fail(DC_E_RANGE, "scalar %u step %u reads a null pointer", idx, s);
    const Obj& to = p->objs[tgt];
    if (r.steps[s].index >= to.count)
      return fail(DC_E_RANGE, "scalar %u step %u: index %llu of %llu", idx, s,
                  (unsigned long long)r.steps[s].index, (unsigned long long)to.count);
    hops.push_back({f.offset, p->types[to.type].size, r.steps[s].index});
    cur = tgt;
    e = r.steps[s].index;
  }
  const Obj& o = p->objs[cur];
  const TypeDesc& ty = p->types[o.type];
  if ((uint64_t)r.offset + r.bytes > ty.size)
    return fail(DC_E_RANGE, "scalar %u: bytes [%u, %u) past the %u-byte %s", idx, r.offset, r.offset + r.bytes,
                ty.size, ty.name.c_str());
  for (const dc_field& f : ty.fields)
    if (r.offset < f.offset + 8 && f.offset < r.offset + r.bytes)
      return fail(DC_E_INVAL, "scalar %u overlaps the pointer member at offset %u of %s", idx, f.offset,
                  ty.name.c_str());
  out->expect_off = o.off + e * ty.size + r.offset;
  out->offset = r.offset;
  out->bytes = r.bytes;
  return DC_OK;
}

static dc_status ensure_aux(dc_ctx ctx, uint64_t bytes) {
  if (ctx->aux_bytes >= bytes) return DC_OK;
  if (ctx->aux) {
    DC_HIP(hipDeviceSynchronize());
    DC_HIP(hipFree(ctx->aux));
    ctx->aux = nullptr;
    ctx->aux_bytes = 0;
  }
  uint64_t cap = 1ull << 16;
  while (cap < bytes) cap *= 2;
  if (hipMalloc((void**)&ctx->aux, cap) != hipSuccess) return fail(DC_E_NOMEM, "scalar descriptors: %llu bytes",
                                                                    (unsigned long long)cap);
  ctx->aux_bytes = cap;
  return DC_OK;
}

static dc_status scalar_pass(dc_tree t, const dc_scalar_ref* refs, uint32_t n, void* d_temps, int update,
                             void* stream) {
  if (!t || t->released || (n && (!refs || !d_temps))) return fail(DC_E_INVAL, "scalar chain: null argument");
  if (!t->attached) return fail(DC_E_STATE, "scalar chain: tree is not attached");
  if ((uintptr_t)d_temps & 7) return fail(DC_E_INVAL, "scalar chain: temporaries must be 8-byte aligned");
  if (n == 0) return DC_OK;
  std::vector<DevScalar> ds(n);
  std::vector<DevScalarHop> hops;
  for (uint32_t i = 0; i < n; i++) DC_TRY(plan_scalar(t->plan, refs[i], i, hops, &ds[i]));
  const uint64_t rbytes = sizeof(DevScalar) * (uint64_t)n;
  const uint64_t hbytes = sizeof(DevScalarHop) * hops.size();
  const uint64_t hoff = (rbytes + 255) & ~255ull;
  dc_ctx ctx = t->ctx;
  DC_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  DC_TRY(ensure_aux(ctx, hoff + hbytes + 16));
  std::vector<Piece> pcs{{0, ds.data(), rbytes}};
  if (hbytes) pcs.push_back({hoff, hops.data(), hbytes});
  DC_TRY(upload_pieces(ctx, ctx->aux, hoff + hbytes, pcs, s));
  hipError_t e = launch_scalar(t->tab, (const DevScalar*)ctx->aux, (const DevScalarHop*)(ctx->aux + hoff), n,
                               (uint64_t*)d_temps, update, s);
  if (e != hipSuccess) return fail(DC_E_HIP, "scalar chain launch: %s", hipGetErrorString(e));
  return tree_check(t, s);
}

}  // namespace dc

using namespace dc;

extern "C" {

dc_status dc_scalar_declare(dc_tree t, const dc_scalar_ref* refs, uint32_t nrefs, void* d_temps, void* stream) {
  return scalar_pass(t, refs, nrefs, d_temps, 0, stream);
}

dc_status dc_scalar_update(dc_tree t, const dc_scalar_ref* refs, uint32_t nrefs, const void* d_temps,
                           void* stream) {
  return scalar_pass(t, refs, nrefs, const_cast<void*>(d_temps), 1, stream);
}

}  // extern "C"
