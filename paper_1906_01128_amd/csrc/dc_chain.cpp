// libdc pointerchain transfer scheme (Section 3): the chain is resolved on
// the host tree and only the array it ends in travels to the device.
#include <string.h>

#include <algorithm>

#include "dc_host.h"

namespace dc {

static uint64_t kind_size(uint32_t kind) {
  switch (kind) {
    case DC_KIND_F32:
    case DC_KIND_I32: return 4;
    case DC_KIND_F64:
    case DC_KIND_I64: return 8;
    case DC_KIND_U8: return 1;
  }
  return 0;
}

// Walks the chain through host memory: the host address, count and kind of
// the array it ends in.
static dc_status host_chain(const dc_schema_s* sc, uint32_t root_type, const void* root, const dc_step* steps,
                            uint32_t nsteps, uint64_t* addr, uint64_t* count, uint32_t* kind) {
  if (!sc || !root || !steps || nsteps == 0 || nsteps > kMaxChainSteps)
    return fail(DC_E_INVAL, "chain: null argument or %u steps", nsteps);
  if (root_type >= sc->types.size()) return fail(DC_E_INVAL, "chain: root type %u", root_type);
  uint32_t type = root_type;
  const uint8_t* elem = (const uint8_t*)root;
  for (uint32_t s = 0; s < nsteps; s++) {
    const TypeDesc& t = sc->types[type];
    if (steps[s].field >= t.fields.size()) return fail(DC_E_INVAL, "chain step %u: field %u", s, steps[s].field);
    const dc_field& f = t.fields[steps[s].field];
    uint64_t p;
    memcpy(&p, elem + f.offset, 8);
    uint64_t n = f.fixed_count;
    if (f.count_offset >= 0) {
      int64_t v;
      if (f.count_bytes == 4) {
        int32_t v32;
        memcpy(&v32, elem + f.count_offset, 4);
        v = v32;
      } else {
        memcpy(&v, elem + f.count_offset, 8);
      }
      if (v < 0) return fail(DC_E_INVAL, "chain step %u: negative count", s);
      n = (uint64_t)v * f.count_mult;
    }
    if (p == 0) return fail(DC_E_RANGE, "chain step %u reads a null pointer", s);
    if (s + 1 == nsteps) {
      *addr = p;
      *count = n;
      *kind = f.kind;
      return DC_OK;
    }
    if (f.kind != DC_KIND_STRUCT) return fail(DC_E_INVAL, "chain step %u leads to a primitive array", s);
    if (steps[s].index >= n) return fail(DC_E_RANGE, "chain step %u: index %llu of %llu", s,
                                         (unsigned long long)steps[s].index, (unsigned long long)n);
    type = f.type_id;
    if (type >= sc->types.size()) return fail(DC_E_INVAL, "chain step %u: type %u", s, type);
    elem = (const uint8_t*)(uintptr_t)p + steps[s].index * sc->types[type].size;
  }
  return fail(DC_E_INVAL, "empty chain");
}

}  // namespace dc

using namespace dc;

extern "C" {

dc_status dc_chain_query(dc_schema schema, uint32_t root_type, const void* root, const dc_step* steps,
                         uint32_t nsteps, dc_chain* out) {
  if (!out) return fail(DC_E_INVAL, "dc_chain_query: null argument");
  uint64_t addr, count;
  uint32_t kind;
  DC_TRY(host_chain(schema, root_type, root, steps, nsteps, &addr, &count, &kind));
  out->dev_addr = 0;
  out->count = count;
  out->kind = kind;
  out->reserved = 0;
  return DC_OK;
}

dc_status dc_chain_to_device(dc_ctx ctx, dc_schema schema, uint32_t root_type, const void* root, const dc_step* steps,
                             uint32_t nsteps, void* d_buf, uint64_t buf_bytes, void* stream, dc_chain* out) {
  if (!ctx || !out || !d_buf) return fail(DC_E_INVAL, "dc_chain_to_device: null argument");
  uint64_t addr, count;
  uint32_t kind;
  DC_TRY(host_chain(schema, root_type, root, steps, nsteps, &addr, &count, &kind));
  if (kind == DC_KIND_STRUCT) return fail(DC_E_INVAL, "dc_chain_to_device: the chain ends in a struct array");
  const uint64_t es = kind_size(kind);
  const uint64_t bytes = count * es;
  if (bytes > buf_bytes) return fail(DC_E_RANGE, "buffer of %llu bytes, the array needs %llu",
                                     (unsigned long long)buf_bytes, (unsigned long long)bytes);
  if ((uintptr_t)d_buf & 15) return fail(DC_E_RANGE, "d_buf must be 16-byte aligned");
  DC_HIP(hipSetDevice(ctx->device));
  std::vector<Piece> pcs;
  if (bytes) pcs.push_back({0, (const void*)(uintptr_t)addr, bytes});
  DC_TRY(upload_pieces(ctx, (uint8_t*)d_buf, bytes, pcs, (hipStream_t)stream));
  out->dev_addr = (uint64_t)(uintptr_t)d_buf;
  out->count = count;
  out->kind = kind;
  out->reserved = 0;
  return DC_OK;
}

dc_status dc_chain_run_kernel(dc_ctx ctx, const dc_chain* c, uint32_t iters, double a, double b, float af, float bf,
                              void* stream) {
  if (!ctx || !c || !c->dev_addr) return fail(DC_E_INVAL, "dc_chain_run_kernel: null argument");
  if (c->kind != DC_KIND_F32 && c->kind != DC_KIND_F64) return fail(DC_E_INVAL, "kind %u is not FP32/FP64", c->kind);
  DC_HIP(hipSetDevice(ctx->device));
  // the array is the whole "arena" of this transfer
  Tables t{};
  t.hdr = ctx->dev_hdr;
  t.arena = (uint8_t*)(uintptr_t)c->dev_addr;
  t.arena_bytes = c->count * kind_size(c->kind);
  LeafArgs la{};
  la.a = a;
  la.b = b;
  la.af = af;
  la.bf = bf;
  hipError_t e = hipSuccess;
  for (uint32_t it = 0; it < iters && e == hipSuccess; it++)
    e = launch_stream_resolved(t, c->dev_addr, c->count, c->kind, la, (hipStream_t)stream);
  if (e != hipSuccess) return fail(DC_E_HIP, "kernel launch: %s", hipGetErrorString(e));
  return DC_OK;
}

dc_status dc_chain_copy_back(dc_ctx ctx, dc_schema schema, uint32_t root_type, const void* root, const dc_step* steps,
                             uint32_t nsteps, const dc_chain* c, void* stream) {
  if (!ctx || !c) return fail(DC_E_INVAL, "dc_chain_copy_back: null argument");
  uint64_t addr, count;
  uint32_t kind;
  DC_TRY(host_chain(schema, root_type, root, steps, nsteps, &addr, &count, &kind));
  if (count != c->count || kind != c->kind) return fail(DC_E_STATE, "the chain no longer ends in the same array shape");
  const uint64_t bytes = count * kind_size(kind);
  DC_HIP(hipSetDevice(ctx->device));
  uint8_t* host = (uint8_t*)(uintptr_t)addr;
  Pool* pool = ctx->pool;
  DC_TRY(download(ctx, (const uint8_t*)(uintptr_t)c->dev_addr, 0, bytes, (hipStream_t)stream,
                  [&](const uint8_t* buf, uint64_t lo, uint64_t hi) {
                    const uint64_t part = 1ull << 20;
                    const int nparts = (int)((hi - lo + part - 1) / part);
                    pool->run(nparts, [&](int k) {
                      const uint64_t a = lo + (uint64_t)k * part, b = std::min(hi, a + part);
                      copy_stream(host + a, buf + (a - lo), b - a);
                    });
                  }));
  return DC_OK;
}

}  // extern "C"
