/* CPU oracle: deep copy, relocation, chain resolution, leaf kernel and copy
 * back, written out plainly. TEST INFRASTRUCTURE (see oracle.h). */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

struct or_copy {
  const or_type* types; /* copied */
  uint32_t ntypes;
  uint32_t* follow;     /* per type: fields to follow (bit per field) */
  uint64_t align, base;
  void* const* roots;
  uint64_t nroots;
  uint64_t* root_obj; /* object index of each root */

  or_object* objs;
  uint64_t nobjs, cap;

  /* visited map: host address -> object index (open addressing) */
  uint64_t* keys;
  uint64_t* vals;
  uint64_t mask;

  uint8_t* arena;
  uint64_t arena_bytes;
  uint64_t nslots;
};

static const uint64_t kEmpty = 0;

static uint64_t elem_size(const or_copy* c, uint32_t kind, uint32_t type) {
  switch (kind) {
    case OR_STRUCT: return c->types[type].size;
    case OR_F32: return 4;
    case OR_F64: return 8;
    case OR_I32: return 4;
    case OR_I64: return 8;
    case OR_U8: return 1;
  }
  return 0;
}

static uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

static uint64_t hash_addr(uint64_t p) { return (p >> 3) * 0x9E3779B97F4A7C15ull; }

static int map_grow(or_copy* c);

static int64_t map_find(const or_copy* c, uint64_t key) {
  uint64_t i = hash_addr(key) & c->mask;
  while (c->keys[i] != kEmpty) {
    if (c->keys[i] == key) return (int64_t)c->vals[i];
    i = (i + 1) & c->mask;
  }
  return -1;
}

static int map_insert(or_copy* c, uint64_t key, uint64_t val) {
  if (2 * (c->nobjs + 1) > c->mask + 1 && map_grow(c)) return OR_E_NOMEM;
  uint64_t i = hash_addr(key) & c->mask;
  while (c->keys[i] != kEmpty) i = (i + 1) & c->mask;
  c->keys[i] = key;
  c->vals[i] = val;
  return OR_OK;
}

static int map_grow(or_copy* c) {
  uint64_t ncap = (c->mask + 1) * 2;
  uint64_t* nk = (uint64_t*)calloc(ncap, sizeof(uint64_t));
  uint64_t* nv = (uint64_t*)calloc(ncap, sizeof(uint64_t));
  if (!nk || !nv) {
    free(nk);
    free(nv);
    return OR_E_NOMEM;
  }
  for (uint64_t i = 0; i <= c->mask; i++) {
    if (c->keys[i] == kEmpty) continue;
    uint64_t j = hash_addr(c->keys[i]) & (ncap - 1);
    while (nk[j] != kEmpty) j = (j + 1) & (ncap - 1);
    nk[j] = c->keys[i];
    nv[j] = c->vals[i];
  }
  free(c->keys);
  free(c->vals);
  c->keys = nk;
  c->vals = nv;
  c->mask = ncap - 1;
  return OR_OK;
}

/* The element count of the array a pointer field refers to: a signed count
 * member of the same element times the multiplier, or the fixed count. */
static int field_count(const or_field* f, const uint8_t* elem, uint64_t* count) {
  if (f->count_offset < 0) {
    *count = f->fixed_count;
    return OR_OK;
  }
  int64_t n;
  if (f->count_bytes == 4) {
    int32_t v;
    memcpy(&v, elem + f->count_offset, 4);
    n = v;
  } else if (f->count_bytes == 8) {
    memcpy(&n, elem + f->count_offset, 8);
  } else {
    return OR_E_INVAL;
  }
  if (n < 0) return OR_E_INVAL;
  *count = (uint64_t)n * f->count_mult;
  return OR_OK;
}

static int push_object(or_copy* c, uint64_t host, uint32_t kind, uint32_t type, uint64_t count, uint64_t* idx) {
  if (c->nobjs == c->cap) {
    uint64_t ncap = c->cap ? 2 * c->cap : 64;
    or_object* no = (or_object*)realloc(c->objs, ncap * sizeof(or_object));
    if (!no) return OR_E_NOMEM;
    c->objs = no;
    c->cap = ncap;
  }
  or_object* o = &c->objs[c->nobjs];
  o->host = host;
  o->kind = kind;
  o->type = type;
  o->count = count;
  o->bytes = count * elem_size(c, kind, type);
  o->off = 0;
  *idx = c->nobjs;
  int rc = map_insert(c, host, c->nobjs);
  if (rc) return rc;
  c->nobjs++;
  return OR_OK;
}

/* Depth-first pre-order: emit the object, then, for each element in index
 * order and each pointer field in ascending offset order, visit a non-null
 * target that has not been visited. A target reached again must have the
 * same kind, type and element count. */
static int visit(or_copy* c, uint64_t idx) {
  or_object o = c->objs[idx];
  if (o.kind != OR_STRUCT) return OR_OK;
  const or_type* t = &c->types[o.type];
  /* field visiting order: ascending byte offset */
  uint32_t order[OR_MAX_FIELDS];
  for (uint32_t i = 0; i < t->nfields; i++) order[i] = i;
  for (uint32_t i = 1; i < t->nfields; i++)
    for (uint32_t j = i; j > 0 && t->fields[order[j]].offset < t->fields[order[j - 1]].offset; j--) {
      uint32_t tmp = order[j];
      order[j] = order[j - 1];
      order[j - 1] = tmp;
    }
  for (uint64_t e = 0; e < o.count; e++) {
    const uint8_t* elem = (const uint8_t*)(uintptr_t)o.host + e * t->size;
    for (uint32_t k = 0; k < t->nfields; k++) {
      if (!((c->follow[o.type] >> order[k]) & 1u)) continue;
      const or_field* f = &t->fields[order[k]];
      uint64_t p;
      memcpy(&p, elem + f->offset, 8);
      if (p == 0) continue;
      uint64_t count;
      int rc = field_count(f, elem, &count);
      if (rc) return rc;
      uint32_t ptype = f->kind == OR_STRUCT ? f->type : 0;
      int64_t seen = map_find(c, p);
      if (seen >= 0) {
        const or_object* s = &c->objs[seen];
        if (s->kind != f->kind || s->type != ptype || s->count != count) return OR_E_CONFLICT;
        continue;
      }
      uint64_t child;
      rc = push_object(c, p, f->kind, ptype, count, &child);
      if (rc) return rc;
      rc = visit(c, child);
      if (rc) return rc;
    }
  }
  return OR_OK;
}

static int cmp_host(const void* a, const void* b) {
  const or_object* x = *(const or_object* const*)a;
  const or_object* y = *(const or_object* const*)b;
  return x->host < y->host ? -1 : x->host > y->host;
}

/* Two objects whose host ranges overlap mean some pointer points into the
 * middle of another array; the deep copy rejects that. */
static int check_no_overlap(const or_copy* c) {
  if (c->nobjs < 2) return OR_OK;
  const or_object** v = (const or_object**)malloc(c->nobjs * sizeof(*v));
  if (!v) return OR_E_NOMEM;
  for (uint64_t i = 0; i < c->nobjs; i++) v[i] = &c->objs[i];
  qsort(v, c->nobjs, sizeof(*v), cmp_host);
  int rc = OR_OK;
  for (uint64_t i = 0; i + 1 < c->nobjs; i++) {
    uint64_t extent = v[i]->bytes ? v[i]->bytes : 1;
    if (v[i]->host + extent > v[i + 1]->host) {
      rc = OR_E_RANGE;
      break;
    }
  }
  free(v);
  return rc;
}

int or_deep_copy(const or_type* types, uint32_t ntypes, uint32_t root_type, void* const* roots, uint64_t nroots,
                 uint64_t align, uint64_t base, or_copy** out) {
  return or_deep_copy_selective(types, ntypes, root_type, roots, nroots, align, base, NULL, out);
}

int or_deep_copy_selective(const or_type* types, uint32_t ntypes, uint32_t root_type, void* const* roots,
                           uint64_t nroots, uint64_t align, uint64_t base, const uint32_t* follow, or_copy** out) {
  *out = NULL;
  if (!types || ntypes == 0 || root_type >= ntypes || (!roots && nroots)) return OR_E_INVAL;
  if (align == 0 || (align & (align - 1))) return OR_E_INVAL;
  for (uint32_t i = 0; i < ntypes; i++) {
    if (types[i].nfields > OR_MAX_FIELDS) return OR_E_INVAL;
    for (uint32_t j = 0; j < types[i].nfields; j++) {
      const or_field* f = &types[i].fields[j];
      if (f->kind > OR_U8 || (f->kind == OR_STRUCT && f->type >= ntypes)) return OR_E_INVAL;
      if (f->offset + 8 > types[i].size) return OR_E_INVAL;
    }
  }
  or_copy* c = (or_copy*)calloc(1, sizeof(or_copy));
  if (!c) return OR_E_NOMEM;
  or_type* tcopy = (or_type*)malloc(ntypes * sizeof(or_type));
  c->root_obj = (uint64_t*)malloc((nroots ? nroots : 1) * sizeof(uint64_t));
  c->keys = (uint64_t*)calloc(64, sizeof(uint64_t));
  c->vals = (uint64_t*)calloc(64, sizeof(uint64_t));
  if (!tcopy || !c->root_obj || !c->keys || !c->vals) {
    free(tcopy);
    or_free(c);
    return OR_E_NOMEM;
  }
  memcpy(tcopy, types, ntypes * sizeof(or_type));
  c->types = tcopy;
  c->follow = (uint32_t*)malloc(ntypes * sizeof(uint32_t));
  if (!c->follow) {
    or_free(c);
    return OR_E_NOMEM;
  }
  for (uint32_t i = 0; i < ntypes; i++) c->follow[i] = follow ? follow[i] : 0xFFFFFFFFu;
  c->ntypes = ntypes;
  c->mask = 63;
  c->align = align;
  c->base = base;
  c->roots = roots;
  c->nroots = nroots;

  /* a) walk every root in order */
  int rc = OR_OK;
  for (uint64_t r = 0; r < nroots && rc == OR_OK; r++) {
    uint64_t p = (uint64_t)(uintptr_t)roots[r];
    if (p == 0) {
      rc = OR_E_INVAL;
      break;
    }
    int64_t seen = map_find(c, p);
    if (seen >= 0) {
      if (c->objs[seen].kind != OR_STRUCT || c->objs[seen].type != root_type || c->objs[seen].count != 1)
        rc = OR_E_CONFLICT;
      c->root_obj[r] = (uint64_t)seen;
      continue;
    }
    uint64_t idx;
    rc = push_object(c, p, OR_STRUCT, root_type, 1, &idx);
    if (rc == OR_OK) {
      c->root_obj[r] = idx;
      rc = visit(c, idx);
    }
  }
  if (rc == OR_OK) rc = check_no_overlap(c);
  if (rc) {
    or_free(c);
    return rc;
  }

  /* b) layout in visiting order */
  uint64_t end = 0;
  for (uint64_t i = 0; i < c->nobjs; i++) {
    c->objs[i].off = i == 0 ? 0 : align_up(end, align);
    end = c->objs[i].off + (c->objs[i].bytes ? c->objs[i].bytes : 1);
  }
  c->arena_bytes = c->nobjs ? align_up(end, align) : 0;

  /* c) copy: zeroed buffer, then each object's bytes */
  c->arena = (uint8_t*)calloc(c->arena_bytes ? c->arena_bytes : 1, 1);
  if (!c->arena) {
    or_free(c);
    return OR_E_NOMEM;
  }
  for (uint64_t i = 0; i < c->nobjs; i++)
    if (c->objs[i].bytes) memcpy(c->arena + c->objs[i].off, (const void*)(uintptr_t)c->objs[i].host, c->objs[i].bytes);

  /* d) relocate every pointer slot of every struct element */
  for (uint64_t i = 0; i < c->nobjs; i++) {
    const or_object* o = &c->objs[i];
    if (o->kind != OR_STRUCT) continue;
    const or_type* t = &c->types[o->type];
    for (uint64_t e = 0; e < o->count; e++) {
      uint8_t* elem = c->arena + o->off + e * t->size;
      for (uint32_t k = 0; k < t->nfields; k++) {
        uint64_t p;
        memcpy(&p, elem + t->fields[k].offset, 8);
        if (p == 0) continue;
        if (!((c->follow[o->type] >> k) & 1u)) {
          /* an unfollowed member reads as null in the copy */
          memset(elem + t->fields[k].offset, 0, 8);
          continue;
        }
        int64_t j = map_find(c, p);
        if (j < 0) {
          or_free(c);
          return OR_E_RANGE;
        }
        uint64_t q = base + c->objs[j].off;
        memcpy(elem + t->fields[k].offset, &q, 8);
        c->nslots++;
      }
    }
  }
  *out = c;
  return OR_OK;
}

void or_free(or_copy* c) {
  if (!c) return;
  free((void*)c->types);
  free(c->follow);
  free(c->root_obj);
  free(c->objs);
  free(c->keys);
  free(c->vals);
  free(c->arena);
  free(c);
}

uint8_t* or_arena(const or_copy* c) { return c->arena; }
uint64_t or_arena_bytes(const or_copy* c) { return c->arena_bytes; }
uint64_t or_nobjects(const or_copy* c) { return c->nobjs; }
const or_object* or_objects(const or_copy* c) { return c->objs; }
uint64_t or_nslots(const or_copy* c) { return c->nslots; }
uint64_t or_payload_bytes(const or_copy* c) {
  uint64_t s = 0;
  for (uint64_t i = 0; i < c->nobjs; i++) s += c->objs[i].bytes;
  return s;
}

/* object whose buffer offset is exactly `off` (objects are in increasing
 * offset order), or -1 */
static int64_t object_at(const or_copy* c, uint64_t off) {
  uint64_t lo = 0, hi = c->nobjs;
  while (lo < hi) {
    uint64_t mid = (lo + hi) / 2;
    if (c->objs[mid].off < off) lo = mid + 1;
    else hi = mid;
  }
  /* several zero-byte objects cannot share an offset, so the match is unique */
  if (lo < c->nobjs && c->objs[lo].off == off) return (int64_t)lo;
  return -1;
}

int or_resolve_chain(const or_copy* c, uint64_t root_index, const uint32_t* fields, const uint64_t* index,
                     uint32_t nsteps, uint64_t* addr, uint64_t* count, uint32_t* kind) {
  if (root_index >= c->nroots || nsteps == 0) return OR_E_INVAL;
  const or_object* cur = &c->objs[c->root_obj[root_index]];
  uint64_t elem = 0;
  for (uint32_t s = 0; s < nsteps; s++) {
    if (cur->kind != OR_STRUCT) return OR_E_INVAL;
    const or_type* t = &c->types[cur->type];
    if (fields[s] >= t->nfields) return OR_E_INVAL;
    const or_field* f = &t->fields[fields[s]];
    const uint8_t* e = c->arena + cur->off + elem * t->size;
    uint64_t p;
    memcpy(&p, e + f->offset, 8);
    if (p == 0) return OR_E_RANGE;
    uint64_t n;
    int rc = field_count(f, e, &n);
    if (rc) return rc;
    if (s + 1 == nsteps) {
      *addr = p;
      *count = n;
      *kind = f->kind;
      return OR_OK;
    }
    int64_t j = object_at(c, p - c->base);
    if (j < 0) return OR_E_RANGE;
    if (index[s] >= n) return OR_E_RANGE;
    cur = &c->objs[j];
    elem = index[s];
  }
  return OR_E_INVAL;
}

/* A scalar member reached through a chain (Section 3, scalar variables):
 * every step reads a pointer member and moves to element index[s] of the
 * struct array it points to; the scalar is `bytes` bytes at `offset` of the
 * element the last step lands on (of the root itself when nsteps is 0). */
int or_scalar_chain(const or_copy* c, uint64_t root_index, const uint32_t* fields, const uint64_t* index,
                    uint32_t nsteps, uint32_t offset, uint32_t bytes, uint64_t* addr) {
  if (root_index >= c->nroots) return OR_E_INVAL;
  if (bytes != 1 && bytes != 4 && bytes != 8) return OR_E_INVAL;
  const or_object* cur = &c->objs[c->root_obj[root_index]];
  uint64_t elem = 0;
  for (uint32_t s = 0; s < nsteps; s++) {
    const or_type* t = &c->types[cur->type];
    if (fields[s] >= t->nfields) return OR_E_INVAL;
    const or_field* f = &t->fields[fields[s]];
    if (f->kind != OR_STRUCT) return OR_E_INVAL;
    const uint8_t* e = c->arena + cur->off + elem * t->size;
    uint64_t p;
    memcpy(&p, e + f->offset, 8);
    if (p == 0) return OR_E_RANGE;
    uint64_t n;
    int rc = field_count(f, e, &n);
    if (rc) return rc;
    if (index[s] >= n) return OR_E_RANGE;
    int64_t j = object_at(c, p - c->base);
    if (j < 0) return OR_E_RANGE;
    cur = &c->objs[j];
    elem = index[s];
  }
  const or_type* t = &c->types[cur->type];
  if ((uint64_t)offset + bytes > t->size) return OR_E_RANGE;
  *addr = c->base + cur->off + elem * t->size + offset;
  return OR_OK;
}

double or_fma64(double x, double a, double b) { return fma(x, a, b); }
float or_fma32(float x, float a, float b) { return fmaf(x, a, b); }

static void kernel_leaf(uint8_t* src, uint8_t* dst, const or_object* o, uint32_t iters, double a, double b,
                        float af, float bf) {
  if (o->kind == OR_F64) {
    for (uint64_t i = 0; i < o->count; i++) {
      double x;
      memcpy(&x, src + 8 * i, 8);
      for (uint32_t it = 0; it < iters; it++) x = fma(x, a, b);
      memcpy(dst + 8 * i, &x, 8);
    }
  } else if (o->kind == OR_F32) {
    for (uint64_t i = 0; i < o->count; i++) {
      float x;
      memcpy(&x, src + 4 * i, 4);
      for (uint32_t it = 0; it < iters; it++) x = fmaf(x, af, bf);
      memcpy(dst + 4 * i, &x, 4);
    }
  }
}

/* the selected leaves: the chain's target, or every FP32/FP64 object */
static int select_leaves(const or_copy* c, int select, uint64_t root_index, const uint32_t* fields,
                         const uint64_t* index, uint32_t nsteps, int64_t* chain_obj) {
  *chain_obj = -1;
  if (select == 1) return OR_OK;
  if (select != 0) return OR_E_INVAL;
  uint64_t addr, count;
  uint32_t kind;
  int rc = or_resolve_chain(c, root_index, fields, index, nsteps, &addr, &count, &kind);
  if (rc) return rc;
  if (kind != OR_F32 && kind != OR_F64) return OR_E_INVAL;
  int64_t j = object_at(c, addr - c->base);
  if (j < 0) return OR_E_RANGE;
  *chain_obj = j;
  return OR_OK;
}

static int is_selected(const or_copy* c, uint64_t i, int64_t chain_obj) {
  if (chain_obj >= 0) return (int64_t)i == chain_obj;
  return c->objs[i].kind == OR_F32 || c->objs[i].kind == OR_F64;
}

uint64_t or_out_bytes(const or_copy* c, int select, uint64_t root_index, const uint32_t* fields,
                      const uint64_t* index, uint32_t nsteps) {
  int64_t chain_obj;
  if (select_leaves(c, select, root_index, fields, index, nsteps, &chain_obj)) return 0;
  uint64_t end = 0;
  int first = 1;
  for (uint64_t i = 0; i < c->nobjs; i++) {
    if (!is_selected(c, i, chain_obj)) continue;
    uint64_t off = first ? 0 : align_up(end, c->align);
    first = 0;
    end = off + (c->objs[i].bytes ? c->objs[i].bytes : 1);
  }
  return first ? 0 : align_up(end, c->align);
}

int or_run_kernel(or_copy* c, int select, uint64_t root_index, const uint32_t* fields, const uint64_t* index,
                  uint32_t nsteps, uint32_t iters, double a, double b, float af, float bf, uint8_t* out,
                  uint64_t out_bytes) {
  int64_t chain_obj;
  int rc = select_leaves(c, select, root_index, fields, index, nsteps, &chain_obj);
  if (rc) return rc;
  if (out && out_bytes < or_out_bytes(c, select, root_index, fields, index, nsteps)) return OR_E_RANGE;
  uint64_t end = 0;
  int first = 1;
  for (uint64_t i = 0; i < c->nobjs; i++) {
    if (!is_selected(c, i, chain_obj)) continue;
    const or_object* o = &c->objs[i];
    uint8_t* src = c->arena + o->off;
    uint8_t* dst = src;
    if (out) {
      uint64_t off = first ? 0 : align_up(end, c->align);
      end = off + (o->bytes ? o->bytes : 1);
      dst = out + off;
    }
    first = 0;
    kernel_leaf(src, dst, o, iters, a, b, af, bf);
  }
  return OR_OK;
}

/* The molecular-dynamics update of every element of struct type `type`
 * (the paper's Listing of atoms in cells; a velocity-Verlet style kick then
 * drift per time step, forces held fixed): for each of the element's count
 * entries,
 *   v <- fma(f, dt_over_m, v)     (kick)
 *   x <- fma(v, dt, x)            (drift, with the kicked v)
 * in binary64 with one rounding per fma. x, v and f are the arrays that pointer
 * fields xf, vf and ff of the element point to; they must have equal counts,
 * be all null or all non-null, and no array may belong to two elements or two
 * roles. */
int or_kick_drift(or_copy* c, uint32_t type, uint32_t xf, uint32_t vf, uint32_t ff, uint32_t steps, double dt,
                  double dt_over_m) {
  if (type >= c->ntypes) return OR_E_INVAL;
  const or_type* t = &c->types[type];
  if (xf >= t->nfields || vf >= t->nfields || ff >= t->nfields) return OR_E_INVAL;
  if (xf == vf || xf == ff || vf == ff) return OR_E_INVAL;
  const uint32_t fl[3] = {xf, vf, ff};
  for (int r = 0; r < 3; r++)
    if (t->fields[fl[r]].kind != OR_F64) return OR_E_INVAL;
  uint8_t* used = calloc(c->nobjs ? c->nobjs : 1, 1);
  if (!used) return OR_E_NOMEM;
  int rc = OR_OK;
  /* validation pass: every element's three arrays */
  for (uint64_t i = 0; i < c->nobjs && rc == OR_OK; i++) {
    const or_object* o = &c->objs[i];
    if (o->kind != OR_STRUCT || o->type != type) continue;
    for (uint64_t e = 0; e < o->count && rc == OR_OK; e++) {
      const uint8_t* el = c->arena + o->off + e * t->size;
      uint64_t p[3], n[3];
      int nnull = 0;
      for (int r = 0; r < 3 && rc == OR_OK; r++) {
        memcpy(&p[r], el + t->fields[fl[r]].offset, 8);
        rc = field_count(&t->fields[fl[r]], el, &n[r]);
        nnull += p[r] == 0;
      }
      if (rc) break;
      if (nnull == 3) continue;
      if (nnull != 0 || n[0] != n[1] || n[0] != n[2]) {
        rc = OR_E_INVAL;
        break;
      }
      for (int r = 0; r < 3; r++) {
        int64_t j = object_at(c, p[r] - c->base);
        if (j < 0) {
          rc = OR_E_RANGE;
          break;
        }
        if (used[j]) {
          rc = OR_E_CONFLICT;
          break;
        }
        used[j] = 1;
      }
    }
  }
  free(used);
  if (rc) return rc;
  for (uint32_t s = 0; s < steps; s++) {
    for (uint64_t i = 0; i < c->nobjs; i++) {
      const or_object* o = &c->objs[i];
      if (o->kind != OR_STRUCT || o->type != type) continue;
      for (uint64_t e = 0; e < o->count; e++) {
        const uint8_t* el = c->arena + o->off + e * t->size;
        uint64_t px, pv, pf, n = 0;
        memcpy(&px, el + t->fields[xf].offset, 8);
        memcpy(&pv, el + t->fields[vf].offset, 8);
        memcpy(&pf, el + t->fields[ff].offset, 8);
        if (px == 0) continue;
        field_count(&t->fields[xf], el, &n);
        uint8_t* X = c->arena + (px - c->base);
        uint8_t* V = c->arena + (pv - c->base);
        const uint8_t* F = c->arena + (pf - c->base);
        for (uint64_t k = 0; k < n; k++) {
          double x, v, f;
          memcpy(&x, X + 8 * k, 8);
          memcpy(&v, V + 8 * k, 8);
          memcpy(&f, F + 8 * k, 8);
          v = fma(f, dt_over_m, v);
          x = fma(v, dt, x);
          memcpy(V + 8 * k, &v, 8);
          memcpy(X + 8 * k, &x, 8);
        }
      }
    }
  }
  return OR_OK;
}

int or_copy_back(const or_copy* c, int scalars) {
  for (uint64_t i = 0; i < c->nobjs; i++) {
    const or_object* o = &c->objs[i];
    uint8_t* host = (uint8_t*)(uintptr_t)o->host;
    if (o->kind != OR_STRUCT) {
      if (o->bytes) memcpy(host, c->arena + o->off, o->bytes);
      continue;
    }
    if (!scalars) continue;
    const or_type* t = &c->types[o->type];
    for (uint64_t e = 0; e < o->count; e++) {
      const uint8_t* src = c->arena + o->off + e * t->size;
      uint8_t* dst = host + e * t->size;
      for (uint32_t byte = 0; byte < t->size; byte++) {
        int in_pointer = 0;
        for (uint32_t k = 0; k < t->nfields; k++)
          if (byte >= t->fields[k].offset && byte < t->fields[k].offset + 8) in_pointer = 1;
        if (!in_pointer) dst[byte] = src[byte];
      }
    }
  }
  return OR_OK;
}
