/* Seeded synthetic input trees (see fx.h). Inputs only: nothing here walks,
 * lays out, relocates or computes on a tree. */
#include "fx.h"

#include <math.h>
#include <pthread.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ---- random numbers: SplitMix64 seeding xoshiro256** (Blackman & Vigna) ---- */

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64(uint64_t* x) {
  uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static void rng_seed(rng_t* r, uint64_t seed) {
  uint64_t x = seed;
  for (int i = 0; i < 4; i++) r->s[i] = splitmix64(&x);
}

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static inline uint64_t rng_next(rng_t* r) {
  uint64_t* s = r->s;
  uint64_t result = rotl(s[1] * 5, 7) * 9;
  uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl(s[3], 45);
  return result;
}

/* uniform [0,1) with 53 random bits */
static inline double rng_unit(rng_t* r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }
/* uniform [-1,1): 2u-1 is exact in binary64 */
static inline double rng_f64(rng_t* r) { return 2.0 * rng_unit(r) - 1.0; }
/* uniform [-1,1) with 24 random bits, exact in binary32 */
static inline float rng_f32(rng_t* r) {
  float u = (float)(rng_next(r) >> 40) * 0x1.0p-24f;
  return 2.0f * u - 1.0f;
}
/* integer uniform in [lo, hi] */
static inline int64_t rng_int(rng_t* r, int64_t lo, int64_t hi) {
  uint64_t span = (uint64_t)(hi - lo) + 1;
  return lo + (int64_t)(((unsigned __int128)rng_next(r) * span) >> 64);
}
/* Poisson(mean) by Knuth's product-of-uniforms method */
static int64_t rng_poisson(rng_t* r, double mean) {
  double L = exp(-mean), p = 1.0;
  int64_t k = 0;
  do {
    k++;
    p *= rng_unit(r);
  } while (p > L);
  return k - 1;
}

void fx_fill_f64(double* x, uint64_t n, uint64_t seed) {
  rng_t r;
  rng_seed(&r, seed);
  for (uint64_t i = 0; i < n; i++) x[i] = rng_f64(&r);
}

void fx_fill_f32(float* x, uint64_t n, uint64_t seed) {
  rng_t r;
  rng_seed(&r, seed);
  for (uint64_t i = 0; i < n; i++) x[i] = rng_f32(&r);
}

static int g_threads = 0;
void fx_set_threads(int n) { g_threads = n; }

/* ---- allocation bookkeeping ---- */

static int track(fx_tree* t, void* p, uint64_t bytes, uint32_t kind) {
  if (!p) return -1;
  if (t->nallocs == t->cap_allocs) {
    uint64_t nc = t->cap_allocs ? 2 * t->cap_allocs : 1024;
    fx_alloc* a = (fx_alloc*)realloc(t->allocs, nc * sizeof(fx_alloc));
    if (!a) return -1;
    t->allocs = a;
    t->cap_allocs = nc;
  }
  fx_alloc* a = &t->allocs[t->nallocs++];
  a->base = p;
  a->bytes = bytes;
  a->kind = kind;
  a->pad = 0;
  return 0;
}

/* malloc that never returns NULL for zero bytes, so a zero-length array still
 * has a distinct address */
static void* fx_malloc(uint64_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  return p;
}

static void* alloc_tracked(fx_tree* t, uint64_t bytes, uint32_t kind) {
  void* p = fx_malloc(bytes);
  if (!p) return NULL;
  if (track(t, p, bytes, kind)) {
    free(p);
    return NULL;
  }
  return p;
}

static double* new_f64(fx_tree* t, rng_t* r, uint64_t n) {
  double* x = (double*)alloc_tracked(t, n * 8, FX_F64);
  if (!x) return NULL;
  for (uint64_t i = 0; i < n; i++) x[i] = rng_f64(r);
  return x;
}

static float* new_f32(fx_tree* t, rng_t* r, uint64_t n) {
  float* x = (float*)alloc_tracked(t, n * 4, FX_F32);
  if (!x) return NULL;
  for (uint64_t i = 0; i < n; i++) x[i] = rng_f32(r);
  return x;
}

static void* new_structs(fx_tree* t, uint64_t n, uint32_t size) {
  void* p = alloc_tracked(t, (uint64_t)n * size, FX_STRUCT);
  if (p) memset(p, 0, n ? (size_t)n * size : 1);
  return p;
}

static void set_type(fx_type* ty, const char* name, uint32_t size, uint32_t align) {
  memset(ty, 0, sizeof(*ty));
  strncpy(ty->name, name, sizeof(ty->name) - 1);
  ty->size = size;
  ty->align = align;
}

static void add_field(fx_type* ty, uint32_t offset, uint32_t kind, uint32_t type, int32_t count_offset,
                      uint32_t count_bytes, uint32_t count_mult, uint64_t fixed_count) {
  fx_field* f = &ty->fields[ty->nfields++];
  f->offset = offset;
  f->kind = kind;
  f->type = type;
  f->count_offset = count_offset;
  f->count_bytes = count_bytes;
  f->count_mult = count_mult;
  f->fixed_count = fixed_count;
}

/* ---- shape: plain (root -> array of children -> one leaf each) ---- */

typedef struct { int64_t n; struct PChild* c; } PRoot;
typedef struct PChild { int64_t n; double* leaf; } PChild;

static int build_plain(fx_tree* t, rng_t* r, const int64_t* p) {
  int64_t nchild = p[0], len = p[1];
  if (nchild < 0 || len < 0) return -1;
  set_type(&t->types[0], "Root", sizeof(PRoot), 8);
  add_field(&t->types[0], offsetof(PRoot, c), FX_STRUCT, 1, offsetof(PRoot, n), 8, 1, 0);
  set_type(&t->types[1], "Child", sizeof(PChild), 8);
  add_field(&t->types[1], offsetof(PChild, leaf), FX_F64, 0, offsetof(PChild, n), 8, 1, 0);
  t->ntypes = 2;
  t->root_type = 0;
  PRoot* root = (PRoot*)new_structs(t, 1, sizeof(PRoot));
  if (!root) return -1;
  root->n = nchild;
  root->c = (PChild*)new_structs(t, (uint64_t)nchild, sizeof(PChild));
  if (!root->c) return -1;
  for (int64_t i = 0; i < nchild; i++) {
    root->c[i].n = len;
    root->c[i].leaf = new_f64(t, r, (uint64_t)len);
    if (!root->c[i].leaf) return -1;
  }
  t->nroots = 1;
  t->roots = (void**)malloc(sizeof(void*));
  t->roots[0] = root;
  return 0;
}

/* ---- shape: Linear (Section 4.1): k nodes, payload A of n doubles ---- */

typedef struct LNode { int32_t nA; int32_t nLnext; double* A; struct LNode* Lnext; } LNode;

static int build_linear(fx_tree* t, rng_t* r, const int64_t* p) {
  int64_t k = p[0], n = p[1], scheme = p[2];
  if (k < 1 || n < 0 || n > INT32_MAX) return -1;
  set_type(&t->types[0], "L", sizeof(LNode), 8);
  add_field(&t->types[0], offsetof(LNode, A), FX_F64, 0, offsetof(LNode, nA), 4, 1, 0);
  add_field(&t->types[0], offsetof(LNode, Lnext), FX_STRUCT, 0, offsetof(LNode, nLnext), 4, 1, 0);
  t->ntypes = 1;
  t->root_type = 0;
  LNode* prev = NULL;
  LNode* root = NULL;
  for (int64_t i = 0; i < k; i++) {
    LNode* node = (LNode*)new_structs(t, 1, sizeof(LNode));
    if (!node) return -1;
    int alloc = (scheme == 0) || (i == k - 1);
    node->nA = alloc ? (int32_t)n : 0;
    node->A = alloc ? new_f64(t, r, (uint64_t)n) : NULL;
    if (alloc && !node->A) return -1;
    node->nLnext = 0;
    node->Lnext = NULL;
    if (prev) {
      prev->Lnext = node;
      prev->nLnext = 1;
    } else {
      root = node;
    }
    prev = node;
  }
  t->nroots = 1;
  t->roots = (void**)malloc(sizeof(void*));
  t->roots[0] = root;
  return 0;
}

/* ---- shape: Dense (Section 4.2): next pointer is an array of q nodes ---- */

typedef struct DNode { int32_t nA; int32_t nLnext; double* A; struct DNode* Lnext; } DNode;
/* last level: 12 bytes as the paper counts it (packed) or 16 bytes aligned */
typedef struct __attribute__((packed)) { int32_t nA; double* A; } DLastPacked;
typedef struct { int32_t nA; double* A; } DLast;

static int dense_fill(fx_tree* t, rng_t* r, void* node, int level, int64_t q, int64_t n, int64_t D,
                      int packed) {
  if (level < D) {
    DNode* d = (DNode*)node;
    d->nA = (int32_t)n;
    d->A = new_f64(t, r, (uint64_t)n);
    if (!d->A) return -1;
    d->nLnext = (int32_t)q;
    uint32_t csize = (level + 1 < D) ? (uint32_t)sizeof(DNode)
                                     : (packed ? (uint32_t)sizeof(DLastPacked) : (uint32_t)sizeof(DLast));
    char* kids = (char*)new_structs(t, (uint64_t)q, csize);
    if (!kids) return -1;
    d->Lnext = (DNode*)kids;
    for (int64_t i = 0; i < q; i++)
      if (dense_fill(t, r, kids + (size_t)i * csize, level + 1, q, n, D, packed)) return -1;
  } else if (packed) {
    DLastPacked* l = (DLastPacked*)node;
    l->nA = (int32_t)n;
    double* a = new_f64(t, r, (uint64_t)n);
    if (!a) return -1;
    memcpy((char*)l + offsetof(DLastPacked, A), &a, sizeof(a));
  } else {
    DLast* l = (DLast*)node;
    l->nA = (int32_t)n;
    l->A = new_f64(t, r, (uint64_t)n);
    if (!l->A) return -1;
  }
  return 0;
}

static int build_dense(fx_tree* t, rng_t* r, const int64_t* p) {
  int64_t q = p[0], n = p[1], D = p[2], packed = p[3];
  if (q < 1 || n < 0 || D < 1 || D > 6) return -1;
  /* one type per level so the last level can use its own struct */
  for (int64_t lv = 0; lv < D; lv++) {
    char nm[16] = "L0";
    nm[1] = (char)('0' + lv);
    set_type(&t->types[lv], nm, sizeof(DNode), 8);
    add_field(&t->types[lv], offsetof(DNode, A), FX_F64, 0, offsetof(DNode, nA), 4, 1, 0);
    add_field(&t->types[lv], offsetof(DNode, Lnext), FX_STRUCT, (uint32_t)(lv + 1), offsetof(DNode, nLnext), 4,
              1, 0);
  }
  char nm[16] = "L0";
  nm[1] = (char)('0' + D);
  if (packed) {
    set_type(&t->types[D], nm, sizeof(DLastPacked), 1);
    add_field(&t->types[D], offsetof(DLastPacked, A), FX_F64, 0, offsetof(DLastPacked, nA), 4, 1, 0);
  } else {
    set_type(&t->types[D], nm, sizeof(DLast), 8);
    add_field(&t->types[D], offsetof(DLast, A), FX_F64, 0, offsetof(DLast, nA), 4, 1, 0);
  }
  t->ntypes = (uint32_t)D + 1;
  t->root_type = 0;
  DNode* root = (DNode*)new_structs(t, 1, sizeof(DNode));
  if (!root) return -1;
  if (dense_fill(t, r, root, 0, q, n, D, (int)packed)) return -1;
  t->nroots = 1;
  t->roots = (void**)malloc(sizeof(void*));
  t->roots[0] = root;
  return 0;
}

/* ---- shape: wide tree, leaves of log-uniform length, half FP32 half FP64 ---- */

typedef struct { int64_t n; struct WMid* mid; } WRoot;
typedef struct WMid { int64_t n; struct WLeaf* leaves; } WMid;
typedef struct WLeaf { int64_t n; float* f32; double* f64; } WLeaf;

static int build_wide(fx_tree* t, rng_t* r, const int64_t* p) {
  int64_t f1 = p[0], f2 = p[1], lo = p[2], hi = p[3];
  if (f1 < 0 || f2 < 0 || lo < 1 || hi < lo) return -1;
  set_type(&t->types[0], "WRoot", sizeof(WRoot), 8);
  add_field(&t->types[0], offsetof(WRoot, mid), FX_STRUCT, 1, offsetof(WRoot, n), 8, 1, 0);
  set_type(&t->types[1], "WMid", sizeof(WMid), 8);
  add_field(&t->types[1], offsetof(WMid, leaves), FX_STRUCT, 2, offsetof(WMid, n), 8, 1, 0);
  set_type(&t->types[2], "WLeaf", sizeof(WLeaf), 8);
  add_field(&t->types[2], offsetof(WLeaf, f32), FX_F32, 0, offsetof(WLeaf, n), 8, 1, 0);
  add_field(&t->types[2], offsetof(WLeaf, f64), FX_F64, 0, offsetof(WLeaf, n), 8, 1, 0);
  t->ntypes = 3;
  t->root_type = 0;
  WRoot* root = (WRoot*)new_structs(t, 1, sizeof(WRoot));
  if (!root) return -1;
  root->n = f1;
  root->mid = (WMid*)new_structs(t, (uint64_t)f1, sizeof(WMid));
  if (!root->mid) return -1;
  double ratio = log2((double)hi / (double)lo);
  int64_t j = 0;
  for (int64_t a = 0; a < f1; a++) {
    WMid* m = &root->mid[a];
    m->n = f2;
    m->leaves = (WLeaf*)new_structs(t, (uint64_t)f2, sizeof(WLeaf));
    if (!m->leaves) return -1;
    for (int64_t b = 0; b < f2; b++, j++) {
      int64_t len = (int64_t)floor((double)lo * exp2(ratio * rng_unit(r)));
      if (len > hi) len = hi;
      WLeaf* l = &m->leaves[b];
      l->n = len;
      if ((j & 1) == 0) {
        l->f32 = new_f32(t, r, (uint64_t)len);
        if (!l->f32) return -1;
      } else {
        l->f64 = new_f64(t, r, (uint64_t)len);
        if (!l->f64) return -1;
      }
    }
  }
  t->nroots = 1;
  t->roots = (void**)malloc(sizeof(void*));
  t->roots[0] = root;
  return 0;
}

/* ---- shape: molecular dynamics, many independent simulations ---- */

typedef struct { int64_t ncells; struct MCell* cells; } MSim;
typedef struct MCell { int64_t natoms; double* pos; double* vel; double* force; } MCell;

typedef struct {
  fx_tree* t;
  uint64_t seed;
  int64_t lo, hi;
  double mean;
  int64_t begin, end;
  fx_tree local; /* per-thread allocation list, merged afterwards */
  int err;
} md_job;

static void* md_worker(void* arg) {
  md_job* J = (md_job*)arg;
  for (int64_t s = J->begin; s < J->end; s++) {
    rng_t r;
    /* each simulation draws from its own stream, so the tree does not depend
     * on how simulations are split among threads */
    rng_seed(&r, J->seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(s + 1)));
    MSim* sim = (MSim*)new_structs(&J->local, 1, sizeof(MSim));
    if (!sim) { J->err = 1; return NULL; }
    int64_t nc = rng_int(&r, J->lo, J->hi);
    sim->ncells = nc;
    sim->cells = (MCell*)new_structs(&J->local, (uint64_t)nc, sizeof(MCell));
    if (!sim->cells) { J->err = 1; return NULL; }
    for (int64_t c = 0; c < nc; c++) {
      MCell* cell = &sim->cells[c];
      int64_t na = rng_poisson(&r, J->mean);
      cell->natoms = na;
      cell->pos = new_f64(&J->local, &r, (uint64_t)(3 * na));
      cell->vel = new_f64(&J->local, &r, (uint64_t)(3 * na));
      cell->force = new_f64(&J->local, &r, (uint64_t)(3 * na));
      if (!cell->pos || !cell->vel || !cell->force) { J->err = 1; return NULL; }
    }
    J->t->roots[s] = sim;
  }
  return NULL;
}

static int build_md(fx_tree* t, uint64_t seed, const int64_t* p) {
  int64_t nsims = p[0], lo = p[1], hi = p[2], mean = p[3];
  if (nsims < 0 || lo < 0 || hi < lo || mean < 0) return -1;
  set_type(&t->types[0], "Sim", sizeof(MSim), 8);
  add_field(&t->types[0], offsetof(MSim, cells), FX_STRUCT, 1, offsetof(MSim, ncells), 8, 1, 0);
  set_type(&t->types[1], "Cell", sizeof(MCell), 8);
  add_field(&t->types[1], offsetof(MCell, pos), FX_F64, 0, offsetof(MCell, natoms), 8, 3, 0);
  add_field(&t->types[1], offsetof(MCell, vel), FX_F64, 0, offsetof(MCell, natoms), 8, 3, 0);
  add_field(&t->types[1], offsetof(MCell, force), FX_F64, 0, offsetof(MCell, natoms), 8, 3, 0);
  t->ntypes = 2;
  t->root_type = 0;
  t->nroots = (uint64_t)nsims;
  t->roots = (void**)calloc(nsims ? (size_t)nsims : 1, sizeof(void*));
  if (!t->roots) return -1;
  int nth = g_threads > 0 ? g_threads : (int)sysconf(_SC_NPROCESSORS_ONLN);
  if (nth < 1) nth = 1;
  if (nth > 64) nth = 64;
  if (nsims < nth * 4) nth = 1;
  md_job jobs[64];
  pthread_t th[64];
  memset(jobs, 0, sizeof(jobs));
  for (int i = 0; i < nth; i++) {
    jobs[i].t = t;
    jobs[i].seed = seed;
    jobs[i].lo = lo;
    jobs[i].hi = hi;
    jobs[i].mean = (double)mean;
    jobs[i].begin = nsims * i / nth;
    jobs[i].end = nsims * (i + 1) / nth;
  }
  for (int i = 1; i < nth; i++) pthread_create(&th[i], NULL, md_worker, &jobs[i]);
  md_worker(&jobs[0]);
  for (int i = 1; i < nth; i++) pthread_join(th[i], NULL);
  int err = 0;
  for (int i = 0; i < nth; i++) {
    err |= jobs[i].err;
    for (uint64_t k = 0; k < jobs[i].local.nallocs; k++) {
      fx_alloc* a = &jobs[i].local.allocs[k];
      if (!err && track(t, a->base, a->bytes, a->kind)) err = 1;
      else if (err) free(a->base);
    }
    free(jobs[i].local.allocs);
  }
  return err ? -1 : 0;
}

/* ---- shape: broom, one served job (chain of nodes, then f leaves) ---- */

typedef struct BNode { int64_t nleaves; struct BNode* next; struct BLeaf* leaves; } BNode;
typedef struct BLeaf { int64_t n; float* f32; double* f64; } BLeaf;

static int build_broom(fx_tree* t, rng_t* r, const int64_t* p) {
  int64_t dlo = p[0], dhi = p[1], flo = p[2], fhi = p[3], blo = p[4], bhi = p[5];
  if (dlo < 2 || dhi < dlo || flo < 1 || fhi < flo || blo < 8 || bhi < blo) return -1;
  set_type(&t->types[0], "Node", sizeof(BNode), 8);
  add_field(&t->types[0], offsetof(BNode, next), FX_STRUCT, 0, -1, 8, 1, 1);
  add_field(&t->types[0], offsetof(BNode, leaves), FX_STRUCT, 1, offsetof(BNode, nleaves), 8, 1, 0);
  set_type(&t->types[1], "Leaf", sizeof(BLeaf), 8);
  add_field(&t->types[1], offsetof(BLeaf, f32), FX_F32, 0, offsetof(BLeaf, n), 8, 1, 0);
  add_field(&t->types[1], offsetof(BLeaf, f64), FX_F64, 0, offsetof(BLeaf, n), 8, 1, 0);
  t->ntypes = 2;
  t->root_type = 0;
  int64_t d = rng_int(r, dlo, dhi);
  int64_t f = rng_int(r, flo, fhi);
  /* d pointer hops from the root to the data: d-2 next hops, one leaves hop,
   * one data hop; the chain therefore has d-1 nodes */
  BNode* root = NULL;
  BNode* prev = NULL;
  for (int64_t i = 0; i < d - 1; i++) {
    BNode* nd = (BNode*)new_structs(t, 1, sizeof(BNode));
    if (!nd) return -1;
    if (prev) prev->next = nd;
    else root = nd;
    prev = nd;
  }
  prev->nleaves = f;
  prev->leaves = (BLeaf*)new_structs(t, (uint64_t)f, sizeof(BLeaf));
  if (!prev->leaves) return -1;
  double ratio = log2((double)bhi / (double)blo);
  for (int64_t i = 0; i < f; i++) {
    uint64_t bytes = (uint64_t)floor((double)blo * exp2(ratio * rng_unit(r)));
    if (bytes > (uint64_t)bhi) bytes = (uint64_t)bhi;
    BLeaf* l = &prev->leaves[i];
    if (rng_next(r) >> 63) {
      l->n = (int64_t)(bytes / 8);
      l->f64 = new_f64(t, r, (uint64_t)l->n);
      if (!l->f64) return -1;
    } else {
      l->n = (int64_t)(bytes / 4);
      l->f32 = new_f32(t, r, (uint64_t)l->n);
      if (!l->f32) return -1;
    }
  }
  t->info[0] = d;
  t->info[1] = f;
  t->nroots = 1;
  t->roots = (void**)malloc(sizeof(void*));
  t->roots[0] = root;
  return 0;
}

fx_tree* fx_build(int shape, uint64_t seed, const int64_t* params, int nparams) {
  int64_t p[8] = {0};
  for (int i = 0; i < nparams && i < 8; i++) p[i] = params[i];
  fx_tree* t = (fx_tree*)calloc(1, sizeof(fx_tree));
  if (!t) return NULL;
  t->shape = shape;
  rng_t r;
  rng_seed(&r, seed);
  int rc;
  switch (shape) {
    case FX_SHAPE_PLAIN: rc = build_plain(t, &r, p); break;
    case FX_SHAPE_LINEAR: rc = build_linear(t, &r, p); break;
    case FX_SHAPE_DENSE: rc = build_dense(t, &r, p); break;
    case FX_SHAPE_WIDE: rc = build_wide(t, &r, p); break;
    case FX_SHAPE_MD: rc = build_md(t, seed, p); break;
    case FX_SHAPE_BROOM: rc = build_broom(t, &r, p); break;
    default: rc = -1;
  }
  if (rc) {
    fx_free(t);
    return NULL;
  }
  return t;
}

void fx_free(fx_tree* t) {
  if (!t) return;
  for (uint64_t i = 0; i < t->nallocs; i++) free(t->allocs[i].base);
  free(t->allocs);
  free(t->roots);
  free(t);
}
