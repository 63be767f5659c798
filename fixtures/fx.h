/* Seeded synthetic input trees for the deep-copy tests and benchmark.
 *
 * This module only builds inputs: pointer-linked host structures in plain
 * malloc'd memory, filled from a counter-free xoshiro256** stream seeded by
 * SplitMix64, plus a plain-data description of each struct layout. It holds
 * none of the deep-copy method (no walk order, layout, relocation or kernel
 * arithmetic); both the CPU oracle and the HIP path consume what it builds.
 *
 * Shapes follow the paper's Linear scenario (Section 4.1, one node type with
 * two ints, a payload array and a next pointer), its Dense scenario
 * (Section 4.2, the next pointer is an array of q nodes, depth D) and the
 * molecular-dynamics chain of the pointerchain example (Section 3, Figure 1).
 */
#ifndef FX_H
#define FX_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { FX_STRUCT = 0, FX_F32 = 1, FX_F64 = 2, FX_I32 = 3, FX_I64 = 4, FX_U8 = 5 };

enum {
  FX_SHAPE_PLAIN = 0,  /* Root{i64 n; Child* c} -> Child[n]{i64 n; double* leaf} */
  FX_SHAPE_LINEAR = 1, /* L{i32 nA; i32 nLnext; double* A; L* Lnext} x k */
  FX_SHAPE_DENSE = 2,  /* L{i32 nA; i32 nLnext; double* A; L* Lnext[q]} to depth D */
  FX_SHAPE_WIDE = 3,   /* Root -> Mid[f1] -> Leaf[f2]{i64 n; float* f32; double* f64} */
  FX_SHAPE_MD = 4,     /* Sim{i64 ncells; Cell*} -> Cell{i64 natoms; double *pos,*vel,*force} */
  FX_SHAPE_BROOM = 5,  /* Node{i64 nleaves; Node* next; Leaf* leaves} chain -> Leaf[f] */
};

#define FX_MAX_FIELDS 8
#define FX_MAX_TYPES 8

typedef struct {
  uint32_t offset;      /* byte offset of the pointer member */
  uint32_t kind;        /* FX_* kind of the pointee elements */
  uint32_t type;        /* pointee type index when kind == FX_STRUCT */
  int32_t count_offset; /* byte offset of the signed element-count member, -1 = fixed */
  uint32_t count_bytes; /* 4 or 8 */
  uint32_t count_mult;  /* elements per count unit */
  uint64_t fixed_count; /* element count when count_offset == -1 */
} fx_field;

typedef struct {
  char name[16];
  uint32_t size, align, nfields;
  fx_field fields[FX_MAX_FIELDS];
} fx_type;

typedef struct {
  void* base;
  uint64_t bytes;
  uint32_t kind; /* FX_* */
  uint32_t pad;
} fx_alloc;

typedef struct fx_tree {
  int shape;
  uint32_t ntypes, root_type;
  fx_type types[FX_MAX_TYPES];
  uint64_t nroots;
  void** roots;
  /* every allocation made, in creation order (leaf arrays and struct arrays) */
  uint64_t nallocs, cap_allocs;
  fx_alloc* allocs;
  /* per-shape scalar outputs, e.g. the chosen depth and fan-out of a broom */
  int64_t info[8];
} fx_tree;

/* params (int64 each; unused entries ignored):
 *  PLAIN : [nchild, leaf_len]
 *  LINEAR: [k, n, scheme]  scheme 0 = every level allocates n (allinit),
 *                          1 = only the last level allocates n (LLinit)
 *  DENSE : [q, n, D, packed_last] packed_last=1 gives the 12-byte last-level node
 *  WIDE  : [f1, f2, lo, hi]  leaf length floor(lo * (hi/lo)^u), even index FP32
 *  MD    : [nsims, cells_lo, cells_hi, mean_atoms]
 *  BROOM : [d_lo, d_hi, f_lo, f_hi, bytes_lo, bytes_hi]  one job's structure
 * Returns NULL on allocation failure or bad parameters. */
fx_tree* fx_build(int shape, uint64_t seed, const int64_t* params, int nparams);
void fx_free(fx_tree* t);

/* Fills the n values of one leaf array with the fixture distribution,
 * uniform[-1,1) from the given seed (used by tests that refill a leaf). */
void fx_fill_f64(double* x, uint64_t n, uint64_t seed);
void fx_fill_f32(float* x, uint64_t n, uint64_t seed);

/* Number of worker threads used by fx_build for the MD shape (0 = all cores). */
void fx_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
