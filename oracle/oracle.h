/* CPU oracle for the deep copy of a pointer-linked struct tree and the leaf
 * kernels that run on it.
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this; the product path never calls it. It shares
 * no code, header or table with the HIP path.
 *
 * What it computes, step by step (the paper: Section 2, Figure 2 steps a-d;
 * Section 4.1.1 and Algorithm 1 for marshalling into one buffer; Section 3 for
 * resolving a pointer chain once; Algorithm 2 steps 4-5 for the kernel and
 * the copy back):
 *   walk      recursive depth-first pre-order from each root; a struct array's
 *             children are visited element by element, fields by ascending
 *             byte offset; a pointer already visited is not visited again
 *   layout    off_0 = 0, off_i = align_up(off_{i-1} + max(bytes_{i-1}, 1), A)
 *   copy      the buffer is zeroed, then every object's bytes are copied in
 *   relocate  every non-null pointer slot becomes B + off(target)
 *   resolve   follow the relocated slots of a chain once, return its address
 *   kernel    x <- fma(x, a, b) per element, FP64 in binary64, FP32 in binary32
 *   copy back primitive arrays (and optionally non-pointer struct bytes) are
 *             written back to the host tree; host pointers are left alone
 *
 * Every function returns 0 or a negative error code (OR_E_*).
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_STRUCT = 0, OR_F32 = 1, OR_F64 = 2, OR_I32 = 3, OR_I64 = 4, OR_U8 = 5 };
enum { OR_OK = 0, OR_E_INVAL = -1, OR_E_RANGE = -2, OR_E_CONFLICT = -3, OR_E_NOMEM = -4 };

#define OR_MAX_FIELDS 16

typedef struct {
  uint32_t offset;      /* byte offset of the pointer member in the struct */
  uint32_t kind;        /* OR_* kind of the pointee elements */
  uint32_t type;        /* pointee struct type when kind == OR_STRUCT */
  int32_t count_offset; /* offset of the signed count member, or -1 */
  uint32_t count_bytes; /* 4 or 8 */
  uint32_t count_mult;  /* elements per count unit */
  uint64_t fixed_count; /* count when count_offset == -1 */
} or_field;

typedef struct {
  uint32_t size;
  uint32_t nfields;
  or_field fields[OR_MAX_FIELDS];
} or_type;

typedef struct {
  uint64_t host;  /* host address of the array */
  uint64_t off;   /* offset in the buffer */
  uint64_t bytes; /* count * element size */
  uint64_t count; /* elements */
  uint32_t kind;
  uint32_t type;
} or_object;

typedef struct or_copy or_copy;

/* Deep copy of the trees under roots[0..nroots) (each root is one struct of
 * root_type) into a freshly allocated host buffer whose pointers are written
 * as if the buffer lived at address `base`. */
int or_deep_copy(const or_type* types, uint32_t ntypes, uint32_t root_type, void* const* roots, uint64_t nroots,
                 uint64_t align, uint64_t base, or_copy** out);
/* Selective deep copy (Section 2, selective or partial deep copy): follow[t]
 * has bit i set when pointer field i (position in type t's field list) is to
 * be followed. An unfollowed field is not walked, its array is not copied,
 * and it reads as a null pointer in the buffer. follow == NULL follows all. */
int or_deep_copy_selective(const or_type* types, uint32_t ntypes, uint32_t root_type, void* const* roots,
                           uint64_t nroots, uint64_t align, uint64_t base, const uint32_t* follow, or_copy** out);
void or_free(or_copy* c);

uint8_t* or_arena(const or_copy* c);
uint64_t or_arena_bytes(const or_copy* c);
uint64_t or_nobjects(const or_copy* c);
const or_object* or_objects(const or_copy* c);
uint64_t or_nslots(const or_copy* c);      /* non-null pointer slots */
uint64_t or_payload_bytes(const or_copy* c); /* sum of object bytes */

/* Follows a chain from root `root_index`: at each step read pointer field
 * fields[s] of the current element; before the last step move to element
 * index[s] of the array it points to. Returns the final pointer (a buffer
 * address), the element count of its array and its kind. */
int or_resolve_chain(const or_copy* c, uint64_t root_index, const uint32_t* fields, const uint64_t* index,
                     uint32_t nsteps, uint64_t* addr, uint64_t* count, uint32_t* kind);

/* The buffer address (as laid out at `base`) of a scalar member reached by a
 * chain: each step reads pointer field fields[s] and moves to element
 * index[s] of the struct array it points to; the scalar is `bytes` (1, 4 or
 * 8) bytes at `offset` in the element reached last (the root if nsteps == 0).
 * Reading it there and writing a new value back there are the two halves of
 * a scalar chain's declare and update (Section 3). */
int or_scalar_chain(const or_copy* c, uint64_t root_index, const uint32_t* fields, const uint64_t* index,
                    uint32_t nsteps, uint32_t offset, uint32_t bytes, uint64_t* addr);

/* select 0: the leaf at the end of the chain; 1: every FP32/FP64 array.
 * out == NULL: in place in the buffer. Otherwise the results go to `out`,
 * leaves in layout order, each at the next multiple of the layout alignment
 * after the previous one's end (the same rule as the buffer layout). */
int or_run_kernel(or_copy* c, int select, uint64_t root_index, const uint32_t* fields, const uint64_t* index,
                  uint32_t nsteps, uint32_t iters, double a, double b, float af, float bf, uint8_t* out,
                  uint64_t out_bytes);
/* bytes needed by the out-of-place results of or_run_kernel */
uint64_t or_out_bytes(const or_copy* c, int select, uint64_t root_index, const uint32_t* fields,
                      const uint64_t* index, uint32_t nsteps);

/* Molecular-dynamics kick then drift, `steps` times, on every element of
 * struct type `type` (in place in the buffer): v <- fma(f, dt_over_m, v),
 * then x <- fma(v, dt, x), over the FP64 arrays that pointer fields xf, vf
 * and ff point to. OR_E_INVAL for unequal counts, a partly null triple or a
 * field that is not FP64; OR_E_CONFLICT when an array serves two elements
 * or roles. */
int or_kick_drift(or_copy* c, uint32_t type, uint32_t xf, uint32_t vf, uint32_t ff, uint32_t steps, double dt,
                  double dt_over_m);

/* Writes primitive arrays back to their host addresses; scalars != 0 also
 * writes the non-pointer bytes of struct elements. */
int or_copy_back(const or_copy* c, int scalars);

/* One fused-multiply-add, exposed for the rounding tests. */
double or_fma64(double x, double a, double b);
float or_fma32(float x, float a, float b);

#ifdef __cplusplus
}
#endif
#endif
