/* dc.h -- deep copy of pointer-linked struct trees into one MI355X device
 * arena, device-side pointer relocation, pointer-chain resolution and leaf
 * kernels. C ABI: plain pointers and sizes, no C++ or torch types.
 *
 * The operations follow the paper's problem statement:
 *   - describing nested structures (Section 2: structs whose members point to
 *     arrays of primitives or of other structs; the Linear node of
 *     Section 4.1 with its count members nA and nLnext);
 *   - the deep copy (Section 2, Figure 2 steps a-d: initialise, copy the main
 *     structure, copy the nested ones, fix the pointers on the device), done
 *     as marshalling into one contiguous buffer (Algorithm 1: size the tree,
 *     allocate once, hand out space in request order, transfer the buffer in
 *     one batch, then attach every pointer on the device);
 *   - resolving a pointer chain once to its effective address (Section 3);
 *   - running the kernel once and transferring the tree back (Algorithm 2,
 *     steps 4 and 5; the scaling kernel of Sections 4.1.2 and 4.2.2);
 *   - the selective deep copy (Section 2), the pointerchain transfer scheme
 *     that moves only the array a chain ends in, and scalar chains with
 *     write-back (Section 3), and a molecular-dynamics leaf kernel on the
 *     atoms-in-cells structure of Section 3's example;
 *   - a batched form (every structure of a plan relocated and computed per
 *     launch, captured in a HIP graph, autotuned) and a served form
 *     (admission under a device-memory budget, resident structures).
 *
 * Conventions for every call:
 *   - Returns dc_status: DC_OK (0) or a negative DC_E_* code. The text of the
 *     last error of the calling thread is returned by dc_last_error().
 *     No C++ exception crosses this boundary.
 *   - A "stream" is a hipStream_t passed as void*; NULL means the null stream.
 *   - "device pointer" arguments are HIP device allocations on the context's
 *     device; "host pointer" arguments are ordinary host memory.
 *   - On error, every output handle is set to NULL and nothing is leaked;
 *     device buffers written before the error hold unspecified bytes.
 *   - One context, and everything made from it, is used by one host thread
 *     at a time. A server (dc_server_*) owns its own threads.
 */
#ifndef DC_H
#define DC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dc_status;
enum {
  DC_OK = 0,
  DC_E_INVAL = -1,    /* null/unknown handle, bad argument, unknown type, negative count */
  DC_E_RANGE = -2,    /* buffer too small, pointer into the middle of an array, chain past a null */
  DC_E_CONFLICT = -3, /* one address reached again as a different kind, type or length */
  DC_E_NOMEM = -4,    /* host or pinned allocation failed */
  DC_E_HIP = -5,      /* a HIP runtime call failed (text names it) */
  DC_E_STATE = -6,    /* call out of order, released tree, device-side check failed */
  DC_E_BUDGET = -7    /* a served job can never fit the device-memory budget */
};

/* element kinds of an array a pointer member refers to */
typedef enum { DC_KIND_STRUCT = 0, DC_KIND_F32 = 1, DC_KIND_F64 = 2, DC_KIND_I32 = 3, DC_KIND_I64 = 4, DC_KIND_U8 = 5 } dc_kind;

typedef struct dc_ctx_s* dc_ctx;
typedef struct dc_schema_s* dc_schema;
typedef struct dc_plan_s* dc_plan;
typedef struct dc_tree_s* dc_tree;
typedef struct dc_graph_s* dc_graph;
typedef struct dc_server_s* dc_server;

/* One pointer member of a struct type. The member holds the address of an
 * array of `count` elements of `kind` (of struct type `type_id` when kind is
 * DC_KIND_STRUCT), or NULL for no array. The count is read from a signed
 * integer member of the same struct element (count_offset >= 0, count_bytes
 * 4 or 8) times count_mult (e.g. 3 for an array of double3), or is
 * fixed_count when count_offset == -1. offset must be a multiple of 8. */
typedef struct {
  uint32_t offset;
  uint32_t kind;
  uint32_t type_id;
  int32_t count_offset;
  uint32_t count_bytes;
  uint32_t count_mult;
  uint64_t fixed_count;
} dc_field;

/* One step of a pointer chain: read pointer member `field` (its position in
 * the field list given to dc_schema_describe) of the current struct element;
 * unless this is the last step, continue at element `index` of the array it
 * points to. */
typedef struct {
  uint32_t field;
  uint32_t reserved;
  uint64_t index;
} dc_step;

/* A resolved chain: the device address of the array at the end of the chain,
 * its element count and kind. */
typedef struct {
  uint64_t dev_addr;
  uint64_t count;
  uint32_t kind;
  uint32_t reserved;
} dc_chain;

/* A placed object: where an array of the host tree lives in the arena. */
typedef struct {
  uint64_t host_addr;
  uint64_t offset;
  uint64_t bytes;
  uint64_t count;
  uint32_t kind;
  uint32_t type_id;
} dc_object;

typedef struct {
  uint64_t nobjects;      /* arrays placed in the arena */
  uint64_t nslots;        /* pointer members of all struct elements (null or not) */
  uint64_t nslots_nonnull;
  uint64_t nleaves;       /* FP32/FP64 arrays with at least one element */
  uint64_t payload_bytes; /* sum of object bytes, no padding */
  uint64_t leaf_bytes;    /* sum of FP32/FP64 array bytes */
  uint64_t arena_bytes;   /* device arena size the plan needs */
  uint64_t scratch_bytes; /* device scratch size the plan needs */
  uint64_t out_bytes;     /* out-of-place leaf image size (see dc_kernel_args) */
  uint64_t nsegments;     /* relocation work units */
  uint64_t nroots;
  uint64_t unit_leaves;   /* 1: every relocation unit's slots first reach one
                             contiguous run of leaves, so the persistent batched
                             launch takes a whole unit per item (dc_batch_run) */
  uint64_t max_unit_leaf_bytes; /* the largest such run, in 16-byte chunks x 16 */
  uint64_t leaf_prefix_offset;  /* byte offset in the scratch buffer of nleaves + 1
                                   uint64 words that the deep copy computes on the
                                   device (the sizing step of Algorithm 1, for the
                                   leaves): word l is the number of 16-byte chunks
                                   of the leaves before leaf l in arena order, each
                                   leaf rounded up to whole chunks, and word nleaves
                                   their total. Read-only for the caller. */
} dc_plan_info;

/* ---- lifecycle --------------------------------------------------------------- */

/* A context on HIP device `device`: owns pinned host staging buffers (eight
 * of 32 MiB, 256 MiB in all, allocated and written once here, so that no
 * deep copy pays the first touch of their pages, and freed by
 * dc_ctx_destroy) and a pool of host threads for packing. Errors:
 * DC_E_NOMEM if the pinned staging cannot be allocated, DC_E_HIP. */
dc_status dc_ctx_create(int device, dc_ctx* out);
/* Frees the context's staging and threads, after every tree, plan and server
 * made with it has been released. Errors: DC_E_INVAL for NULL. */
dc_status dc_ctx_destroy(dc_ctx ctx);

/* An empty schema; dc_schema_describe adds its struct types. Errors:
 * DC_E_INVAL for a NULL out. */
dc_status dc_schema_create(dc_schema* out);
/* Frees a schema, after the plans and servers made from it. Errors:
 * DC_E_INVAL for NULL. */
dc_status dc_schema_destroy(dc_schema schema);

/* Registers a struct type of `size` bytes and alignment `align` with its
 * pointer members (Section 2: the nested, user-defined members that must be
 * followed; non-pointer members are copied as plain bytes). Type ids are
 * assigned 0, 1, 2, ... in call order; a field may name a type id that is
 * described later. At most 16 pointer fields per type and 64 types.
 * DC_E_INVAL for misaligned or overlapping pointer members, count members
 * outside the struct, or bad kinds. */
dc_status dc_schema_describe(dc_schema schema, const char* name, uint32_t size, uint32_t align,
                             const dc_field* fields, uint32_t nfields, uint32_t* out_type_id);

/* ---- deep copy (Section 2, Figure 2; Algorithm 1) ------------------------------ */

/* Plans the deep copy of the trees under roots[0..nroots): each root is the
 * host address of one struct of type root_type. The host tree is walked
 * depth-first in pre-order (elements in index order, pointer members in
 * ascending offset order; an address reached again is not visited again),
 * and every array gets an arena offset: the first at 0, each next one at the
 * next multiple of `align` at or after the previous one's end (a zero-length
 * array occupies one byte). align: power of two, 16..4096 (64 if 0).
 * ctx may be NULL (planning needs no device).
 * The plan reads the host tree; the tree's shape (pointers and counts) must
 * not change while the plan is used. Values may change.
 * Errors: DC_E_INVAL (null root, negative count, unknown type),
 * DC_E_CONFLICT (an address reached as two different arrays), DC_E_RANGE
 * (a pointer into the middle of another array). */
dc_status dc_plan_create(dc_ctx ctx, dc_schema schema, uint32_t root_type, const void* const* roots, uint64_t nroots,
                         uint64_t align, dc_plan* out, uint64_t* arena_bytes, uint64_t* scratch_bytes);
/* Selective (partial) deep copy (Section 2): only the pointer members a
 * kernel needs are followed. follow[t] (t < nfollow) has bit i set when
 * pointer field i of type t (its position in the field list given to
 * dc_schema_describe) is followed; types at or past nfollow follow every
 * field. An unfollowed member is not walked, its array is not copied, and it
 * reads as NULL in the device copy. Otherwise as dc_plan_create.
 * Errors: DC_E_INVAL also for nfollow above the number of types or a mask
 * with a bit past its type's field count. */
dc_status dc_plan_create_selective(dc_ctx ctx, dc_schema schema, uint32_t root_type, const void* const* roots,
                                   uint64_t nroots, uint64_t align, const uint32_t* follow, uint32_t nfollow,
                                   dc_plan* out, uint64_t* arena_bytes, uint64_t* scratch_bytes);
/* Frees a plan, after the trees made from it. Errors: DC_E_INVAL for NULL. */
dc_status dc_plan_destroy(dc_plan plan);
/* The plan's sizes and counts. Errors: DC_E_INVAL for a NULL argument. */
dc_status dc_plan_query(dc_plan plan, dc_plan_info* out);
/* Copies up to cap placed objects, in arena order, into out; *n receives the
 * total number of objects. Errors: DC_E_INVAL for a NULL plan or n, or a
 * NULL out with cap > 0. */
dc_status dc_plan_objects(dc_plan plan, dc_object* out, uint64_t cap, uint64_t* n);

/* The deep copy: packs the host tree into pinned staging in arena order
 * (padding zeroed), transfers it to d_arena over the host link in pipelined
 * chunks, uploads the plan's relocation tables into d_scratch and relocates
 * every pointer member on the device (host address -> d_arena + offset; null
 * stays null). Returns once the host tree has been read; the transfer and the
 * relocation may still be running on `stream`.
 * d_arena (>= arena_bytes) and d_scratch (>= scratch_bytes) are device
 * buffers owned by the caller, 256-byte aligned, that must outlive the tree.
 * Errors: DC_E_RANGE (buffers too small or misaligned), DC_E_HIP. */
dc_status dc_deep_copy_to_device(dc_ctx ctx, dc_plan plan, void* d_arena, uint64_t arena_bytes, void* d_scratch,
                                 uint64_t scratch_bytes, void* stream, dc_tree* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the deep copy
 * of dc_deep_copy_to_device, with the relocation tables and the device header
 * in a fixed array of DC_NOALLOC_SCRATCH_BYTES that the library holds on each
 * device from its load until the process ends, instead of a caller scratch
 * buffer. Makes no device or pinned allocation (the staging ring and the
 * array's address are set up by dc_ctx_create). The tree it returns works
 * with every other call. One such tree at a time per device: the array keeps
 * the last copy's tables, so while a tree made here is alive, another call on
 * the same device returns DC_E_STATE; dc_tree_release of such a tree first
 * waits until the device is idle (nothing queued still reads its tables),
 * then frees the array for the next call. Calls for one device from several
 * threads are serialised by that rule; a caller that bypasses it by using a
 * released tree races with the next copy. d_arena as for
 * dc_deep_copy_to_device. Errors: DC_E_RANGE if the plan's tables (the
 * scratch_bytes dc_plan_create reported) exceed DC_NOALLOC_SCRATCH_BYTES or
 * d_arena is too small or misaligned; DC_E_STATE as above; DC_E_INVAL for
 * NULL arguments; DC_E_HIP. */
#define DC_NOALLOC_SCRATCH_BYTES (64ull << 20)
dc_status dc_deep_copy_to_device_noalloc(dc_ctx ctx, dc_plan plan, void* d_arena, uint64_t arena_bytes, void* stream,
                                         dc_tree* out);

/* Like dc_deep_copy_to_device but without the relocation: the arena holds
 * the host bytes verbatim (host addresses in every pointer member) until
 * dc_attach or dc_batch_run relocates it. Errors: as dc_deep_copy_to_device. */
dc_status dc_stage_to_device(dc_ctx ctx, dc_plan plan, void* d_arena, uint64_t arena_bytes, void* d_scratch,
                             uint64_t scratch_bytes, void* stream, dc_tree* out);

/* Device pointer passes over every pointer member of the arena (Algorithm 1's
 * attach of each pointer; the reverse, detach, is part of demarshalling):
 * attach rewrites host addresses to device addresses, detach rewrites device
 * addresses back to the host addresses they came from. The tree must be in
 * the opposite state (DC_E_STATE otherwise). Asynchronous on `stream`; an
 * address that is not a planned array start is counted in a device error
 * flag that the next synchronous call reports as DC_E_STATE. Errors also:
 * DC_E_INVAL for a NULL or released tree, DC_E_HIP. */
dc_status dc_attach(dc_tree tree, void* stream);
dc_status dc_detach(dc_tree tree, void* stream);

/* ---- pointerchain (Section 3) ---------------------------------------------------- */

/* Resolves a chain once, on the device, by following the relocated pointers
 * of root `root_index`; checks the result against the plan. Synchronous.
 * Errors: DC_E_INVAL (bad field or steps), DC_E_RANGE (null before the last
 * step, index past the array), DC_E_STATE (not attached). */
dc_status dc_resolve_chain(dc_tree tree, uint64_t root_index, const dc_step* steps, uint32_t nsteps, void* stream,
                           dc_chain* out);

/* The pointerchain transfer scheme (Section 3): resolve a chain on the host
 * tree and transfer only the array it ends in; the structures along the
 * chain are not copied, since the kernel needs only the effective address.
 *
 * dc_chain_query: the count and kind of the host array a chain ends in
 * (out->dev_addr = 0), so that the caller can size d_buf. Needs no device.
 * Errors: DC_E_INVAL (bad field or steps), DC_E_RANGE (null before the end,
 * index past an array). */
dc_status dc_chain_query(dc_schema schema, uint32_t root_type, const void* root, const dc_step* steps,
                         uint32_t nsteps, dc_chain* out);
/* dc_chain_to_device walks the chain from the host struct `root` (type
 * root_type) and copies the final FP32/FP64 array (count * element size
 * bytes) into d_buf (a 16-byte aligned device buffer of buf_bytes); *out
 * receives d_buf, the count and the kind. Returns once the host array has
 * been read. Errors: as dc_chain_query, DC_E_RANGE for a buffer too small
 * or misaligned, DC_E_INVAL for a chain that ends in a struct array. */
dc_status dc_chain_to_device(dc_ctx ctx, dc_schema schema, uint32_t root_type, const void* root, const dc_step* steps,
                             uint32_t nsteps, void* d_buf, uint64_t buf_bytes, void* stream, dc_chain* out);
/* `iters` passes of x = fma(x, a, b) (FP64: a, b; FP32: af, bf) over an array
 * placed by dc_chain_to_device. Asynchronous on `stream`. Errors: DC_E_INVAL
 * for a NULL context or chain or a kind other than FP32/FP64, DC_E_HIP. */
dc_status dc_chain_run_kernel(dc_ctx ctx, const dc_chain* c, uint32_t iters, double a, double b, float af, float bf,
                              void* stream);
/* Transfers such an array back into the host array the same chain ends in.
 * Returns when the host array is updated. Errors: as dc_chain_query;
 * DC_E_STATE if the chain now ends in an array of another count or kind than
 * the device copy (the host tree changed); DC_E_HIP. */
dc_status dc_chain_copy_back(dc_ctx ctx, dc_schema schema, uint32_t root_type, const void* root, const dc_step* steps,
                             uint32_t nsteps, const dc_chain* c, void* stream);

/* Scalar chains (Section 3, scalar variables): a scalar member reached by a
 * chain is copied into a temporary before a region and written back through
 * the same chain when the region ends, so the structure sees the update. */
typedef struct {
  uint64_t root_index;
  const dc_step* steps; /* each step: pointer field, then the element to move to */
  uint32_t nsteps;      /* 0: a member of the root struct itself (at most 32) */
  uint32_t offset;      /* byte offset of the scalar in the element reached last */
  uint32_t bytes;       /* 1, 4 or 8; may not overlap a pointer member */
  uint32_t reserved;
} dc_scalar_ref;
/* Walks every chain on the device (attached tree) and stores each scalar,
 * zero-extended, in d_temps[i] (device, 8 bytes per ref, 8-byte aligned).
 * Returns when the values are in d_temps.
 * Errors: DC_E_INVAL (bad field, a step through a primitive array, bytes,
 * overlap with a pointer member), DC_E_RANGE (null pointer or index past an
 * array on the way), DC_E_STATE (not attached; the device walk disagreed
 * with the plan). */
dc_status dc_scalar_declare(dc_tree tree, const dc_scalar_ref* refs, uint32_t nrefs, void* d_temps, void* stream);
/* Writes the low `bytes` bytes of d_temps[i] back to the scalar its chain
 * reaches, walking the chain again on the device. Returns when written.
 * Errors as dc_scalar_declare. dc_copy_back with DC_COPY_SCALARS then takes
 * the values to the host structure. */
dc_status dc_scalar_update(dc_tree tree, const dc_scalar_ref* refs, uint32_t nrefs, const void* d_temps,
                           void* stream);

/* Molecular-dynamics leaf kernel on sibling leaves (the atoms-in-cells
 * structure of the pointerchain example in Section 3): for every element of
 * struct type `type`, `steps` times, over the FP64 arrays its members x_field,
 * v_field and f_field point to (positions, velocities, forces):
 *   v <- fma(f, dt_over_m, v)   then   x <- fma(v, dt, x)
 * one rounding per fma. Each element's three arrays must have equal counts
 * and be all null (skipped) or all non-null; no array may serve two elements
 * or two roles. The element list is built on the first call for a
 * (type, fields) choice and kept in device memory the library owns until
 * dc_tree_release. Asynchronous on `stream`.
 * Errors: DC_E_INVAL (type, fields, counts, a partly null element),
 * DC_E_CONFLICT (a shared array), DC_E_STATE (not attached). */
typedef struct {
  uint32_t type;
  uint32_t x_field, v_field, f_field;
  uint32_t steps;
  uint32_t reserved;
  double dt;
  double dt_over_m;
} dc_kick_drift_args;
dc_status dc_run_kick_drift(dc_tree tree, const dc_kick_drift_args* args, void* stream);

/* ---- leaf kernels (Algorithm 2 step 4) --------------------------------------------- */

enum { DC_MODE_RESOLVED = 0, DC_MODE_DEREF_EACH = 1 };
enum { DC_SELECT_CHAIN = 0, DC_SELECT_ALL_LEAVES = 1 };

/* x <- fma(x, a, b) for every element of the selected leaves, `iters` full
 * passes (each pass a separate sweep over the data). FP64 leaves use a and b
 * in binary64, FP32 leaves use af and bf in binary32; both are single
 * correctly rounded fused multiply-adds.
 * select CHAIN: the FP32/FP64 array at the end of `chain` from root
 * root_index; ALL_LEAVES: every FP32/FP64 array of the tree.
 * mode RESOLVED: the array address is resolved once (Section 3) and the kernel
 * indexes it directly. DEREF_EACH: every element access walks the whole chain
 * from the root again, reading each pointer from the arena (the paper's
 * per-iteration dereference); for ALL_LEAVES the chain of a leaf is the path
 * by which the walk first reached it.
 * d_out NULL: in place. Otherwise a device buffer of at least out_bytes that
 * receives the results as a leaf image: the selected leaves in arena order,
 * each at the next multiple of the plan alignment after the previous one's
 * end, the first at 0; the arena is left unchanged.
 * Asynchronous on `stream`. No other work may write the arena's pointer
 * members while a kernel runs on it: the per-access walks rely on the slots
 * one checked walk per wavefront has validated.
 * Errors reported by the kernel (a slot or leaf outside the arena) surface in
 * dc_tree_check. */
typedef struct {
  uint32_t mode;
  uint32_t select;
  uint32_t iters;
  uint32_t nsteps;
  double a, b;
  float af, bf;
  uint64_t root_index;
  const dc_step* chain;
  void* d_out;
  uint64_t out_bytes;
} dc_kernel_args;

dc_status dc_run_kernel(dc_tree tree, const dc_kernel_args* args, void* stream);

/* Bytes of the out-of-place leaf image for args (select and chain). Errors:
 * DC_E_INVAL for a NULL argument or an invalid chain. */
dc_status dc_out_bytes(dc_tree tree, const dc_kernel_args* args, uint64_t* out);

/* ---- copy back (Algorithm 2 step 5) ------------------------------------------------ */

enum { DC_COPY_LEAVES = 1, DC_COPY_SCALARS = 2 };
/* Transfers the arena back and writes into the host tree: LEAVES = every
 * primitive array; SCALARS = the non-pointer bytes of every struct element.
 * Host pointer members are never written. Returns when the host tree is
 * updated (waits for earlier work on `stream`). Errors: DC_E_INVAL for a NULL
 * or released tree or unknown flags, DC_E_STATE when the device check after
 * the transfer fails (the host tree has been written), DC_E_HIP. */
dc_status dc_copy_back(dc_tree tree, uint32_t flags, void* stream);

/* Releases the tree's host-side state (not the caller's device buffers).
 * Destroy the tree's graphs first: a graph refers to its tree. Errors:
 * DC_E_INVAL for NULL. */
dc_status dc_tree_release(dc_tree tree);
/* Waits for `stream`, then reports a device-side error recorded by earlier
 * passes of this tree (DC_E_STATE) or DC_OK. */
dc_status dc_tree_check(dc_tree tree, void* stream);
/* The layout of a deep copy on the device: as dc_plan_objects, except that
 * `offset` is replaced by the object's device address (d_arena + offset).
 * Errors: DC_E_INVAL for a NULL or released tree, as dc_plan_objects. */
dc_status dc_tree_objects(dc_tree tree, dc_object* out, uint64_t cap, uint64_t* n);

/* ---- batched form ------------------------------------------------------------------ */

/* Launch shape of the batched relocate+compute work. Zero fields (other than
 * launches) take the tuned or default choice. */
typedef struct {
  uint32_t block;          /* threads per workgroup: 256, 512 or 1024 */
  uint32_t wg_per_cu;      /* resident workgroups per compute unit */
  uint32_t tile_chunks;    /* 16-byte chunks per compute tile: a power of two,
                              512..2^20 (DC_E_INVAL otherwise) */
  uint32_t launches;       /* 0: one persistent launch; 1: three ordinary launches
                              (relocate, every leaf, reverse relocate), for which
                              block and wg_per_cu are not used; 2: one persistent
                              launch in three phases (what 0 runs when the plan's
                              relocation units do not own contiguous leaf runs);
                              3: one fused launch of tiles that relocate their own
                              leaves' slots (block and wg_per_cu not used); 4: the
                              fused launch's work in one persistent launch (block
                              256, wg_per_cu at most 8, else DC_E_INVAL) */
  uint32_t spin_limit;     /* persistent launch: polls (about 1 us each) a workgroup
                              waits for a phase to finish before it records an error
                              and goes on, so that every launch ends; 0: 2^24 */
} dc_tune;

/* DC_BATCH_FORCE_WAIT_BOUND is for tests of the error path only: it runs the
 * three-phase persistent launch, in which every wait waits for one item more
 * than its phase has, so each wait ends at its bound (keep tune->spin_limit
 * small); the launch still ends, the tree's leaf values and slots are then
 * unspecified, and the next check of the tree returns DC_E_STATE. DC_E_INVAL
 * with three launches or either fused launch (no waits to force). */
enum { DC_BATCH_ATTACH = 1, DC_BATCH_DETACH = 2, DC_BATCH_FORCE_WAIT_BOUND = 4 };
/* Every structure's relocation and its leaves' kernel (args: RESOLVED,
 * ALL_LEAVES, iters == 1), the batched use of Figure 2(d) and Algorithm 2
 * step 4. tune->launches 0: one persistent launch whose workgroups take items
 * from one device work queue. When every relocation unit's slots first reach
 * one contiguous run of leaves (depth-first layouts whose structs list leaf
 * members before deeper struct members), an item is a whole unit: its attach,
 * the kernel over its leaves (addresses read from the slots it just wrote)
 * and its detach, with no wait between workgroups. Otherwise the launch runs
 * in three phases: attach units, then compute tiles, then (DETACH) reverse
 * relocation units, each phase waiting for the one before. 2: always the
 * three phases. 1: the same work as three stream-ordered launches. 3: one
 * launch over the compute tiles in which every tile translates the slot each
 * of its leaves was first reached through (the tile holding the leaf's first
 * chunk checks it and, after its compute, attaches and then detaches it as the
 * flags ask; a tile holding later chunks of the same leaf accepts either value;
 * every tile computes at the leaf's planned address, the value the attach
 * writes), and
 * workgroups past the tiles translate every other slot; no workgroup waits for
 * another, and any plan can use it. 4: the items of 3 in a persistent grid of
 * wg_per_cu workgroups per compute unit that take them from eight interleaved
 * device queues (reset by a one-workgroup kernel before the launch). ATTACH
 * requires a staged (unrelocated) tree; DETACH leaves it staged again. tune
 * NULL: the cached autotuner choice, else the fused launch (3) over 1024-chunk
 * tiles. Asynchronous on `stream`.
 * Runs on one tree must not overlap on different streams: they share its
 * arena and, in the persistent forms, its work queues in the device header. */
dc_status dc_batch_run(dc_tree tree, const dc_kernel_args* args, const dc_tune* tune, uint32_t flags, void* stream);

/* Times candidate tile shapes of dc_batch_run with ATTACH|DETACH on this
 * tree (which leaves its leaf values changed: deep copy again before a run
 * whose values matter) and returns the fastest; the choice is cached on disk
 * keyed by device and workload shape (DC_TUNE_CACHE, default
 * ~/.cache/dc_tune.json). Synchronous: it first waits for all work queued on
 * the device (the tree's deep copy may still be in flight on the caller's
 * stream), then times the candidates on a stream of its own. Errors: DC_E_INVAL for a NULL argument or args
 * other than RESOLVED, ALL_LEAVES, one pass; DC_E_STATE if the tree is
 * attached or a device check fails; DC_E_RANGE for a d_out too small or
 * misaligned; DC_E_HIP. */
dc_status dc_autotune(dc_tree tree, const dc_kernel_args* args, uint32_t reps, dc_tune* out);
/* The candidates the tree's last dc_autotune timed, in order, with the median
 * time of each in microseconds: up to `cap` of them into tunes[] and us[]
 * (caller-owned), their number in *n (0 before any autotune). Errors:
 * DC_E_INVAL for a NULL or released tree, NULL n, or NULL arrays with cap > 0. */
dc_status dc_autotune_results(dc_tree tree, dc_tune* tunes, double* us, uint32_t cap, uint32_t* n);

/* Captures dc_batch_run(tree, args, tune, flags) into a HIP graph; optionally
 * preceded by the host-to-device transfer of the staged image (upload != 0,
 * which keeps a pinned copy of the whole image) and followed by the transfer
 * back of the arena into pinned memory (download != 0). Creation first waits
 * for all work queued on the device (the tree's deep copy included) and
 * returns when the capture is complete. dc_graph_launch
 * replays it; if a call with another tile size has rebuilt the tree's tile
 * list since the capture, the launch first rebuilds the captured one.
 * Errors (create): DC_E_INVAL for flags other than ATTACH|DETACH or bad args
 * or tune, DC_E_STATE if the tree is attached, DC_E_NOMEM for the pinned
 * image, DC_E_HIP. Errors (launch): DC_E_INVAL for NULL, DC_E_STATE if the
 * tree is attached, DC_E_HIP. */
dc_status dc_graph_create(dc_tree tree, const dc_kernel_args* args, const dc_tune* tune, uint32_t flags,
                          int upload, int download, dc_graph* out);
dc_status dc_graph_launch(dc_graph graph, void* stream);
/* The page-locked host buffer a graph captured with download != 0 transfers
 * the arena into (Algorithm 2 step 5's transfer back, as a graph node):
 * *host and *bytes (the arena's size). The buffer belongs to the graph and
 * lives until dc_graph_destroy; after a replay has completed on its stream
 * it holds the arena as that replay left it (device addresses in the slots
 * only if the tree was left attached, which a graph never does). Errors:
 * DC_E_INVAL for a NULL argument, DC_E_STATE for a graph captured without
 * download. */
dc_status dc_graph_image(dc_graph graph, const void** host, uint64_t* bytes);
/* Destroys a graph (before its tree is released). */
dc_status dc_graph_destroy(dc_graph graph);

/* ---- served form ---------------------------------------------------------------- */

/* A server admits deep-copy+kernel jobs against a device-memory budget,
 * keeps copied structures resident for reuse, and admits new jobs while
 * others are on the device (continuous batching), overlapping their
 * transfers and kernels on several streams. */
typedef struct {
  uint64_t budget_bytes;   /* device bytes for arenas, scratch and outputs */
  uint32_t max_inflight;   /* jobs on the device at once */
  uint32_t nstreams;       /* copy/compute streams */
  uint64_t align;          /* arena alignment (0: 64) */
  uint32_t fail_copy_at;   /* tests of the error path only: the admission of the
                              n-th new structure (1-based) fails after its deep
                              copy, as a failing later step would; 0 = never */
  uint32_t reserved;
} dc_server_config;

typedef struct {
  uint32_t root_type;
  uint32_t reserved;
  const void* root;        /* host address of the structure's root struct */
  uint64_t key;            /* identity for residency: equal keys name the same
                              unchanged structure; 0 = never reuse */
  double a, b;             /* the job's kernel: out = fma(leaf, a, b) */
  float af, bf;
  void* out_host;          /* host buffer receiving the leaf image; when it is
                              page-locked (hipHostMalloc) each leaf is copied
                              into it directly, else through pinned staging */
  uint64_t out_bytes;      /* its size; must be >= the structure's leaf image */
} dc_request;

typedef struct {
  uint64_t id;
  dc_status status;
  uint32_t reused;         /* 1 if the structure was already resident */
  double t_submit, t_admit, t_done; /* seconds, steady clock */
  uint64_t out_bytes;
} dc_result;

typedef struct {
  uint64_t submitted, completed, reused, evictions, batches;
  uint64_t h2d_bytes, d2h_bytes, kernel_bytes;
  uint64_t resident_bytes, peak_bytes;
} dc_server_stats;

/* A server on ctx's device for structures of `schema`: one device allocation
 * of cfg->budget_bytes (at least 1 MiB), two contexts of its own (pinned
 * staging for each direction) and its two threads. Errors: DC_E_INVAL for a
 * NULL argument or a budget under 1 MiB, DC_E_NOMEM, DC_E_HIP (the budget's
 * allocation or a stream). */
dc_status dc_server_create(dc_ctx ctx, dc_schema schema, const dc_server_config* cfg, dc_server* out);
/* Queues a job (the structure is read when the job is admitted, so it must
 * stay unchanged until its result arrives); returns its id. DC_E_BUDGET if
 * it can never fit the budget. */
dc_status dc_server_submit(dc_server srv, const dc_request* req, uint64_t* id);
/* Waits for job `id` (timeout_s < 0: forever) and returns its result.
 * Errors: DC_E_INVAL for a NULL argument or an unknown id, DC_E_STATE if the
 * job has not finished within timeout_s, else the job's own status. */
dc_status dc_server_wait(dc_server srv, uint64_t id, double timeout_s, dc_result* out);
/* Counters since creation. Errors: DC_E_INVAL for a NULL argument. */
dc_status dc_server_stats_get(dc_server srv, dc_server_stats* out);
/* Lets admitted jobs finish, stops the threads and frees the budget and the
 * server's contexts. Errors: DC_E_INVAL for NULL. */
dc_status dc_server_destroy(dc_server srv);

/* ---- misc ------------------------------------------------------------------------ */

const char* dc_last_error(void);
/* Library version string. */
const char* dc_version(void);

#ifdef __cplusplus
}
#endif
#endif
