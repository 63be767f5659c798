"""Seeded synthetic input trees shared by the CPU oracle and the HIP path.

Inputs only: this package builds pointer-linked host structures and describes
their struct layouts as plain data. It contains no part of the deep-copy
method (no walk order, layout, relocation or kernel arithmetic).

Shapes:
  plain  -- root -> array of children -> one FP64 leaf per child
  linear -- the Linear scenario (Section 4.1): k nodes, payload of n doubles
  dense  -- the Dense scenario (Section 4.2): the next pointer is an array of q
  wide   -- root -> mids -> leaf structs, each pointing to an FP32 or FP64 array
  md     -- simulations -> cells -> pos/vel/force double3 arrays (the pointer
            chain of Figure 1, many independent structures)
  broom  -- one served job: a chain of nodes ending in f leaf arrays
  random -- tiny random graphs with nulls, aliases, cycles and empty arrays
"""
from __future__ import annotations

import ctypes
import os
import random as _random
from dataclasses import dataclass, field
from typing import List, Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfx.so")

KINDS = {0: "struct", 1: "f32", 2: "f64", 3: "i32", 4: "i64", 5: "u8"}
KIND_CODE = {v: k for k, v in KINDS.items()}
ELEM_SIZE = {"f32": 4, "f64": 8, "i32": 4, "i64": 8, "u8": 1}

SHAPES = {"plain": 0, "linear": 1, "dense": 2, "wide": 3, "md": 4, "broom": 5}

# Seeds of the five workloads: 190601128 + i.
SEED_BASE = 190601128


@dataclass
class Field:
    offset: int
    kind: str           # "struct", "f32", "f64", ...
    type: int = 0       # pointee type index when kind == "struct"
    count_offset: int = -1
    count_bytes: int = 8
    count_mult: int = 1
    fixed_count: int = 0


@dataclass
class Type:
    name: str
    size: int
    align: int
    fields: List[Field] = field(default_factory=list)


class _CField(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_uint32), ("kind", ctypes.c_uint32), ("type", ctypes.c_uint32),
                ("count_offset", ctypes.c_int32), ("count_bytes", ctypes.c_uint32),
                ("count_mult", ctypes.c_uint32), ("fixed_count", ctypes.c_uint64)]


class _CType(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 16), ("size", ctypes.c_uint32), ("align", ctypes.c_uint32),
                ("nfields", ctypes.c_uint32), ("fields", _CField * 8)]


class _CAlloc(ctypes.Structure):
    _fields_ = [("base", ctypes.c_void_p), ("bytes", ctypes.c_uint64), ("kind", ctypes.c_uint32),
                ("pad", ctypes.c_uint32)]


class _CTree(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int), ("ntypes", ctypes.c_uint32), ("root_type", ctypes.c_uint32),
                ("types", _CType * 8), ("nroots", ctypes.c_uint64), ("roots", ctypes.POINTER(ctypes.c_void_p)),
                ("nallocs", ctypes.c_uint64), ("cap_allocs", ctypes.c_uint64),
                ("allocs", ctypes.POINTER(_CAlloc)), ("info", ctypes.c_int64 * 8)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"fixture library missing: {LIB_PATH} (run __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        lib.fx_build.restype = ctypes.POINTER(_CTree)
        lib.fx_build.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
        lib.fx_free.argtypes = [ctypes.POINTER(_CTree)]
        lib.fx_free.restype = None
        lib.fx_fill_f64.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64]
        lib.fx_fill_f32.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64]
        lib.fx_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


@dataclass
class Alloc:
    base: int
    bytes: int
    kind: str


class Tree:
    """A host tree: roots, the layout of every struct type, and every allocation."""

    def __init__(self):
        self.types: List[Type] = []
        self.root_type = 0
        self.roots: List[int] = []
        self.allocs: List[Alloc] = []
        self.info: List[int] = []
        self._c = None
        self._keep = []  # Python-owned memory of random trees

    # -- helpers for reading host memory -------------------------------------------
    def read(self, addr: int, nbytes: int) -> bytes:
        return ctypes.string_at(addr, nbytes) if nbytes else b""

    def leaf_allocs(self, kinds=("f32", "f64")) -> List[Alloc]:
        return [a for a in self.allocs if a.kind in kinds]

    def snapshot(self, kinds=("f32", "f64")) -> List[bytes]:
        return [self.read(a.base, a.bytes) for a in self.leaf_allocs(kinds)]

    def payload_bytes(self) -> int:
        return sum(a.bytes for a in self.allocs)

    def free(self):
        if self._c is not None:
            _load().fx_free(self._c)
            self._c = None
        self._keep = []

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build(shape: str, seed: int, params) -> Tree:
    """Builds one of the C-side shapes (see fx.h for the meaning of params)."""
    lib = _load()
    arr = (ctypes.c_int64 * max(1, len(params)))(*params)
    p = lib.fx_build(SHAPES[shape], seed, arr, len(params))
    if not p:
        raise MemoryError(f"fx_build({shape}) failed")
    c = p.contents
    t = Tree()
    t._c = p
    t.root_type = c.root_type
    for i in range(c.ntypes):
        ct = c.types[i]
        ty = Type(ct.name.decode(), ct.size, ct.align)
        for j in range(ct.nfields):
            f = ct.fields[j]
            ty.fields.append(Field(f.offset, KINDS[f.kind], f.type, f.count_offset, f.count_bytes,
                                   f.count_mult, f.fixed_count))
        t.types.append(ty)
    t.roots = [c.roots[i] for i in range(c.nroots)]
    allocs = ctypes.cast(c.allocs, ctypes.POINTER(_CAlloc * c.nallocs)).contents if c.nallocs else []
    t.allocs = [Alloc(a.base, a.bytes, KINDS[a.kind]) for a in allocs]
    t.info = list(c.info)
    return t


def set_threads(n: int):
    _load().fx_set_threads(n)


# ---- the five workloads -----------------------------------------------------------

def plain(seed=SEED_BASE + 0, nchild=16, leaf_len=1024) -> Tree:
    return build("plain", seed, [nchild, leaf_len])


def linear(seed=SEED_BASE + 1, k=8, n=1 << 24, scheme=1) -> Tree:
    """scheme 0: every level allocates n doubles; 1: only the last level does."""
    return build("linear", seed, [k, n, scheme])


def dense(seed=SEED_BASE, q=2, n=10, D=3, packed_last=0) -> Tree:
    return build("dense", seed, [q, n, D, packed_last])


def wide(seed=SEED_BASE + 2, f1=64, f2=64, lo=256, hi=65536) -> Tree:
    return build("wide", seed, [f1, f2, lo, hi])


def md(seed=SEED_BASE + 3, nsims=10000, cells_lo=8, cells_hi=512, mean_atoms=64) -> Tree:
    return build("md", seed, [nsims, cells_lo, cells_hi, mean_atoms])


def broom(seed=SEED_BASE + 4, d_lo=2, d_hi=8, f_lo=1, f_hi=64, bytes_lo=4096, bytes_hi=256 << 20) -> Tree:
    return build("broom", seed, [d_lo, d_hi, f_lo, f_hi, bytes_lo, bytes_hi])


# ---- tiny random graphs (Python-owned memory) ----------------------------------------
#
# Type 0 "A" (40 B): i32 na @0, i32 nb @4, A* next @8 (fixed 1), B* arr @16 (na),
#                    double* vals @24 (nb), i64 tag @32
# Type 1 "B" (24 B): i64 n @0, float* f @8 (2n), A* back @16 (fixed 1)
# The field lists name vals, next, arr and back, f: not in offset order.

RANDOM_TYPES = [
    # both field lists are deliberately out of offset order
    Type("A", 40, 8, [Field(24, "f64", 0, 4, 4, 1, 0), Field(8, "struct", 0, -1, 8, 1, 1),
                      Field(16, "struct", 1, 0, 4, 1, 0)]),
    Type("B", 24, 8, [Field(16, "struct", 0, -1, 8, 1, 1), Field(8, "f32", 0, 0, 8, 2, 0)]),
]


def random_tree(seed: int, max_objects: int = 7, p_null: float = 0.3, p_alias: float = 0.25,
                nroots: int = 1) -> Tree:
    """A random pointer graph of at most about max_objects allocations, with null
    pointers, aliases, cycles and zero-length arrays. Values come from the
    fixture stream. Memory is owned by the returned Tree."""
    rng = _random.Random(seed)
    t = Tree()
    t.types = RANDOM_TYPES
    t.root_type = 0
    budget = [max_objects]
    a_nodes: List[int] = []           # addresses of A structs (count 1 each)
    b_arrays: List[tuple] = []        # (addr, count)
    f64_arrays: List[tuple] = []      # (addr, count)

    def alloc(nbytes: int, kind: str) -> int:
        buf = ctypes.create_string_buffer(max(nbytes, 1))
        t._keep.append(buf)
        addr = ctypes.addressof(buf)
        t.allocs.append(Alloc(addr, nbytes, kind))
        budget[0] -= 1
        return addr

    def put(addr, off, fmt_bytes, val, signed=True):
        ctypes.memmove(addr + off, int(val).to_bytes(fmt_bytes, "little", signed=signed), fmt_bytes)

    def fill(addr, n, kind):
        lib = _load()
        s = rng.getrandbits(63)
        if kind == "f64":
            lib.fx_fill_f64(addr, n, s)
        else:
            lib.fx_fill_f32(addr, n, s)

    def new_a() -> int:
        a = alloc(40, "struct")
        a_nodes.append(a)
        put(a, 32, 8, rng.getrandbits(62))
        # vals
        if budget[0] > 0 and rng.random() > p_null:
            if f64_arrays and rng.random() < p_alias:
                v, nb = rng.choice(f64_arrays)
            else:
                nb = rng.choice([0, 1, 2, 3])
                v = alloc(8 * nb, "f64")
                fill(v, nb, "f64")
                f64_arrays.append((v, nb))
            put(a, 4, 4, nb)
            put(a, 24, 8, v, signed=False)
        else:
            put(a, 4, 4, rng.choice([0, 2]))  # count without an object: ignored
        # arr
        if budget[0] > 0 and rng.random() > p_null:
            if b_arrays and rng.random() < p_alias:
                b, na = rng.choice(b_arrays)
                put(a, 0, 4, na)
                put(a, 16, 8, b, signed=False)
            else:
                na = rng.choice([0, 1, 2])
                b = alloc(24 * na, "struct")
                b_arrays.append((b, na))
                put(a, 0, 4, na)
                put(a, 16, 8, b, signed=False)
                for e in range(na):
                    be = b + 24 * e
                    if budget[0] > 0 and rng.random() > p_null:
                        n = rng.choice([0, 1, 2])
                        f = alloc(4 * 2 * n, "f32")
                        fill(f, 2 * n, "f32")
                        put(be, 0, 8, n)
                        put(be, 8, 8, f, signed=False)
                    if a_nodes and rng.random() < 0.5:
                        put(be, 16, 8, rng.choice(a_nodes), signed=False)
        # next
        if budget[0] > 0 and rng.random() > p_null:
            if a_nodes and rng.random() < p_alias:
                put(a, 8, 8, rng.choice(a_nodes), signed=False)
            else:
                nxt = new_a()
                put(a, 8, 8, nxt, signed=False)
        return a

    for _ in range(nroots):
        t.roots.append(new_a())
    return t
