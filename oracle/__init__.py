"""CPU oracle for the deep copy and the leaf kernels (ctypes wrapper).

TEST INFRASTRUCTURE: only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import this package. It shares no code with the HIP path
(paper_1906_01128_amd); the two meet only in the seeded inputs of fixtures/.

The C source (oracle.c) says what each step computes and which part of the
paper it follows. Parity status: the walk/layout/copy/relocation, chain
resolution, kernel and copy back are pinned by tests/test_oracle_pins.py, the
selective walk by tests/test_selective.py, scalar chains by
tests/test_scalar_chain.py and the kick-drift update by
tests/test_kick_drift.py; nothing here is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB lets the mutation tests load a deliberately broken build
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

OR_KIND = {"struct": 0, "f32": 1, "f64": 2, "i32": 3, "i64": 4, "u8": 5}
OR_KIND_NAME = {v: k for k, v in OR_KIND.items()}
ERRORS = {0: "OK", -1: "INVAL", -2: "RANGE", -3: "CONFLICT", -4: "NOMEM"}


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {ERRORS.get(code, code)}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class _Field(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_uint32), ("kind", ctypes.c_uint32), ("type", ctypes.c_uint32),
                ("count_offset", ctypes.c_int32), ("count_bytes", ctypes.c_uint32),
                ("count_mult", ctypes.c_uint32), ("fixed_count", ctypes.c_uint64)]


class _Type(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("nfields", ctypes.c_uint32), ("fields", _Field * 16)]


class _Object(ctypes.Structure):
    _fields_ = [("host", ctypes.c_uint64), ("off", ctypes.c_uint64), ("bytes", ctypes.c_uint64),
                ("count", ctypes.c_uint64), ("kind", ctypes.c_uint32), ("type", ctypes.c_uint32)]


OBJECT_DTYPE = np.dtype([("host", "<u8"), ("off", "<u8"), ("bytes", "<u8"), ("count", "<u8"),
                         ("kind", "<u4"), ("type", "<u4")])

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH} (run __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        u64, u32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        lib.or_deep_copy.argtypes = [ctypes.POINTER(_Type), u32, u32, ctypes.POINTER(vp), u64, u64, u64,
                                     ctypes.POINTER(vp)]
        lib.or_deep_copy.restype = ctypes.c_int
        lib.or_deep_copy_selective.argtypes = [ctypes.POINTER(_Type), u32, u32, ctypes.POINTER(vp), u64, u64, u64,
                                               ctypes.POINTER(u32), ctypes.POINTER(vp)]
        lib.or_deep_copy_selective.restype = ctypes.c_int
        lib.or_free.argtypes = [vp]
        lib.or_free.restype = None
        lib.or_arena.argtypes = [vp]
        lib.or_arena.restype = vp
        for name in ("or_arena_bytes", "or_nobjects", "or_nslots", "or_payload_bytes"):
            getattr(lib, name).argtypes = [vp]
            getattr(lib, name).restype = u64
        lib.or_objects.argtypes = [vp]
        lib.or_objects.restype = vp
        lib.or_resolve_chain.argtypes = [vp, u64, ctypes.POINTER(u32), ctypes.POINTER(u64), u32,
                                         ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u32)]
        lib.or_resolve_chain.restype = ctypes.c_int
        lib.or_scalar_chain.argtypes = [vp, u64, ctypes.POINTER(u32), ctypes.POINTER(u64), u32, u32, u32,
                                        ctypes.POINTER(u64)]
        lib.or_scalar_chain.restype = ctypes.c_int
        lib.or_kick_drift.argtypes = [vp, u32, u32, u32, u32, u32, ctypes.c_double, ctypes.c_double]
        lib.or_kick_drift.restype = ctypes.c_int
        lib.or_run_kernel.argtypes = [vp, ctypes.c_int, u64, ctypes.POINTER(u32), ctypes.POINTER(u64), u32, u32,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_float, ctypes.c_float, vp, u64]
        lib.or_run_kernel.restype = ctypes.c_int
        lib.or_out_bytes.argtypes = [vp, ctypes.c_int, u64, ctypes.POINTER(u32), ctypes.POINTER(u64), u32]
        lib.or_out_bytes.restype = u64
        lib.or_copy_back.argtypes = [vp, ctypes.c_int]
        lib.or_copy_back.restype = ctypes.c_int
        lib.or_fma64.argtypes = [ctypes.c_double] * 3
        lib.or_fma64.restype = ctypes.c_double
        lib.or_fma32.argtypes = [ctypes.c_float] * 3
        lib.or_fma32.restype = ctypes.c_float
        _lib = lib
    return _lib


def make_types(types):
    """Converts a list of struct descriptions (objects with .size and .fields,
    each field with .offset .kind .type .count_offset .count_bytes .count_mult
    .fixed_count) into the oracle's type array."""
    arr = (_Type * len(types))()
    for i, t in enumerate(types):
        arr[i].size = t.size
        arr[i].nfields = len(t.fields)
        for j, f in enumerate(t.fields):
            cf = arr[i].fields[j]
            cf.offset = f.offset
            cf.kind = OR_KIND[f.kind]
            cf.type = f.type
            cf.count_offset = f.count_offset
            cf.count_bytes = f.count_bytes
            cf.count_mult = f.count_mult
            cf.fixed_count = f.fixed_count
    return arr


def _chain_arrays(chain):
    chain = list(chain or [])
    fields = (ctypes.c_uint32 * max(1, len(chain)))(*[int(f) for f, _ in chain])
    index = (ctypes.c_uint64 * max(1, len(chain)))(*[int(i) for _, i in chain])
    return fields, index, len(chain)


class OracleCopy:
    """The oracle's deep copy of a host tree, laid out as if at address `base`."""

    def __init__(self, types, root_type, roots, align=64, base=0, follow=None):
        """follow: None (every pointer member) or one bitmask per type over
        its field list (selective deep copy)."""
        lib = _load()
        self._types = make_types(types)
        self._roots = (ctypes.c_void_p * max(1, len(roots)))(*roots)
        h = ctypes.c_void_p()
        if follow is None:
            rc = lib.or_deep_copy(self._types, len(types), root_type, self._roots, len(roots), align, base,
                                  ctypes.byref(h))
        else:
            fm = (ctypes.c_uint32 * len(types))(*follow)
            rc = lib.or_deep_copy_selective(self._types, len(types), root_type, self._roots, len(roots), align,
                                            base, fm, ctypes.byref(h))
        if rc:
            raise OracleError(rc, "or_deep_copy")
        self._h = h
        self.base = base
        self.align = align

    @property
    def arena_bytes(self) -> int:
        return _load().or_arena_bytes(self._h)

    def arena(self) -> np.ndarray:
        """A view (no copy) of the oracle's buffer as uint8."""
        n = self.arena_bytes
        if n == 0:
            return np.zeros(0, np.uint8)
        ptr = _load().or_arena(self._h)
        return np.ctypeslib.as_array((ctypes.c_uint8 * n).from_address(ptr))

    def objects(self) -> np.ndarray:
        lib = _load()
        n = lib.or_nobjects(self._h)
        if n == 0:
            return np.zeros(0, OBJECT_DTYPE)
        ptr = lib.or_objects(self._h)
        raw = (ctypes.c_uint8 * (n * OBJECT_DTYPE.itemsize)).from_address(ptr)
        return np.frombuffer(bytes(raw), OBJECT_DTYPE).copy()

    @property
    def nslots(self) -> int:
        return _load().or_nslots(self._h)

    @property
    def payload_bytes(self) -> int:
        return _load().or_payload_bytes(self._h)

    def resolve_chain(self, root_index, chain):
        fields, index, n = _chain_arrays(chain)
        addr, count, kind = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint32()
        rc = _load().or_resolve_chain(self._h, root_index, fields, index, n, ctypes.byref(addr),
                                      ctypes.byref(count), ctypes.byref(kind))
        if rc:
            raise OracleError(rc, "or_resolve_chain")
        return addr.value, count.value, OR_KIND_NAME[kind.value]

    def scalar_chain(self, root_index, chain, offset, nbytes) -> int:
        """Buffer address (as laid out at `base`) of a scalar member reached
        by `chain` (struct steps only; empty for the root's own member)."""
        fields, index, n = _chain_arrays(chain)
        addr = ctypes.c_uint64()
        rc = _load().or_scalar_chain(self._h, root_index, fields, index, n, offset, nbytes, ctypes.byref(addr))
        if rc:
            raise OracleError(rc, "or_scalar_chain")
        return addr.value

    def out_bytes(self, select="all", root_index=0, chain=None) -> int:
        fields, index, n = _chain_arrays(chain)
        return _load().or_out_bytes(self._h, 1 if select == "all" else 0, root_index, fields, index, n)

    def run_kernel(self, a, b, iters=1, select="all", root_index=0, chain=None, out=None):
        """out: None (in place) or a writable numpy uint8 array."""
        fields, index, n = _chain_arrays(chain)
        af = float(np.float32(a))
        bf = float(np.float32(b))
        optr = out.ctypes.data if out is not None else None
        olen = out.nbytes if out is not None else 0
        rc = _load().or_run_kernel(self._h, 1 if select == "all" else 0, root_index, fields, index, n, iters,
                                   a, b, af, bf, optr, olen)
        if rc:
            raise OracleError(rc, "or_run_kernel")

    def kick_drift(self, type_id, x_field, v_field, f_field, dt, dt_over_m, steps=1):
        """v <- fma(f, dt_over_m, v); x <- fma(v, dt, x) per time step on every
        element of struct type `type_id`."""
        rc = _load().or_kick_drift(self._h, type_id, x_field, v_field, f_field, steps, dt, dt_over_m)
        if rc:
            raise OracleError(rc, "or_kick_drift")

    def copy_back(self, scalars=False):
        rc = _load().or_copy_back(self._h, 1 if scalars else 0)
        if rc:
            raise OracleError(rc, "or_copy_back")

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _load().or_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def fma64(x, a, b):
    return _load().or_fma64(x, a, b)


def fma32(x, a, b):
    return _load().or_fma32(x, a, b)
