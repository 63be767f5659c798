"""Python binding of libdc (include/dc.h): argument marshalling only.

Every step of the deep copy, relocation, chain resolution and leaf kernels
runs inside libdc.so (HIP for gfx950). PyTorch supplies device memory (the
arena, scratch and output buffers are torch uint8 tensors) and streams. There
is no CPU fallback: if the library is missing, importing this module fails.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libdc.so")

OK, E_INVAL, E_RANGE, E_CONFLICT, E_NOMEM, E_HIP, E_STATE, E_BUDGET = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "OK", -1: "INVAL", -2: "RANGE", -3: "CONFLICT", -4: "NOMEM", -5: "HIP", -6: "STATE",
                -7: "BUDGET"}
KIND = {"struct": 0, "f32": 1, "f64": 2, "i32": 3, "i64": 4, "u8": 5}
KIND_NAME = {v: k for k, v in KIND.items()}
MODE = {"resolved": 0, "deref_each": 1}
SELECT = {"chain": 0, "all": 1}
NOALLOC_SCRATCH_BYTES = 64 << 20   # DC_NOALLOC_SCRATCH_BYTES of include/dc.h
COPY_LEAVES, COPY_SCALARS = 1, 2
BATCH_ATTACH, BATCH_DETACH, BATCH_FORCE_WAIT_BOUND = 1, 2, 4

u32, u64, i32, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p


class DcError(RuntimeError):
    def __init__(self, status: int, where: str, text: str):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: DC_E_{self.name}: {text}")


class Field(ctypes.Structure):
    _fields_ = [("offset", u32), ("kind", u32), ("type_id", u32), ("count_offset", i32), ("count_bytes", u32),
                ("count_mult", u32), ("fixed_count", u64)]


class Step(ctypes.Structure):
    _fields_ = [("field", u32), ("reserved", u32), ("index", u64)]


class Chain(ctypes.Structure):
    _fields_ = [("dev_addr", u64), ("count", u64), ("kind", u32), ("reserved", u32)]


class ScalarRef(ctypes.Structure):
    _fields_ = [("root_index", ctypes.c_uint64), ("steps", ctypes.c_void_p), ("nsteps", ctypes.c_uint32),
                ("offset", ctypes.c_uint32), ("bytes", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class KickDriftArgs(ctypes.Structure):
    _fields_ = [("type", ctypes.c_uint32), ("x_field", ctypes.c_uint32), ("v_field", ctypes.c_uint32),
                ("f_field", ctypes.c_uint32), ("steps", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("dt", ctypes.c_double), ("dt_over_m", ctypes.c_double)]


class Object(ctypes.Structure):
    _fields_ = [("host_addr", u64), ("offset", u64), ("bytes", u64), ("count", u64), ("kind", u32), ("type_id", u32)]


OBJECT_DTYPE = np.dtype([("host", "<u8"), ("off", "<u8"), ("bytes", "<u8"), ("count", "<u8"), ("kind", "<u4"),
                         ("type", "<u4")])


class PlanInfo(ctypes.Structure):
    _fields_ = [(n, u64) for n in ("nobjects", "nslots", "nslots_nonnull", "nleaves", "payload_bytes", "leaf_bytes",
                                   "arena_bytes", "scratch_bytes", "out_bytes", "nsegments", "nroots",
                                   "unit_leaves", "max_unit_leaf_bytes", "leaf_prefix_offset")]


class KernelArgs(ctypes.Structure):
    _fields_ = [("mode", u32), ("select", u32), ("iters", u32), ("nsteps", u32), ("a", ctypes.c_double),
                ("b", ctypes.c_double), ("af", ctypes.c_float), ("bf", ctypes.c_float), ("root_index", u64),
                ("chain", ctypes.POINTER(Step)), ("d_out", vp), ("out_bytes", u64)]


class Tune(ctypes.Structure):
    _fields_ = [("block", u32), ("wg_per_cu", u32), ("tile_chunks", u32), ("launches", u32), ("spin_limit", u32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", u64), ("max_inflight", u32), ("nstreams", u32), ("align", u64),
                ("fail_copy_at", u32), ("reserved", u32)]


class Request(ctypes.Structure):
    _fields_ = [("root_type", u32), ("reserved", u32), ("root", vp), ("key", u64), ("a", ctypes.c_double),
                ("b", ctypes.c_double), ("af", ctypes.c_float), ("bf", ctypes.c_float), ("out_host", vp),
                ("out_bytes", u64)]


class Result(ctypes.Structure):
    _fields_ = [("id", u64), ("status", i32), ("reused", u32), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("out_bytes", u64)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, u64) for n in ("submitted", "completed", "reused", "evictions", "batches", "h2d_bytes",
                                   "d2h_bytes", "kernel_bytes", "resident_bytes", "peak_bytes")]


# (name, argtypes) of every exported call; all return dc_status unless noted
_SIGS = {
    "dc_ctx_create": [ctypes.c_int, ctypes.POINTER(vp)],
    "dc_ctx_destroy": [vp],
    "dc_schema_create": [ctypes.POINTER(vp)],
    "dc_schema_destroy": [vp],
    "dc_schema_describe": [vp, ctypes.c_char_p, u32, u32, ctypes.POINTER(Field), u32, ctypes.POINTER(u32)],
    "dc_plan_create": [vp, vp, u32, ctypes.POINTER(vp), u64, u64, ctypes.POINTER(vp), ctypes.POINTER(u64),
                       ctypes.POINTER(u64)],
    "dc_plan_create_selective": [vp, vp, u32, ctypes.POINTER(vp), u64, u64, ctypes.POINTER(u32), u32,
                                 ctypes.POINTER(vp), ctypes.POINTER(u64), ctypes.POINTER(u64)],
    "dc_plan_destroy": [vp],
    "dc_plan_query": [vp, ctypes.POINTER(PlanInfo)],
    "dc_plan_objects": [vp, ctypes.POINTER(Object), u64, ctypes.POINTER(u64)],
    "dc_deep_copy_to_device": [vp, vp, vp, u64, vp, u64, vp, ctypes.POINTER(vp)],
    "dc_stage_to_device": [vp, vp, vp, u64, vp, u64, vp, ctypes.POINTER(vp)],
    "dc_deep_copy_to_device_noalloc": [vp, vp, vp, u64, vp, ctypes.POINTER(vp)],
    "dc_attach": [vp, vp],
    "dc_detach": [vp, vp],
    "dc_resolve_chain": [vp, u64, ctypes.POINTER(Step), u32, vp, ctypes.POINTER(Chain)],
    "dc_chain_query": [vp, u32, vp, ctypes.POINTER(Step), u32, ctypes.POINTER(Chain)],
    "dc_chain_to_device": [vp, vp, u32, vp, ctypes.POINTER(Step), u32, vp, u64, vp, ctypes.POINTER(Chain)],
    "dc_chain_run_kernel": [vp, ctypes.POINTER(Chain), u32, ctypes.c_double, ctypes.c_double, ctypes.c_float,
                            ctypes.c_float, vp],
    "dc_chain_copy_back": [vp, vp, u32, vp, ctypes.POINTER(Step), u32, ctypes.POINTER(Chain), vp],
    "dc_scalar_declare": [vp, ctypes.POINTER(ScalarRef), u32, vp, vp],
    "dc_scalar_update": [vp, ctypes.POINTER(ScalarRef), u32, vp, vp],
    "dc_run_kick_drift": [vp, ctypes.POINTER(KickDriftArgs), vp],
    "dc_run_kernel": [vp, ctypes.POINTER(KernelArgs), vp],
    "dc_out_bytes": [vp, ctypes.POINTER(KernelArgs), ctypes.POINTER(u64)],
    "dc_copy_back": [vp, u32, vp],
    "dc_tree_release": [vp],
    "dc_tree_check": [vp, vp],
    "dc_tree_objects": [vp, ctypes.POINTER(Object), u64, ctypes.POINTER(u64)],
    "dc_batch_run": [vp, ctypes.POINTER(KernelArgs), ctypes.POINTER(Tune), u32, vp],
    "dc_autotune": [vp, ctypes.POINTER(KernelArgs), u32, ctypes.POINTER(Tune)],
    "dc_autotune_results": [vp, ctypes.POINTER(Tune), ctypes.POINTER(ctypes.c_double), u32, ctypes.POINTER(u32)],
    "dc_graph_create": [vp, ctypes.POINTER(KernelArgs), ctypes.POINTER(Tune), u32, ctypes.c_int, ctypes.c_int,
                        ctypes.POINTER(vp)],
    "dc_graph_launch": [vp, vp],
    "dc_graph_image": [vp, ctypes.POINTER(vp), ctypes.POINTER(u64)],
    "dc_graph_destroy": [vp],
    "dc_server_create": [vp, vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)],
    "dc_server_submit": [vp, ctypes.POINTER(Request), ctypes.POINTER(u64)],
    "dc_server_wait": [vp, u64, ctypes.c_double, ctypes.POINTER(Result)],
    "dc_server_stats_get": [vp, ctypes.POINTER(ServerStats)],
    "dc_server_destroy": [vp],
}

_lib = None


def load():
    """Loads libdc.so; raises if it is missing (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libdc.so not built: {LIB_PATH} (run python -m paper_1906_01128_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, argtypes in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = argtypes
            fn.restype = ctypes.c_int32
        lib.dc_last_error.restype = ctypes.c_char_p
        lib.dc_last_error.argtypes = []
        lib.dc_version.restype = ctypes.c_char_p
        lib.dc_version.argtypes = []
        _lib = lib
    return _lib


def _check(st: int, where: str):
    if st != OK:
        raise DcError(st, where, load().dc_last_error().decode(errors="replace"))


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev_ptr(t) -> int:
    return t.data_ptr()


def steps_array(chain: Sequence[Tuple[int, int]]):
    arr = (Step * max(1, len(chain)))()
    for i, (f, idx) in enumerate(chain):
        arr[i].field = int(f)
        arr[i].index = int(idx)
    return arr


class Context:
    def __init__(self, device: int = 0):
        h = vp()
        _check(load().dc_ctx_create(device, ctypes.byref(h)), "dc_ctx_create")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load().dc_ctx_destroy(self.h)
            self.h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Schema:
    """Struct types: describe(name, size, align, fields) with fields given as
    objects or dicts carrying offset, kind, type, count_offset, count_bytes,
    count_mult and fixed_count."""

    def __init__(self, types: Iterable = ()):
        h = vp()
        _check(load().dc_schema_create(ctypes.byref(h)), "dc_schema_create")
        self.h = h
        for t in types:
            self.describe(t.name, t.size, t.align, t.fields)

    def describe(self, name: str, size: int, align: int, fields) -> int:
        arr = (Field * max(1, len(fields)))()
        for i, f in enumerate(fields):
            g = (lambda k: f[k]) if isinstance(f, dict) else (lambda k: getattr(f, k))
            arr[i].offset = g("offset")
            kind = g("kind")
            arr[i].kind = KIND[kind] if isinstance(kind, str) else int(kind)
            arr[i].type_id = g("type")
            arr[i].count_offset = g("count_offset")
            arr[i].count_bytes = g("count_bytes")
            arr[i].count_mult = g("count_mult")
            arr[i].fixed_count = g("fixed_count")
        tid = u32()
        _check(load().dc_schema_describe(self.h, name.encode(), size, align, arr, len(fields), ctypes.byref(tid)),
               f"dc_schema_describe({name})")
        return tid.value

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load().dc_schema_destroy(self.h)
            self.h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    def __init__(self, schema: Schema, root_type: int, roots: Sequence[int], align: int = 64,
                 ctx: Optional[Context] = None, follow: Optional[Sequence[int]] = None):
        """follow: None, or one bitmask per type over its field list (a
        selective deep copy follows only the set fields)."""
        self._roots = (vp * max(1, len(roots)))(*roots)
        h, ab, sb = vp(), u64(), u64()
        if follow is None:
            _check(load().dc_plan_create(ctx.h if ctx else None, schema.h, root_type, self._roots, len(roots),
                                         align, ctypes.byref(h), ctypes.byref(ab), ctypes.byref(sb)),
                   "dc_plan_create")
        else:
            fm = (u32 * max(1, len(follow)))(*follow)
            _check(load().dc_plan_create_selective(ctx.h if ctx else None, schema.h, root_type, self._roots,
                                                   len(roots), align, fm, len(follow), ctypes.byref(h),
                                                   ctypes.byref(ab), ctypes.byref(sb)), "dc_plan_create_selective")
        self.h = h
        self.schema = schema
        self.arena_bytes = ab.value
        self.scratch_bytes = sb.value
        self.align = align

    def info(self) -> PlanInfo:
        pi = PlanInfo()
        _check(load().dc_plan_query(self.h, ctypes.byref(pi)), "dc_plan_query")
        return pi

    def objects(self) -> np.ndarray:
        n = u64()
        _check(load().dc_plan_objects(self.h, None, 0, ctypes.byref(n)), "dc_plan_objects")
        arr = (Object * max(1, n.value))()
        _check(load().dc_plan_objects(self.h, arr, n.value, ctypes.byref(n)), "dc_plan_objects")
        return np.frombuffer(bytes(arr), OBJECT_DTYPE, count=n.value).copy()

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load().dc_plan_destroy(self.h)
            self.h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _kargs(mode="resolved", select="all", iters=1, a=1.0, b=0.0, af=None, bf=None, root_index=0, chain=(),
           out=None):
    import numpy as _np
    ka = KernelArgs()
    ka.mode = MODE[mode] if isinstance(mode, str) else mode
    ka.select = SELECT[select] if isinstance(select, str) else select
    ka.iters = iters
    ka.a = a
    ka.b = b
    ka.af = float(_np.float32(a)) if af is None else af
    ka.bf = float(_np.float32(b)) if bf is None else bf
    ka.root_index = root_index
    steps = steps_array(chain)
    ka.chain = ctypes.cast(steps, ctypes.POINTER(Step))
    ka.nsteps = len(chain)
    if out is not None:
        ka.d_out = _dev_ptr(out)
        ka.out_bytes = out.numel() * out.element_size()
    ka._steps = steps  # keep alive
    return ka


class Tree:
    """A deep-copied tree on the device (the arena and scratch tensors are the
    caller's and are kept referenced here)."""

    def __init__(self, ctx: Context, plan: Plan, arena, scratch, stream=None, relocate: bool = True):
        h = vp()
        fn = load().dc_deep_copy_to_device if relocate else load().dc_stage_to_device
        _check(fn(ctx.h, plan.h, _dev_ptr(arena), arena.numel(), _dev_ptr(scratch), scratch.numel(),
                  _stream_ptr(stream), ctypes.byref(h)), "dc_deep_copy_to_device" if relocate else "dc_stage_to_device")
        self.h = h
        self.ctx, self.plan, self.arena, self.scratch = ctx, plan, arena, scratch

    @classmethod
    def noalloc(cls, ctx: Context, plan: Plan, arena, stream=None) -> "Tree":
        """dc_deep_copy_to_device_noalloc: the deep copy with the relocation
        tables in the library's fixed per-device array (no scratch tensor)."""
        h = vp()
        _check(load().dc_deep_copy_to_device_noalloc(ctx.h, plan.h, _dev_ptr(arena), arena.numel(),
                                                     _stream_ptr(stream), ctypes.byref(h)),
               "dc_deep_copy_to_device_noalloc")
        self = cls.__new__(cls)
        self.h = h
        self.ctx, self.plan, self.arena, self.scratch = ctx, plan, arena, None
        return self

    def attach(self, stream=None):
        _check(load().dc_attach(self.h, _stream_ptr(stream)), "dc_attach")

    def detach(self, stream=None):
        _check(load().dc_detach(self.h, _stream_ptr(stream)), "dc_detach")

    def resolve_chain(self, chain, root_index=0, stream=None):
        steps = steps_array(chain)
        out = Chain()
        _check(load().dc_resolve_chain(self.h, root_index, steps, len(chain), _stream_ptr(stream),
                                       ctypes.byref(out)), "dc_resolve_chain")
        return out.dev_addr, out.count, KIND_NAME[out.kind]

    def run_kernel(self, stream=None, **kw):
        ka = _kargs(**kw)
        _check(load().dc_run_kernel(self.h, ctypes.byref(ka), _stream_ptr(stream)), "dc_run_kernel")

    def out_bytes(self, **kw) -> int:
        ka = _kargs(**kw)
        n = u64()
        _check(load().dc_out_bytes(self.h, ctypes.byref(ka), ctypes.byref(n)), "dc_out_bytes")
        return n.value

    def copy_back(self, leaves=True, scalars=False, stream=None):
        flags = (COPY_LEAVES if leaves else 0) | (COPY_SCALARS if scalars else 0)
        _check(load().dc_copy_back(self.h, flags, _stream_ptr(stream)), "dc_copy_back")

    def check(self, stream=None):
        _check(load().dc_tree_check(self.h, _stream_ptr(stream)), "dc_tree_check")

    def objects(self) -> np.ndarray:
        """The plan's objects with `off` holding each object's device address."""
        n = u64()
        _check(load().dc_tree_objects(self.h, None, 0, ctypes.byref(n)), "dc_tree_objects")
        arr = (Object * max(1, n.value))()
        _check(load().dc_tree_objects(self.h, arr, n.value, ctypes.byref(n)), "dc_tree_objects")
        return np.frombuffer(bytes(arr), OBJECT_DTYPE, count=n.value).copy()

    def kick_drift(self, type_id, x_field, v_field, f_field, dt, dt_over_m, steps=1, stream=None):
        """v <- fma(f, dt_over_m, v); x <- fma(v, dt, x) per step on every
        element of struct type `type_id`."""
        ka = KickDriftArgs(type_id, x_field, v_field, f_field, steps, 0, dt, dt_over_m)
        _check(load().dc_run_kick_drift(self.h, ctypes.byref(ka), _stream_ptr(stream)), "dc_run_kick_drift")

    @staticmethod
    def _scalar_refs(refs):
        """refs: (root_index, chain, offset, nbytes) tuples; chain as for
        resolve_chain, each step landing on an element."""
        arr = (ScalarRef * max(1, len(refs)))()
        keep = []
        for i, (root, chain, off, nb) in enumerate(refs):
            st = steps_array(chain)
            keep.append(st)
            arr[i].root_index, arr[i].steps = root, ctypes.cast(st, ctypes.c_void_p)
            arr[i].nsteps, arr[i].offset, arr[i].bytes = len(chain), off, nb
        return arr, keep

    def scalar_declare(self, refs, temps, stream=None):
        """Copies each scalar into temps (a device tensor of 8 bytes per ref)."""
        arr, _keep = self._scalar_refs(refs)
        _check(load().dc_scalar_declare(self.h, arr, len(refs), _dev_ptr(temps), _stream_ptr(stream)),
               "dc_scalar_declare")

    def scalar_update(self, refs, temps, stream=None):
        """Writes temps back through each chain."""
        arr, _keep = self._scalar_refs(refs)
        _check(load().dc_scalar_update(self.h, arr, len(refs), _dev_ptr(temps), _stream_ptr(stream)),
               "dc_scalar_update")

    def batch_run(self, a=1.0001, b=0.5, tune=None, attach=True, detach=False, out=None, stream=None,
                  force_wait_bound=False):
        """force_wait_bound: the error path of the persistent launch's waits
        (tests only; see DC_BATCH_FORCE_WAIT_BOUND)."""
        ka = _kargs(mode="resolved", select="all", iters=1, a=a, b=b, out=out)
        tu = _tune(tune)
        flags = ((BATCH_ATTACH if attach else 0) | (BATCH_DETACH if detach else 0) |
                 (BATCH_FORCE_WAIT_BOUND if force_wait_bound else 0))
        _check(load().dc_batch_run(self.h, ctypes.byref(ka), ctypes.byref(tu) if tu else None, flags,
                                   _stream_ptr(stream)), "dc_batch_run")

    def autotune(self, a=1.0001, b=0.5, reps=3) -> dict:
        ka = _kargs(mode="resolved", select="all", iters=1, a=a, b=b)
        tu = Tune()
        _check(load().dc_autotune(self.h, ctypes.byref(ka), reps, ctypes.byref(tu)), "dc_autotune")
        return {"block": tu.block, "wg_per_cu": tu.wg_per_cu, "tile_chunks": tu.tile_chunks,
                "launches": tu.launches}

    def autotune_results(self) -> list:
        """The candidates the last autotune timed: (shape, median microseconds)."""
        n = u32()
        _check(load().dc_autotune_results(self.h, None, None, 0, ctypes.byref(n)), "dc_autotune_results")
        tunes = (Tune * max(n.value, 1))()
        us = (ctypes.c_double * max(n.value, 1))()
        _check(load().dc_autotune_results(self.h, tunes, us, n.value, ctypes.byref(n)), "dc_autotune_results")
        return [({"block": t.block, "wg_per_cu": t.wg_per_cu, "tile_chunks": t.tile_chunks,
                  "launches": t.launches}, us[i]) for i, t in enumerate(tunes[: n.value])]

    def graph(self, a=1.0001, b=0.5, tune=None, upload=False, download=False, out=None) -> "Graph":
        return Graph(self, a, b, tune, upload, download, out)

    def release(self):
        if getattr(self, "h", None) and self.h.value:
            load().dc_tree_release(self.h)
            self.h = vp()

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


ELEM_BYTES = {1: 4, 2: 8, 3: 4, 4: 8, 5: 1}


def chain_query(schema: Schema, root_type: int, root: int, chain) -> Chain:
    """Count and kind of the host array a chain ends in."""
    c = Chain()
    _check(load().dc_chain_query(schema.h, root_type, root, steps_array(chain), len(chain), ctypes.byref(c)),
           "dc_chain_query")
    return c


class ChainCopy:
    """The pointerchain transfer scheme: only the array at the end of a chain
    is copied to the device (into `buf`, a torch uint8 device tensor)."""

    def __init__(self, ctx: Context, schema: Schema, root_type: int, root: int, chain, buf=None, stream=None):
        """buf None: a device buffer of the array's size is allocated here."""
        self._steps = steps_array(chain)
        self._n = len(chain)
        if buf is None:
            q = chain_query(schema, root_type, root, chain)
            import torch
            buf = torch.empty(max(16, (q.count * ELEM_BYTES[q.kind] + 15) // 16 * 16), dtype=torch.uint8,
                              device="cuda")
        self.ctx, self.schema, self.root_type, self.root, self.buf = ctx, schema, root_type, root, buf
        self.c = Chain()
        _check(load().dc_chain_to_device(ctx.h, schema.h, root_type, root, self._steps, self._n, _dev_ptr(buf),
                                         buf.numel(), _stream_ptr(stream), ctypes.byref(self.c)),
               "dc_chain_to_device")

    @property
    def count(self):
        return self.c.count

    @property
    def kind(self):
        return KIND_NAME[self.c.kind]

    def run_kernel(self, iters=1, a=1.0, b=0.0, af=None, bf=None, stream=None):
        af = float(np.float32(a)) if af is None else af
        bf = float(np.float32(b)) if bf is None else bf
        _check(load().dc_chain_run_kernel(self.ctx.h, ctypes.byref(self.c), iters, a, b, af, bf,
                                          _stream_ptr(stream)), "dc_chain_run_kernel")

    def copy_back(self, stream=None):
        _check(load().dc_chain_copy_back(self.ctx.h, self.schema.h, self.root_type, self.root, self._steps,
                                         self._n, ctypes.byref(self.c), _stream_ptr(stream)), "dc_chain_copy_back")


def _tune(tune):
    if tune is None:
        return None
    tu = Tune()
    tu.block = tune.get("block", 0)
    tu.wg_per_cu = tune.get("wg_per_cu", 0)
    tu.tile_chunks = tune.get("tile_chunks", 0)
    tu.launches = tune.get("launches", 0)
    tu.spin_limit = tune.get("spin_limit", 0)
    return tu


class Graph:
    def __init__(self, tree: Tree, a, b, tune, upload, download, out):
        self.tree = tree
        ka = _kargs(mode="resolved", select="all", iters=1, a=a, b=b, out=out)
        tu = _tune(tune)
        h = vp()
        _check(load().dc_graph_create(tree.h, ctypes.byref(ka), ctypes.byref(tu) if tu else None,
                                      BATCH_ATTACH | BATCH_DETACH, int(upload), int(download), ctypes.byref(h)),
               "dc_graph_create")
        self.h = h

    def launch(self, stream=None):
        _check(load().dc_graph_launch(self.h, _stream_ptr(stream)), "dc_graph_launch")

    def image(self) -> np.ndarray:
        """A copy of the arena as the last replay brought it back (a graph
        captured with download=True; synchronize with the replay's stream first)."""
        host, n = vp(), u64()
        _check(load().dc_graph_image(self.h, ctypes.byref(host), ctypes.byref(n)), "dc_graph_image")
        if n.value == 0:
            return np.zeros(0, np.uint8)
        return np.frombuffer((ctypes.c_uint8 * n.value).from_address(host.value), np.uint8).copy()

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load().dc_graph_destroy(self.h)
            self.h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching deep-copy+kernel server (see dc_server_* in dc.h)."""

    def __init__(self, ctx: Context, schema: Schema, budget_bytes: int, max_inflight: int = 8, nstreams: int = 4,
                 align: int = 64, fail_copy_at: int = 0):
        """fail_copy_at: tests of the error path only (dc_server_config)."""
        cfg = ServerConfig(budget_bytes, max_inflight, nstreams, align, fail_copy_at, 0)
        h = vp()
        _check(load().dc_server_create(ctx.h, schema.h, ctypes.byref(cfg), ctypes.byref(h)), "dc_server_create")
        self.h = h
        self.ctx, self.schema = ctx, schema

    def submit(self, root_type: int, root: int, out_host: int, out_bytes: int, a: float, b: float, key: int = 0,
               af=None, bf=None) -> int:
        r = Request()
        r.root_type = root_type
        r.root = root
        r.key = key
        r.a, r.b = a, b
        r.af = float(np.float32(a)) if af is None else af
        r.bf = float(np.float32(b)) if bf is None else bf
        r.out_host = out_host
        r.out_bytes = out_bytes
        rid = u64()
        _check(load().dc_server_submit(self.h, ctypes.byref(r), ctypes.byref(rid)), "dc_server_submit")
        return rid.value

    def wait(self, rid: int, timeout: float = -1.0) -> Result:
        res = Result()
        _check(load().dc_server_wait(self.h, rid, timeout, ctypes.byref(res)), "dc_server_wait")
        return res

    def stats(self) -> ServerStats:
        st = ServerStats()
        _check(load().dc_server_stats_get(self.h, ctypes.byref(st)), "dc_server_stats_get")
        return st

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            _check(load().dc_server_destroy(self.h), "dc_server_destroy")
            self.h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version() -> str:
    return load().dc_version().decode()
