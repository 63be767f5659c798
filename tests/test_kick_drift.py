"""The molecular-dynamics leaf kernel: kick then drift on the sibling
position, velocity and force arrays of every cell (the atoms-in-cells
structure of the pointerchain example, Section 3).

Oracle pins (CPU):
  * closed form: with fixed forces and dyadic inputs small enough that no
    operation rounds, s steps give v_s = v_0 + s c f and
    x_s = x_0 + dt (s v_0 + c f s(s+1)/2), c = dt/m. A drift that used the
    old velocity would give s(s-1)/2; swapped roles change every value;
  * one step against exactly rounded arithmetic (Fractions): each fma rounds
    once;
  * error cases: unequal counts, a partly null cell, a shared array, a field
    that is not FP64, the same field in two roles.
GPU (marked gpu): the C ABI against the oracle, bit for bit, on the MD
workload's shape and on hand-made cells with odd, zero and one-element counts.
"""
import ctypes
import random
from fractions import Fraction

import numpy as np
import pytest

import fixtures as fx
import oracle as orc
from tests import exact

BASE = 0x7F0000000000
CELL = 1                          # the MD cell type: natoms@0, pos@8, vel@16, force@24
X, V, F = 0, 1, 2                 # its fields in list order: pos, vel, force


def _f64_arrays(c):
    return [o for o in c.objects() if o["kind"] == 2]


def _set_host(o, values):
    arr = np.asarray(values, np.float64)
    assert arr.size == int(o["count"])
    ctypes.memmove(int(o["host"]), arr.ctypes.data, arr.nbytes)


def _cell_triples(t):
    """(pos, vel, force) object rows of every cell, from the full oracle copy."""
    c = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE)
    objs = c.objects()
    by_off = {int(o["off"]): o for o in objs}
    out = []
    ar = c.arena()
    for o in objs:
        if o["kind"] != 0 or o["type"] != CELL:
            continue
        for e in range(int(o["count"])):
            el = int(o["off"]) + 32 * e
            ptr = [int(ar[el + 8 * (1 + r): el + 8 * (2 + r)].view(np.uint64)[0]) for r in range(3)]
            if ptr[0] == 0:
                continue
            out.append(tuple(by_off[p - BASE] for p in ptr))
    return out


def _small_md(seed=31):
    return fx.md(seed=seed, nsims=6, cells_lo=1, cells_hi=9, mean_atoms=5)


@pytest.mark.parametrize("steps", [1, 2, 7])
def test_closed_form(steps):
    t = _small_md()
    rng = random.Random(steps)
    init = []
    for xo, vo, fo in _cell_triples(t):
        n = int(xo["count"])
        x0 = [rng.randrange(-64, 64) / 8 for _ in range(n)]
        v0 = [rng.randrange(-64, 64) / 16 for _ in range(n)]
        f0 = [rng.randrange(-64, 64) / 32 for _ in range(n)]
        _set_host(xo, x0), _set_host(vo, v0), _set_host(fo, f0)
        init.append((xo, vo, x0, v0, f0))
    dt, c1 = 0.125, 0.25
    c = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE)
    c.kick_drift(CELL, X, V, F, dt, c1, steps=steps)
    ar = c.arena()
    s = steps
    for xo, vo, x0, v0, f0 in init:
        xs = ar[int(xo["off"]): int(xo["off"]) + int(xo["bytes"])].view(np.float64)
        vs = ar[int(vo["off"]): int(vo["off"]) + int(vo["bytes"])].view(np.float64)
        for i in range(len(x0)):
            assert vs[i] == v0[i] + s * c1 * f0[i]
            want_x = Fraction(x0[i]) + Fraction(dt) * (s * Fraction(v0[i]) +
                                                       Fraction(c1) * Fraction(f0[i]) * s * (s + 1) / 2)
            assert Fraction(float(xs[i])) == want_x


def test_one_step_exact_rounding():
    t = _small_md(seed=32)
    dt, m = 1e-3, 39.948
    c1 = dt / m
    c = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE)
    before = c.arena().copy()
    c.kick_drift(CELL, X, V, F, dt, c1)
    ar = c.arena()
    checked = 0
    for xo, vo, fo in _cell_triples(t):
        def view(a, o):
            return a[int(o["off"]): int(o["off"]) + int(o["bytes"])].view(np.float64)
        x0, v0, f0 = view(before, xo), view(before, vo), view(before, fo)
        for i in range(len(x0)):
            v1 = exact.fma64(float(f0[i]), c1, float(v0[i]))
            x1 = exact.fma64(v1, dt, float(x0[i]))
            assert view(ar, vo)[i] == v1 and view(ar, xo)[i] == x1
            assert view(ar, fo)[i] == f0[i]
            checked += 1
    assert checked > 50


# ---- hand-made cells ---------------------------------------------------------------------

SIM = fx.Type("Sim", 16, 8, [fx.Field(8, "struct", 1, 0, 8, 1, 0)])
CELL3 = fx.Type("Cell3", 48, 8, [fx.Field(8, "f64", 0, 0, 8, 1, 0),     # x, count nx@0
                                 fx.Field(24, "f64", 0, 16, 8, 1, 0),    # v, count nv@16
                                 fx.Field(40, "f64", 0, 32, 8, 1, 0)])   # f, count nf@32


def make_cells(counts, seed=0, share=None, null=None, values=None):
    """A Sim with len(counts) Cell3 elements; counts[i] = (nx, nv, nf).
    share=(i, j): cell j's f is cell i's f. null: (i, role) pairs whose pointer
    is null. values: {(i, role): list} replaces the random contents."""
    t = fx.Tree()
    t.types = [SIM, CELL3]
    t.root_type = 0
    rng = np.random.default_rng(seed)
    cells = ctypes.create_string_buffer(48 * max(1, len(counts)))
    t._keep.append(cells)
    base = ctypes.addressof(cells)
    arrays = {}
    for i, cnt in enumerate(counts):
        for r, n in enumerate(cnt):
            vals = (values or {}).get((i, r))
            vals = rng.uniform(-1, 1, max(1, n)) if vals is None else vals
            buf = (ctypes.c_double * max(1, n))(*vals)
            t._keep.append(buf)
            arrays[(i, r)] = ctypes.addressof(buf)
    if share:
        arrays[(share[1], 2)] = arrays[(share[0], 2)]
    for i, cnt in enumerate(counts):
        for r, n in enumerate(cnt):
            p = 0 if (i, r) in (null or []) else arrays[(i, r)]
            ctypes.c_int64.from_address(base + 48 * i + 16 * r).value = n
            ctypes.c_uint64.from_address(base + 48 * i + 16 * r + 8).value = p
    sim = ctypes.create_string_buffer(16)
    t._keep.append(sim)
    ctypes.c_int64.from_address(ctypes.addressof(sim)).value = len(counts)
    ctypes.c_uint64.from_address(ctypes.addressof(sim) + 8).value = base
    t.roots = [ctypes.addressof(sim)]
    return t


def test_hand_made_cells_match_one_step_rounding():
    t = make_cells([(1, 1, 1), (2, 2, 2), (3, 3, 3), (0, 0, 0), (5, 5, 5)], seed=4)
    c = orc.OracleCopy(t.types, 0, t.roots, 64, BASE)
    before = c.arena().copy()
    c.kick_drift(1, 0, 1, 2, 0.5, 0.75)
    objs = [o for o in c.objects() if o["kind"] == 2]
    ar = c.arena()
    for k in range(0, len(objs), 3):
        xo, vo, fo = objs[k], objs[k + 1], objs[k + 2]
        for i in range(int(xo["count"])):
            def at(a, o):
                return float(a[int(o["off"]) + 8 * i: int(o["off"]) + 8 * i + 8].view(np.float64)[0])
            v1 = exact.fma64(at(before, fo), 0.75, at(before, vo))
            assert at(ar, vo) == v1
            assert at(ar, xo) == exact.fma64(v1, 0.5, at(before, xo))


def test_cancellation_exposes_single_rounding():
    """v0 = -(f c rounded) leaves, after a fused kick, exactly the product's
    rounding error; a separately rounded kick would leave 0. The same trick on
    x0 exposes the drift's single rounding."""
    rng = random.Random(12)
    c1, dt = 0.1, 0.3
    f = [rng.uniform(0.5, 2.0) for _ in range(16)]
    v = [-(fi * c1) for fi in f]                       # Python rounds the product once
    v1 = [exact.fma64(fi, c1, vi) for fi, vi in zip(f, v)]
    assert sum(1 for x in v1 if x != 0.0) >= 8         # the residuals are mostly nonzero
    x = [-(vi * dt) for vi in v1]
    t = make_cells([(16, 16, 16)], values={(0, 0): x, (0, 1): v, (0, 2): f})
    c = orc.OracleCopy(t.types, 0, t.roots, 64, BASE)
    c.kick_drift(1, 0, 1, 2, dt, c1)
    objs = [o for o in c.objects() if o["kind"] == 2]
    ar = c.arena()
    got_x = ar[int(objs[0]["off"]): int(objs[0]["off"]) + 128].view(np.float64)
    got_v = ar[int(objs[1]["off"]): int(objs[1]["off"]) + 128].view(np.float64)
    assert list(got_v) == v1
    assert list(got_x) == [exact.fma64(a, dt, b) for a, b in zip(v1, x)]


@pytest.mark.parametrize("case,err", [
    (dict(counts=[(3, 3, 4)]), "INVAL"),
    (dict(counts=[(3, 3, 3), (2, 2, 2)], null=[(1, 1)]), "INVAL"),
    (dict(counts=[(3, 3, 3), (3, 3, 3)], share=(0, 1)), "CONFLICT"),
])
def test_oracle_rejects(case, err):
    t = make_cells(**case)
    c = orc.OracleCopy(t.types, 0, t.roots, 64, BASE)
    with pytest.raises(orc.OracleError, match=err):
        c.kick_drift(1, 0, 1, 2, 0.5, 0.75)


def test_oracle_rejects_bad_fields():
    t = make_cells([(2, 2, 2)])
    c = orc.OracleCopy(t.types, 0, t.roots, 64, BASE)
    with pytest.raises(orc.OracleError):
        c.kick_drift(1, 0, 0, 2, 0.5, 0.75)      # x and v the same field
    with pytest.raises(orc.OracleError):
        c.kick_drift(0, 0, 0, 0, 0.5, 0.75)      # the Sim type has no FP64 fields


def test_all_null_cell_is_skipped():
    t = make_cells([(2, 2, 2), (4, 4, 4), (3, 3, 3)], null=[(1, 0), (1, 1), (1, 2)])
    c = orc.OracleCopy(t.types, 0, t.roots, 64, BASE)
    before = c.arena().copy()
    c.kick_drift(1, 0, 1, 2, 0.5, 0.75)
    objs = [o for o in c.objects() if o["kind"] == 2]
    assert len(objs) == 6
    changed = [not np.array_equal(c.arena()[int(o["off"]): int(o["off"]) + int(o["bytes"])],
                                  before[int(o["off"]): int(o["off"]) + int(o["bytes"])]) for o in objs]
    assert changed == [True, True, False] * 2   # x and v change, f does not


# ---- GPU ----------------------------------------------------------------------------------


def _gpu_copy(t):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_01128_amd import dc
    from tests.test_gpu_parity import Copy
    return Copy(dc.Context(0), t)


@pytest.mark.gpu
@pytest.mark.parametrize("steps", [1, 3])
def test_gpu_md_kick_drift(steps):
    from tests.test_gpu_parity import assert_same_bytes
    t = fx.md(seed=33, nsims=40, cells_lo=2, cells_hi=60, mean_atoms=11)
    c = _gpu_copy(t)
    dt, m = 1e-3, 39.948
    c.tree.kick_drift(CELL, X, V, F, dt, dt / m, steps=steps)
    c.oracle.kick_drift(CELL, X, V, F, dt, dt / m, steps=steps)
    assert_same_bytes(c.device_arena(), c.oracle.arena(), f"kick-drift x{steps}")
    c.tree.check()
    # the cached element list serves the next call
    c.tree.kick_drift(CELL, X, V, F, dt, dt / m, steps=1)
    c.oracle.kick_drift(CELL, X, V, F, dt, dt / m, steps=1)
    assert_same_bytes(c.device_arena(), c.oracle.arena(), "kick-drift again")


@pytest.mark.gpu
def test_gpu_ragged_cells():
    from tests.test_gpu_parity import assert_same_bytes
    counts = [(n, n, n) for n in [1, 2, 3, 0, 5, 8191, 8192, 8193, 1, 0, 7]]
    t = make_cells(counts, seed=8)
    c = _gpu_copy(t)
    c.tree.kick_drift(1, 0, 1, 2, 0.5, 0.75, steps=2)
    c.oracle.kick_drift(1, 0, 1, 2, 0.5, 0.75, steps=2)
    assert_same_bytes(c.device_arena(), c.oracle.arena(), "ragged cells")


@pytest.mark.gpu
def test_gpu_kick_drift_errors():
    from paper_1906_01128_amd import dc
    for case in [dict(counts=[(3, 3, 4)]), dict(counts=[(3, 3, 3), (2, 2, 2)], null=[(1, 1)]),
                 dict(counts=[(3, 3, 3), (3, 3, 3)], share=(0, 1))]:
        c = _gpu_copy(make_cells(**case))
        with pytest.raises(dc.DcError):
            c.tree.kick_drift(1, 0, 1, 2, 0.5, 0.75)
    c = _gpu_copy(make_cells([(2, 2, 2)]))
    with pytest.raises(dc.DcError):
        c.tree.kick_drift(1, 0, 0, 2, 0.5, 0.75)
    with pytest.raises(dc.DcError):
        c.tree.kick_drift(0, 0, 0, 0, 0.5, 0.75)
    with pytest.raises(dc.DcError):
        c.tree.kick_drift(7, 0, 1, 2, 0.5, 0.75)
