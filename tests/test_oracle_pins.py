"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
not by the oracle itself.

  * payload bytes of the paper's Linear and Dense trees against Equations
    (1)-(3) and every cell of Tables 1 and 2 (Section 4, Section 6);
  * hand-derived layouts of the plain and Linear workloads;
  * brute-force pointer-graph isomorphism on tiny random graphs (deep copy =
    the same graph, Figure 2 steps a-d);
  * invariants: relocated pointers land on object starts inside the buffer,
    leaf bytes conserved, chain depth preserved, aligned non-overlapping
    objects in depth-first pre-order with zero padding, nulls and aliases kept;
  * the kernel's rounding against exact rational arithmetic, special cases,
    and 100 passes against 100 exactly rounded steps;
  * chain resolution (Section 3) and copy back (Algorithm 2 step 5).
"""
import ctypes
import math
import os
import random
import struct

import numpy as np
import pytest

import fixtures as fx
import oracle as orc
from tests import exact, graphs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
UNITS = {"KB": 1024, "MB": 1024 ** 2, "GB": 1024 ** 3}
BASE = 0x7F3200000000


def copy_of(t, align=64, base=BASE):
    return orc.OracleCopy(t.types, t.root_type, t.roots, align, base)


# ---------------------------------------------------------------- sizes ------------

def _table(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        if line.strip() and not line.startswith("#"):
            rows.append(line.split())
    return rows


def eq1(k, n):  # Equation (1), allinit: sum over k levels of (24 + 8n)
    return 24 * k + 8 * n * k


def eq2(k, n):  # Equation (2), LLinit: k nodes plus one payload
    return 24 * k + 8 * n


def eq3(q, n, D):  # Equation (3), Dense, 12-byte last level
    return 12 + 8 * n if D == 0 else 24 + 8 * n + q * eq3(q, n, D - 1)


@pytest.mark.parametrize("k", range(2, 11))
def test_linear_allinit_payload_matches_eq1_and_table1(k):
    for row in _table("table1_linear_sizes.txt"):
        n, unit, cells = int(row[0]), row[1], row[2:]
        printed = cells[k - 2]
        assert f"{eq1(k, n) / UNITS[unit]:.2f}" == printed
        if n <= 100000:
            t = fx.linear(seed=11, k=k, n=n, scheme=0)
            c = copy_of(t)
            assert c.payload_bytes == eq1(k, n)
            assert f"{c.payload_bytes / UNITS[unit]:.2f}" == printed
            assert c.nslots == (k - 1) + k  # k-1 next pointers, k payload pointers


@pytest.mark.parametrize("k", [2, 5, 8, 10])
def test_linear_llinit_payload_matches_eq2(k):
    for n in (0, 1, 100, 4096):
        t = fx.linear(seed=12, k=k, n=n, scheme=1)
        c = copy_of(t)
        assert c.payload_bytes == eq2(k, n)
        assert c.nslots == k  # k-1 next pointers and the last payload pointer


def test_dense_payload_matches_eq3_and_table2():
    rows = _table("table2_dense_sizes.txt")
    checked = 0
    for row in rows:
        n = int(row[0])
        for q, cell in zip(range(2, 17, 2), row[1:]):
            val, unit = cell.split(":")
            assert f"{eq3(q, n, 3) / UNITS[unit]:.2f}" == val
            if eq3(q, n, 3) <= 8 << 20:
                t = fx.dense(seed=13, q=q, n=n, D=3, packed_last=1)
                c = copy_of(t, align=8)
                assert c.payload_bytes == eq3(q, n, 3)
                assert f"{c.payload_bytes / UNITS[unit]:.2f}" == val
                # nodes at levels 1..3 each hold one pointer to their array; every
                # node holds a payload pointer, non-last nodes a next pointer
                nodes = sum(q ** lv for lv in range(4))
                assert c.nslots == nodes + sum(q ** lv for lv in range(3))
                checked += 1
    assert checked >= 20


# ---------------------------------------------------------------- layouts ----------

def test_plain_layout_worked_example():
    # Root{i64 n; Child* c} 16 B at 0; Child[16] 256 B at 64; leaf i (1024
    # doubles, 8192 B) at 320 + 8192 i; end 320 + 16*8192 = 131392 = 64*2053.
    t = fx.plain()
    c = copy_of(t)
    o = c.objects()
    assert list(o["off"][:2]) == [0, 64]
    assert list(o["bytes"][:2]) == [16, 256]
    assert list(o["off"][2:]) == [320 + 8192 * i for i in range(16)]
    assert c.arena_bytes == 131392
    assert c.payload_bytes == 16 + 256 + 16 * 8192 == 131344
    assert c.nslots == 17
    arena = c.arena()
    # root's pointer -> B + 64; child i's pointer -> B + 320 + 8192 i
    assert int.from_bytes(arena[8:16].tobytes(), "little") == BASE + 64
    for i in range(16):
        s = 64 + 16 * i + 8
        assert int.from_bytes(arena[s:s + 8].tobytes(), "little") == BASE + 320 + 8192 * i


def test_linear_layout_worked_example():
    # L{i32 nA; i32 nLnext; double* A; L* Lnext} is 24 B; only L7 owns A.
    # Pre-order: L0..L7 at 64 i, then L7.A (2^27 B) at 512.
    t = fx.linear()
    c = copy_of(t)
    o = c.objects()
    assert list(o["off"]) == [64 * i for i in range(8)] + [512]
    assert c.arena_bytes == 512 + (1 << 27) == 134218240
    assert c.payload_bytes == eq2(8, 1 << 24) == 134217920
    chain = [(1, 0)] * 7 + [(0, 0)]
    assert c.resolve_chain(0, chain) == (BASE + 512, 1 << 24, "f64")


# ---------------------------------------------------------------- graph pins -------

def _root_offsets(c, t):
    objs = c.objects()
    by_host = {int(h): int(o) for h, o in zip(objs["host"], objs["off"])}
    return [by_host[r] for r in t.roots]


@pytest.mark.parametrize("seed", range(40))
def test_isomorphism_tiny_random_graphs(seed):
    t = fx.random_tree(seed, max_objects=6)
    c = copy_of(t)
    hg, _ = graphs.host_graph(t.types, t.root_type, t.roots)
    ag, _ = graphs.arena_graph(t.types, t.root_type, c.arena().tobytes(), BASE, _root_offsets(c, t))
    assert len(hg) == len(ag) == len(c.objects())
    maps = graphs.preserving_bijections(hg, ag)
    objs = c.objects()
    layout = {int(h): BASE + int(o) for h, o in zip(objs["host"], objs["off"])}
    assert layout in maps
    # every surviving bijection differs from the layout map by an automorphism
    autos = graphs.preserving_bijections(hg, hg)
    assert len(maps) == len(autos)


def _check_invariants(t, c, align):
    arena = c.arena().tobytes()
    objs = c.objects()
    starts = {BASE + int(o) for o in objs["off"]}
    # I4: aligned, non-overlapping, increasing, zero padding
    end = 0
    covered = np.zeros(len(arena), bool)
    for i, o in enumerate(objs):
        off, nb = int(o["off"]), int(o["bytes"])
        assert off % align == 0
        assert off >= end
        assert arena[end:off] == b"\0" * (off - end)
        end = off + max(nb, 1)
        covered[off:off + nb] = True
    # I6
    assert c.arena_bytes == (end + align - 1) // align * align
    assert not arena[end:].strip(b"\0")
    # I1: every non-null pointer is the start of an object inside the buffer
    slots = graphs.pointer_slots(t.types, objs, arena)
    nonnull = [v for _, v in slots if v]
    assert all(BASE <= v < BASE + c.arena_bytes and v in starts for v in nonnull)
    assert len(nonnull) == c.nslots
    # I5: nulls stay null and aliasing is preserved slot by slot
    host_slots = []
    for o in objs:
        if o["kind"] != 0:
            continue
        ty = t.types[int(o["type"])]
        for e in range(int(o["count"])):
            for f in ty.fields:
                a = int(o["host"]) + e * ty.size + f.offset
                host_slots.append(int.from_bytes(ctypes.string_at(a, 8), "little"))
    assert len(host_slots) == len(slots)
    hmap = {int(h): BASE + int(o) for h, o in zip(objs["host"], objs["off"])}
    for hv, (_, av) in zip(host_slots, slots):
        assert (hv == 0) == (av == 0)
        if hv:
            assert hmap[hv] == av
    # I2: leaf bytes conserved per kind and identical before any kernel
    for o in objs:
        if o["kind"] != 0:
            h = ctypes.string_at(int(o["host"]), int(o["bytes"])) if o["bytes"] else b""
            assert arena[int(o["off"]): int(o["off"]) + int(o["bytes"])] == h
    for kind in ("f32", "f64"):
        reach = {int(h) for h, k in zip(objs["host"], objs["kind"]) if k == orc.OR_KIND[kind]}
        host_bytes = sum(a.bytes for a in t.allocs if a.kind == kind and a.base in reach)
        assert host_bytes == sum(int(o["bytes"]) for o in objs if o["kind"] == orc.OR_KIND[kind])
    # I3: hop depth of every object from the roots is preserved
    hg, _ = graphs.host_graph(t.types, t.root_type, t.roots)
    ag, _ = graphs.arena_graph(t.types, t.root_type, arena, BASE, _root_offsets(c, t))
    hd = graphs.depths(hg, t.roots)
    ad = graphs.depths(ag, [BASE + o for o in _root_offsets(c, t)])
    for h, o in hmap.items():
        assert hd[h] == ad[o]


def _check_preorder(t, c):
    """Depth-first pre-order, checked by its characterisation: after the
    first i objects, object i+1 is the first not-yet-emitted target (in
    element, then field-offset order) of the latest emitted object that still
    has one; when none has, it is the next root not yet emitted."""
    objs = c.objects()
    order = [int(h) for h in objs["host"]]
    hg, _ = graphs.host_graph(t.types, t.root_type, t.roots)

    def targets(h):
        node = hg[h]
        flds = t.types[node.type].fields if node.kind == "struct" else []
        return [tgt for e, f, tgt in sorted(node.edges, key=lambda x: (x[0], flds[x[1]].offset))]

    emitted = set()
    for i, h in enumerate(order):
        want = None
        for k in range(i - 1, -1, -1):
            cand = [x for x in targets(order[k]) if x not in emitted]
            if cand:
                want = cand[0]
                break
        if want is None:
            want = next(r for r in t.roots if r not in emitted)
        assert h == want, f"object {i} out of depth-first pre-order"
        emitted.add(h)


@pytest.mark.parametrize("seed", range(25))
def test_invariants_random_graphs(seed):
    t = fx.random_tree(1000 + seed, max_objects=40, nroots=1 + seed % 3)
    align = [8, 16, 64, 256][seed % 4]
    c = copy_of(t, align=align)
    _check_invariants(t, c, align)
    _check_preorder(t, c)


def test_invariants_small_workloads():
    for t in (fx.plain(), fx.wide(f1=4, f2=8, lo=16, hi=300), fx.md(nsims=12, cells_lo=1, cells_hi=6),
              fx.broom(seed=5, bytes_lo=64, bytes_hi=4096)):
        c = copy_of(t)
        _check_invariants(t, c, 64)
        _check_preorder(t, c)


# ---------------------------------------------------------------- errors -----------

def _mem(n):
    b = ctypes.create_string_buffer(n)
    return b, ctypes.addressof(b)


def _put(addr, off, val, nbytes=8, signed=False):
    ctypes.memmove(addr + off, int(val).to_bytes(nbytes, "little", signed=signed), nbytes)


def test_errors_conflict_interior_negative_null():
    types = fx.RANDOM_TYPES
    keep = []
    # two A nodes whose vals pointers reach the same array with different counts
    a1, p1 = _mem(40); a2, p2 = _mem(40); v, pv = _mem(32)
    keep += [a1, a2, v]
    _put(p1, 8, p2)          # a1.next = a2
    _put(p1, 4, 4, 4, True); _put(p1, 24, pv)  # a1.vals = v, nb = 4
    _put(p2, 4, 3, 4, True); _put(p2, 24, pv)  # a2.vals = v, nb = 3
    with pytest.raises(orc.OracleError) as e:
        orc.OracleCopy(types, 0, [p1])
    assert e.value.name == "CONFLICT"
    # interior pointer: a2.vals points into the middle of a1.vals
    _put(p2, 4, 1, 4, True); _put(p2, 24, pv + 8)
    with pytest.raises(orc.OracleError) as e:
        orc.OracleCopy(types, 0, [p1])
    assert e.value.name == "RANGE"
    # negative count
    _put(p2, 24, 0); _put(p1, 4, -1, 4, True)
    with pytest.raises(orc.OracleError) as e:
        orc.OracleCopy(types, 0, [p1])
    assert e.value.name == "INVAL"
    # null root
    with pytest.raises(orc.OracleError) as e:
        orc.OracleCopy(types, 0, [0])
    assert e.value.name == "INVAL"
    # a null pointer with a non-zero count is no object
    _put(p1, 4, 5, 4, True); _put(p1, 24, 0)
    c = orc.OracleCopy(types, 0, [p1])
    assert len(c.objects()) == 2


def test_cycle_and_alias_copied_once():
    types = fx.RANDOM_TYPES
    a1, p1 = _mem(40); a2, p2 = _mem(40)
    _put(p1, 8, p2); _put(p2, 8, p1)  # a1 <-> a2
    c = orc.OracleCopy(types, 0, [p1, p2, p1], 64, BASE)
    assert len(c.objects()) == 2 and c.nslots == 2
    ar = c.arena().tobytes()
    assert int.from_bytes(ar[8:16], "little") == BASE + 64
    assert int.from_bytes(ar[64 + 8:64 + 16], "little") == BASE + 0


# ---------------------------------------------------------------- rounding ---------

def _samples(n, seed):
    rng = random.Random(seed)
    out = []
    for i in range(n):
        x = rng.uniform(-1, 1)
        if i % 3 == 0:
            a, b = rng.choice([1.0001, 0.9999]), rng.choice([0.5, -0.25])
        else:
            a, b = rng.uniform(-2, 2), rng.uniform(-2, 2) * 2.0 ** rng.randint(-60, 2)
        out.append((x, a, b))
    return out


def test_fma64_correctly_rounded():
    s = _samples(100000, 1)
    xs, as_, bs = (np.array(v) for v in zip(*s))
    # through the kernel itself: one pass over an FP64 leaf per (a, b) pair is
    # too many leaves, so check the scalar entry on all samples ...
    got = np.array([orc.fma64(x, a, b) for x, a, b in s])
    want = np.array([exact.fma64(x, a, b) for x, a, b in s])
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    # ... and make sure the sample would catch a separately rounded x*a + b
    assert np.count_nonzero((xs * as_ + bs) != want) > 1000


def test_fma32_correctly_rounded():
    s = [(exact.f32(x), exact.f32(a), exact.f32(b)) for x, a, b in _samples(100000, 2)]
    got = np.array([orc.fma32(x, a, b) for x, a, b in s], np.float32)
    want = np.array([exact.fma32(x, a, b) for x, a, b in s], np.float32)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    f = np.float32
    sep = np.array([f(f(x) * f(a)) + f(b) for x, a, b in s], np.float32)
    assert np.count_nonzero(sep != want) > 1000
    # a case where rounding through binary64 first gives a different answer:
    # x = a = 1 + 2^-12, b = 2^-80: x*a + b sits just above a binary32 midpoint
    x = 1 + 2.0 ** -12
    want1 = exact.fma32(x, x, 2.0 ** -80)
    assert want1 == 1 + 2.0 ** -11 + 2.0 ** -23
    assert orc.fma32(x, x, 2.0 ** -80) == want1
    assert exact.f32(x * x + 2.0 ** -80) != want1


def test_fma_special_cases():
    rng = random.Random(3)
    for _ in range(1000):
        x = rng.uniform(-1, 1)
        assert orc.fma64(x, 1.0, 0.0) == x
        assert orc.fma32(exact.f32(x), 1.0, 0.0) == exact.f32(x)
    for z in (0.0, -0.0):
        for a, b in ((1.0001, 0.5), (0.9999, -0.25)):
            assert orc.fma64(z, a, b) == b
            assert orc.fma32(z, a, b) == exact.f32(b)
    assert math.copysign(1, orc.fma64(-0.0, 1.0, 0.0)) == 1.0  # -0 + +0 = +0


def test_kernel_passes_match_exact_steps():
    t = fx.plain(seed=21, nchild=3, leaf_len=40)
    c = copy_of(t)
    objs = c.objects()
    ar = c.arena()
    leaves = [o for o in objs if o["kind"] == 2]
    before = [np.frombuffer(ar[int(o["off"]):int(o["off"]) + int(o["bytes"])].tobytes(), np.float64).copy()
              for o in leaves]
    c.run_kernel(1.0001, 0.5, iters=100, select="all")
    ar = c.arena()
    for o, x0 in zip(leaves, before):
        got = np.frombuffer(ar[int(o["off"]):int(o["off"]) + int(o["bytes"])].tobytes(), np.float64)
        want = []
        for x in x0:
            for _ in range(100):
                x = exact.fma64(float(x), 1.0001, 0.5)
            want.append(x)
        assert np.array_equal(got.view(np.uint64), np.array(want).view(np.uint64))
    # struct bytes untouched by the kernel
    assert int.from_bytes(ar[8:16].tobytes(), "little") == BASE + 64


def test_kernel_fp32_leaves_exact():
    t = fx.wide(seed=22, f1=1, f2=4, lo=50, hi=60)
    c = copy_of(t)
    objs = c.objects()
    ar0 = c.arena().copy()
    c.run_kernel(0.9999, -0.25, iters=3, select="all")
    ar = c.arena()
    a32, b32 = exact.f32(0.9999), exact.f32(-0.25)
    n = 0
    for o in objs:
        lo, hi = int(o["off"]), int(o["off"]) + int(o["bytes"])
        if o["kind"] == 1:
            x0 = np.frombuffer(ar0[lo:hi].tobytes(), np.float32)
            got = np.frombuffer(ar[lo:hi].tobytes(), np.float32)
            for xa, g in zip(x0, got):
                x = float(xa)
                for _ in range(3):
                    x = exact.fma32(x, a32, b32)
                assert np.float32(x) == g
                n += 1
    assert n > 50


def test_out_of_place_image():
    t = fx.wide(seed=23, f1=2, f2=3, lo=5, hi=40)
    c = copy_of(t)
    objs = c.objects()
    before = c.arena().copy()
    nb = c.out_bytes("all")
    out = np.zeros(nb, np.uint8)
    c.run_kernel(1.0001, 0.5, iters=2, select="all", out=out)
    assert np.array_equal(c.arena(), before)  # buffer untouched
    off = None
    for o in objs:
        if o["kind"] not in (1, 2):
            continue
        off = 0 if off is None else (off + 63) // 64 * 64
        lo, n = int(o["off"]), int(o["bytes"])
        if o["kind"] == 2:
            x0 = np.frombuffer(before[lo:lo + n].tobytes(), np.float64)
            want = [exact.fma64(exact.fma64(float(x), 1.0001, 0.5), 1.0001, 0.5) for x in x0]
            got = np.frombuffer(out[off:off + n].tobytes(), np.float64)
            assert np.array_equal(got.view(np.uint64), np.array(want).view(np.uint64))
        off += max(n, 1)
    assert nb == (off + 63) // 64 * 64


# ---------------------------------------------------------------- chains -----------

def test_resolve_chain_plain_and_errors():
    t = fx.plain()
    c = copy_of(t)
    for i in range(16):
        assert c.resolve_chain(0, [(0, i), (0, 0)]) == (BASE + 320 + 8192 * i, 1024, "f64")
    with pytest.raises(orc.OracleError) as e:
        c.resolve_chain(0, [(0, 16), (0, 0)])
    assert e.value.name == "RANGE"
    tl = fx.linear(k=4, n=10)
    cl = copy_of(tl)
    with pytest.raises(orc.OracleError) as e:  # L0.A is null under LLinit
        cl.resolve_chain(0, [(0, 0)])
    assert e.value.name == "RANGE"
    # the chain kernel touches only the chain's leaf
    t2 = fx.plain(seed=9, nchild=4, leaf_len=8)
    c2 = copy_of(t2)
    ar0 = c2.arena().copy()
    c2.run_kernel(1.0001, 0.5, select="chain", chain=[(0, 2), (0, 0)])
    ar = c2.arena()
    o = c2.objects()
    changed = np.nonzero(ar != ar0)[0]
    lo = int(o["off"][2 + 2])
    assert changed.min() >= lo and changed.max() < lo + 64


def test_dense_chain_last_element():
    # the Dense kernel reaches a0->Lnext[q-1].Lnext[q-1].Lnext[q-1].A
    q = 3
    t = fx.dense(seed=31, q=q, n=5, D=3, packed_last=0)
    c = copy_of(t)
    addr, n, kind = c.resolve_chain(0, [(1, q - 1)] * 3 + [(0, 0)])
    assert (n, kind) == (5, "f64")
    # walk the host tree by hand to the same array and compare contents
    p = t.roots[0]
    for _ in range(3):
        arr = int.from_bytes(ctypes.string_at(p + 16, 8), "little")
        p = arr + (q - 1) * 24 if _ < 2 else arr + (q - 1) * 16
    host_a = int.from_bytes(ctypes.string_at(p + 8, 8), "little")
    ar = c.arena().tobytes()
    assert ar[addr - BASE: addr - BASE + 40] == ctypes.string_at(host_a, 40)


# ---------------------------------------------------------------- copy back --------

def test_copy_back_leaves_and_scalars():
    t = fx.plain(seed=41, nchild=5, leaf_len=33)
    roots_ptr = [int.from_bytes(ctypes.string_at(t.roots[0] + 8, 8), "little")]
    c = copy_of(t)
    c.run_kernel(1.0001, 0.5, iters=2, select="all")
    # change a count in the buffer to see the scalar path
    ar = c.arena()
    ar[64:72] = np.frombuffer((7).to_bytes(8, "little"), np.uint8)
    c.copy_back(scalars=False)
    objs = c.objects()
    for o in objs:
        if o["kind"] == 2:
            assert ctypes.string_at(int(o["host"]), int(o["bytes"])) == \
                ar[int(o["off"]):int(o["off"]) + int(o["bytes"])].tobytes()
    host_child0 = int(objs["host"][1])
    assert int.from_bytes(ctypes.string_at(host_child0, 8), "little") == 33  # scalars untouched
    c.copy_back(scalars=True)
    assert int.from_bytes(ctypes.string_at(host_child0, 8), "little") == 7
    # host pointers never overwritten
    assert int.from_bytes(ctypes.string_at(t.roots[0] + 8, 8), "little") == roots_ptr[0]
    assert int.from_bytes(ctypes.string_at(host_child0 + 8, 8), "little") == int(objs["host"][2])
