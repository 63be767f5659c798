"""Host logic of libdc that needs no GPU: the library loads and exports every
call include/dc.h declares, schemas are validated, and the planner's walk and
layout agree with the CPU oracle object by object (same order, offsets, sizes)
and report the same errors."""
import ctypes
import os
import re

import numpy as np
import pytest

import fixtures as fx
import oracle as orc
from tests.helpers import plan_of, same_objects

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_call():
    from paper_1906_01128_amd import dc
    header = open(os.path.join(ROOT, "include", "dc.h")).read()
    names = set(re.findall(r"^(?:dc_status|const char\*)\s+(dc_\w+)\s*\(", header, re.M))
    assert len(names) >= 30
    lib = ctypes.CDLL(dc.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    # and the binding declares a signature for each
    bound = set(dc._SIGS) | {"dc_last_error", "dc_version"}
    assert names <= bound, f"no binding for {sorted(names - bound)}"


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1906_01128_amd import dc
    monkeypatch.setattr(dc, "_lib", None)
    monkeypatch.setattr(dc, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        dc.load()


def test_schema_validation():
    from paper_1906_01128_amd import dc
    s = dc.Schema()
    ok = s.describe("T", 24, 8, [dict(offset=8, kind="f64", type=0, count_offset=0, count_bytes=8, count_mult=1,
                                      fixed_count=0)])
    assert ok == 0
    bad = [
        dict(offset=4, kind="f64", type=0, count_offset=0, count_bytes=4, count_mult=1, fixed_count=0),  # misaligned
        dict(offset=24, kind="f64", type=0, count_offset=0, count_bytes=8, count_mult=1, fixed_count=0),  # outside
        dict(offset=8, kind="f64", type=0, count_offset=8, count_bytes=8, count_mult=1, fixed_count=0),  # overlaps
        dict(offset=8, kind="f64", type=0, count_offset=0, count_bytes=2, count_mult=1, fixed_count=0),  # width
        dict(offset=8, kind=9, type=0, count_offset=0, count_bytes=8, count_mult=1, fixed_count=0),  # kind
        dict(offset=8, kind="f64", type=0, count_offset=0, count_bytes=8, count_mult=0, fixed_count=0),  # mult
    ]
    for f in bad:
        with pytest.raises(dc.DcError) as e:
            s.describe("Bad", 24, 8, [f])
        assert e.value.name == "INVAL"


def _compare(t, align=64):
    p = plan_of(t, align)
    c = orc.OracleCopy(t.types, t.root_type, t.roots, align, 0)
    same_objects(p.objects(), c.objects())
    info = p.info()
    assert info.arena_bytes == c.arena_bytes == p.arena_bytes
    assert info.nslots_nonnull == c.nslots
    assert info.payload_bytes == c.payload_bytes
    objs = c.objects()
    leaves = objs[np.isin(objs["kind"], (1, 2))]
    assert info.leaf_bytes == int(leaves["bytes"].sum())
    assert info.nleaves == int((leaves["count"] > 0).sum())
    assert info.out_bytes == c.out_bytes("all")
    return p, c


@pytest.mark.parametrize("seed", range(30))
def test_plan_matches_oracle_random(seed):
    t = fx.random_tree(500 + seed, max_objects=60, nroots=1 + seed % 4)
    _compare(t, align=[16, 64, 256, 4096][seed % 4])


def test_plan_matches_oracle_workloads():
    _compare(fx.plain())
    _compare(fx.linear(n=1000))
    _compare(fx.linear(k=10, n=100, scheme=0))
    _compare(fx.dense(q=4, n=50, D=3))
    _compare(fx.wide(f1=8, f2=16))
    _compare(fx.md(nsims=50))
    _compare(fx.broom(seed=3, bytes_hi=1 << 16))


def test_leaf_prefix_table_lies_in_scratch():
    """The table the deep copy fills on the device (one word per leaf and a
    total) sits 8-byte aligned inside the scratch buffer the plan asks for,
    and the leaf count is that of the oracle's layout (FP32/FP64 arrays with
    at least one element)."""
    for t in (fx.linear(k=3, n=0), fx.plain(), fx.wide(f1=8, f2=300, lo=1, hi=300), fx.md(nsims=40),
              fx.random_tree(11, max_objects=4000, nroots=300)):
        p = plan_of(t)
        info = p.info()
        ref = orc.OracleCopy(t.types, t.root_type, t.roots, 64, 1 << 40)
        objs = ref.objects()
        leaves = int((((objs["kind"] == 1) | (objs["kind"] == 2)) & (objs["count"] > 0)).sum())
        assert info.nleaves == leaves
        assert info.leaf_prefix_offset % 8 == 0
        assert info.leaf_prefix_offset + 8 * (info.nleaves + 1) <= info.scratch_bytes
        ref.free()


def test_plan_segments_cover_many_targets():
    # more targets than one relocation unit holds, and a struct array with
    # more slots than a unit takes
    p, _ = _compare(fx.wide(f1=40, f2=64, lo=1, hi=4))
    assert p.info().nsegments >= 3
    p, _ = _compare(fx.plain(nchild=20000, leaf_len=1))
    assert p.info().nsegments >= 2


def test_unit_leaf_runs():
    """The per-unit persistent batched form needs every relocation unit's
    slots to be the first to reach one contiguous run of leaves. The MD,
    wide, plain, broom and Linear shapes have it (their structs list leaf
    members before deeper struct members, so a depth-first layout places a
    unit's leaves together); the 16-way Dense tree, whose nodes reach their
    own array and then their children's subtrees, spreads over several
    units that do not."""
    for t in (fx.md(nsims=50), fx.wide(f1=8, f2=16), fx.plain(nchild=20000, leaf_len=1),
              fx.broom(seed=3, bytes_hi=1 << 16), fx.linear(k=10, n=100, scheme=0)):
        i = plan_of(t).info()
        assert i.unit_leaves == 1
        assert 0 < i.max_unit_leaf_bytes <= i.leaf_bytes + 16 * i.nleaves
    i = plan_of(fx.md(nsims=50)).info()
    assert i.nsegments > 100 and i.max_unit_leaf_bytes < i.leaf_bytes // 50
    i = plan_of(fx.dense(q=16, n=10, D=3)).info()
    assert i.nsegments > 1 and i.unit_leaves == 0


def test_plan_errors_match_oracle():
    from paper_1906_01128_amd import dc
    types = fx.RANDOM_TYPES
    keep = []

    def mem(n):
        b = ctypes.create_string_buffer(n)
        keep.append(b)
        return ctypes.addressof(b)

    def put(a, off, v, n=8, signed=False):
        ctypes.memmove(a + off, int(v).to_bytes(n, "little", signed=signed), n)

    p1, p2, v = mem(40), mem(40), mem(32)
    put(p1, 8, p2)
    put(p1, 4, 4, 4, True); put(p1, 24, v)
    put(p2, 4, 3, 4, True); put(p2, 24, v)
    cases = []
    cases.append("CONFLICT")
    for want in ("CONFLICT", "RANGE", "INVAL"):
        if want == "RANGE":
            put(p2, 4, 1, 4, True); put(p2, 24, v + 8)
        if want == "INVAL":
            put(p2, 24, 0); put(p1, 4, -1, 4, True)
        with pytest.raises(orc.OracleError) as eo:
            orc.OracleCopy(types, 0, [p1])
        with pytest.raises(dc.DcError) as ed:
            dc.Plan(dc.Schema(types), 0, [p1])
        assert eo.value.name == ed.value.name == want
    with pytest.raises(dc.DcError) as ed:
        dc.Plan(dc.Schema(types), 0, [0])
    assert ed.value.name == "INVAL"
    with pytest.raises(dc.DcError) as ed:
        dc.Plan(dc.Schema(types), 0, [p1], align=8)
    assert ed.value.name == "INVAL"


# ---- plans over many roots: walked in chunks of consecutive roots on host threads ----------


def test_plan_many_independent_roots_matches_oracle():
    """300 MD simulations: the chunked walk is kept (no array is reached from
    two chunks) and must equal the walk in root order object by object."""
    p, _ = _compare(fx.md(seed=77, nsims=300))
    assert p.info().nroots == 300 and p.info().unit_leaves == 1


@pytest.mark.slow
def test_plan_full_md_matches_oracle():
    """The full batched MD workload (10,000 simulations, ~7.75 M arrays):
    the chunked plan equals the oracle's walk object by object."""
    fx.set_threads(0)
    t = fx.md()
    p = plan_of(t)
    c = orc.OracleCopy(t.types, t.root_type, t.roots, 64, 0)
    same_objects(p.objects(), c.objects())
    assert p.info().arena_bytes == c.arena_bytes and p.info().nslots_nonnull == c.nslots
    assert p.info().unit_leaves == 1


@pytest.mark.parametrize("seed", range(4))
def test_plan_many_roots_with_shared_arrays_matches_oracle(seed):
    """Random graphs over 200 roots whose structs point into other roots'
    arrays (aliases, cycles, zero-length arrays): the chunked walk sees an
    array reached from two chunks and the walk in root order decides."""
    _compare(fx.random_tree(900 + seed, max_objects=3000, nroots=200), align=[16, 64, 256, 4096][seed])


def _md_roots(n):
    t = fx.md(seed=78, nsims=n, cells_lo=2, cells_hi=6, mean_atoms=3)
    cells = [int.from_bytes(ctypes.string_at(r + 8, 8), "little") for r in t.roots]
    return t, cells


def test_plan_many_roots_aliases_and_errors_match_oracle():
    """Across chunks: an array shared by two roots is copied once (as the walk
    in root order does), a pointer into the middle of another root's array
    is DC_E_RANGE, the same array reached with another length is
    DC_E_CONFLICT, and a negative count in a late root is DC_E_INVAL."""
    from paper_1906_01128_amd import dc

    def put(a, off, v, signed=False):
        ctypes.memmove(a + off, int(v).to_bytes(8, "little", signed=signed), 8)

    def both(t):
        try:
            c = orc.OracleCopy(t.types, t.root_type, t.roots, 64, 0)
        except orc.OracleError as e:
            with pytest.raises(dc.DcError) as ed:
                plan_of(t)
            assert ed.value.name == e.name
            return e.name
        p = plan_of(t)
        same_objects(p.objects(), c.objects())
        assert p.info().arena_bytes == c.arena_bytes
        return "OK"

    t, cells = _md_roots(200)
    put(t.roots[180], 8, cells[20])             # root 180 shares root 20's cells (same count?)
    put(t.roots[180], 0, int.from_bytes(ctypes.string_at(t.roots[20], 8), "little"), True)
    assert both(t) == "OK"
    t, cells = _md_roots(200)
    put(t.roots[190], 8, cells[10] + 32)        # one cell into root 10's array
    put(t.roots[190], 0, 1, True)
    assert both(t) == "RANGE"
    t, cells = _md_roots(200)
    n10 = int.from_bytes(ctypes.string_at(t.roots[10], 8), "little")
    put(t.roots[170], 8, cells[10])             # root 10's cells with one cell more
    put(t.roots[170], 0, n10 + 1, True)
    assert both(t) == "CONFLICT"
    t, cells = _md_roots(200)
    put(t.roots[150], 0, -1, True)
    assert both(t) == "INVAL"


# ---- dc_chain_query: the host walk of the pointerchain transfer (no device) ----------------


def test_chain_query_matches_oracle_chains():
    from paper_1906_01128_amd import dc
    import oracle as orc
    t = fx.dense(seed=fx.SEED_BASE + 5, q=3, n=17, D=3, packed_last=0)
    schema = dc.Schema(t.types)
    ref = orc.OracleCopy(t.types, t.root_type, t.roots, 64, 0)
    for lv in range(4):
        for idx in range(3):
            chain = [(1, idx)] * lv + [(0, 0)]
            q = dc.chain_query(schema, t.root_type, t.roots[0], chain)
            _, count, kind = ref.resolve_chain(0, chain)
            assert (q.count, dc.KIND_NAME[q.kind], q.dev_addr) == (count, kind, 0)


def test_chain_query_errors():
    from paper_1906_01128_amd import dc
    t = fx.linear(seed=fx.SEED_BASE + 6, k=3, n=10, scheme=1)
    schema = dc.Schema(t.types)
    for bad in ([(0, 0)],                      # level 0 has no data array
                [(1, 1), (1, 0), (0, 0)],      # index past the one-element next array
                [(1, 0), (0, 0), (0, 0)],      # a step through a primitive array
                [(2, 0)],                      # no such field
                []):                           # empty chain
        with pytest.raises(dc.DcError):
            dc.chain_query(schema, 0, t.roots[0], bad)
    q = dc.chain_query(schema, 0, t.roots[0], [(1, 0), (1, 0), (0, 0)])
    assert q.count == 10 and dc.KIND_NAME[q.kind] == "f64"
    # a chain that ends in a struct array is described (the transfer itself refuses it)
    q = dc.chain_query(schema, 0, t.roots[0], [(1, 0)])
    assert dc.KIND_NAME[q.kind] == "struct" and q.count == 1
