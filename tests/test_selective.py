"""Selective deep copy (Section 2: only the members a kernel needs are
followed). Pins for the oracle's selective walk, then the planner against it.

Pins, independent of the oracle's own code:
  * pruned-graph equivalence: a selective copy equals the full deep copy of the
    same graph with the unfollowed pointer members set to null on the host
    (a different route through the walk: nulls instead of masks);
  * the Linear tree with every level allocated (Section 4.2) and only the
    next-level member followed has k struct objects, k*24 payload bytes, no
    primitive array, and a buffer whose data-array members read null while
    the counts keep their host values;
  * a mask with every bit set is the full deep copy.
"""
import ctypes
import random

import numpy as np
import pytest

import fixtures as fx
import oracle as orc
from tests.helpers import plan_of, same_objects

BASE = 0x7F0000000000


def _mask_all(types):
    return [(1 << len(t.fields)) - 1 for t in types]


def _prune(t, follow):
    """Sets every unfollowed pointer member of every struct reachable in the
    full copy to null, in host memory."""
    full = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE)
    for o in full.objects():
        if o["kind"] != 0:
            continue
        ty = t.types[int(o["type"])]
        for e in range(int(o["count"])):
            elem = int(o["host"]) + e * ty.size
            for fi, f in enumerate(ty.fields):
                if not (follow[int(o["type"])] >> fi) & 1:
                    ctypes.memmove(elem + f.offset, b"\0" * 8, 8)
    full.free()


@pytest.mark.parametrize("seed", range(40))
def test_pruned_graph_equivalence(seed):
    rng = random.Random(1000 + seed)
    follow = [rng.getrandbits(3), rng.getrandbits(2)]
    t1 = fx.random_tree(seed, max_objects=12, nroots=1 + seed % 3)
    t2 = fx.random_tree(seed, max_objects=12, nroots=1 + seed % 3)
    sel = orc.OracleCopy(t1.types, t1.root_type, t1.roots, 64, BASE, follow=follow)
    _prune(t2, follow)
    ref = orc.OracleCopy(t2.types, t2.root_type, t2.roots, 64, BASE)
    assert sel.arena_bytes == ref.arena_bytes
    assert np.array_equal(sel.arena(), ref.arena())
    a, b = sel.objects(), ref.objects()
    for name in ("off", "bytes", "count", "kind"):
        assert np.array_equal(a[name], b[name]), name
    assert sel.nslots == ref.nslots
    assert sel.payload_bytes == ref.payload_bytes


def test_linear_allinit_next_only():
    k, n = 8, 1000
    t = fx.linear(k=k, n=n, scheme=0)
    # field 0 of type L is the data array A (offset 8), field 1 the next level (offset 16)
    c = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE, follow=[0b10])
    objs = c.objects()
    assert len(objs) == k
    assert np.all(objs["kind"] == 0)
    assert c.payload_bytes == k * 24
    assert c.nslots == k - 1
    ar = c.arena()
    for i, o in enumerate(objs):
        off = int(o["off"])
        assert off == 64 * i
        node = ar[off:off + 24]
        assert int(node[0:4].view(np.int32)[0]) == n          # nA kept
        assert int(node[8:16].view(np.uint64)[0]) == 0        # A not followed: null
        nxt = int(node[16:24].view(np.uint64)[0])
        assert nxt == (BASE + 64 * (i + 1) if i < k - 1 else 0)


def test_linear_allinit_data_only():
    k, n = 8, 1000
    t = fx.linear(k=k, n=n, scheme=0)
    c = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE, follow=[0b01])
    objs = c.objects()
    # the root struct and its own data array; nothing below the root
    assert len(objs) == 2
    assert list(objs["kind"]) == [0, 2]
    assert c.payload_bytes == 24 + 8 * n
    root = c.arena()[0:24]
    assert int(root[16:24].view(np.uint64)[0]) == 0
    assert int(root[8:16].view(np.uint64)[0]) == BASE + 64


@pytest.mark.parametrize("seed", range(10))
def test_full_mask_is_full_copy(seed):
    t = fx.random_tree(seed, max_objects=10)
    a = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE, follow=_mask_all(t.types))
    b = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE)
    assert np.array_equal(a.arena(), b.arena())


# ---- the planner (host logic of the library) against the oracle --------------------------


@pytest.mark.parametrize("seed", range(30))
def test_planner_selective_matches_oracle(seed):
    rng = random.Random(2000 + seed)
    follow = [rng.getrandbits(3), rng.getrandbits(2)]
    t = fx.random_tree(seed, max_objects=12, nroots=1 + seed % 2)
    p = plan_of(t, follow=follow)
    o = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE, follow=follow)
    same_objects(p.objects(), o.objects())
    assert p.info().nslots_nonnull == o.nslots
    assert p.info().payload_bytes == o.payload_bytes


@pytest.mark.parametrize("follow", [[0b10], [0b01], [0b00], [0b11]])
def test_planner_selective_linear(follow):
    t = fx.linear(k=6, n=300, scheme=0)
    p = plan_of(t, follow=follow)
    o = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE, follow=follow)
    same_objects(p.objects(), o.objects())


def test_planner_selective_wide():
    t = fx.wide(seed=5, f1=8, f2=8, lo=1, hi=100)
    follow = [(1 << len(ty.fields)) - 1 for ty in t.types]
    follow[2] &= ~1  # leaves drop their FP32 array
    p = plan_of(t, follow=follow)
    o = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE, follow=follow)
    same_objects(p.objects(), o.objects())


def test_planner_selective_rejects_bad_masks():
    from paper_1906_01128_amd import dc
    t = fx.random_tree(3)
    with pytest.raises(dc.DcError):
        plan_of(t, follow=[0b1000, 0])   # a bit past type A's three members
    with pytest.raises(dc.DcError):
        plan_of(t, follow=[0b111, 0b11, 0])  # a mask for a type that does not exist
    # a short list leaves the remaining types fully followed
    p = plan_of(t, follow=[0b111])
    o = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE)
    same_objects(p.objects(), o.objects())
