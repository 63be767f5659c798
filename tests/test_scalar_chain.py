"""Scalar chains (Section 3, scalar variables): a scalar member reached by a
chain is read into a temporary and written back through the chain.

Oracle pins (CPU): the value at the oracle's address equals what plain
pointer chasing through the host structure reads (Python, one load at a
time); two chains reaching one element by different paths give one
address; the Linear tree's counts follow from its construction (Section
4.2). GPU: declare/update through the C ABI against the oracle's buffer,
bit for bit, then the update reaches the host through the scalar copy back.
"""
import ctypes
import random

import numpy as np
import pytest

import fixtures as fx
import oracle as orc

BASE = 0x7F0000000000


def _u64(addr):
    return ctypes.c_uint64.from_address(addr).value


def _host_scalar(t, root_index, chain, offset, nbytes):
    """Pointer chasing through host memory, one member at a time."""
    ty = t.types[t.root_type]
    elem = t.roots[root_index]
    for field, index in chain:
        f = ty.fields[field]
        p = _u64(elem + f.offset)
        ty = t.types[f.type]
        elem = p + index * ty.size
    return ctypes.string_at(elem + offset, nbytes)


def _oracle_scalar(c, root_index, chain, offset, nbytes):
    a = c.scalar_chain(root_index, chain, offset, nbytes) - c.base
    return c.arena()[a:a + nbytes].tobytes()


def test_md_natoms_match_host_chasing():
    t = fx.md(seed=21, nsims=20, cells_lo=1, cells_hi=30, mean_atoms=7)
    c = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE)
    rng = random.Random(5)
    for _ in range(200):
        i = rng.randrange(20)
        ncells = int.from_bytes(_host_scalar(t, i, [], 0, 8), "little")
        j = rng.randrange(ncells)
        assert _oracle_scalar(c, i, [(0, j)], 0, 8) == _host_scalar(t, i, [(0, j)], 0, 8)
        # and the count agrees with the size of the position array the walk copied
        natoms = int.from_bytes(_host_scalar(t, i, [(0, j)], 0, 8), "little")
        _, count, _ = c.resolve_chain(i, [(0, j), (0, 0)])
        assert count == 3 * natoms


@pytest.mark.parametrize("k", [1, 2, 5])
def test_linear_counts(k):
    t = fx.linear(k=k, n=777, scheme=1)
    c = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE)
    for level in range(k):
        chain = [(1, 0)] * level
        nA = int.from_bytes(_oracle_scalar(c, 0, chain, 0, 4), "little")
        nnext = int.from_bytes(_oracle_scalar(c, 0, chain, 4, 4), "little")
        assert nA == (777 if level == k - 1 else 0)
        assert nnext == (0 if level == k - 1 else 1)
        # the scalar's address is the level's struct offset: 64 * level
        assert c.scalar_chain(0, chain, 0, 4) == BASE + 64 * level


@pytest.mark.parametrize("seed", range(20))
def test_random_tags_match_host(seed):
    t = fx.random_tree(seed, max_objects=12)
    c = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE)
    assert _oracle_scalar(c, 0, [], 32, 8) == _host_scalar(t, 0, [], 32, 8)
    # every A reached by next-hops: its tag
    chain = []
    while True:
        try:
            got = _oracle_scalar(c, 0, chain + [(1, 0)], 32, 8)
        except orc.OracleError:
            break
        assert got == _host_scalar(t, 0, chain + [(1, 0)], 32, 8)
        chain.append((1, 0))
        if len(chain) > 12:   # a cycle of next pointers
            break


def test_alias_paths_share_one_address():
    # a two-node cycle: following next twice returns to the root
    found = 0
    for seed in range(200):
        t = fx.random_tree(seed, max_objects=8)
        c = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE)
        try:
            a2 = c.scalar_chain(0, [(1, 0), (1, 0)], 32, 8)
        except orc.OracleError:
            continue
        host_root = t.roots[0]
        p1 = _u64(host_root + 8)
        p2 = _u64(p1 + 8)
        if p2 == host_root:
            assert a2 == c.scalar_chain(0, [], 32, 8)
            found += 1
        elif p2 == p1:
            assert a2 == c.scalar_chain(0, [(1, 0)], 32, 8)
            found += 1
    assert found > 0


def test_oracle_scalar_errors():
    t = fx.linear(k=3, n=10, scheme=1)
    c = orc.OracleCopy(t.types, t.root_type, t.roots, 64, BASE)
    with pytest.raises(orc.OracleError):
        c.scalar_chain(0, [(1, 1)], 0, 4)          # index past the one-element next array
    with pytest.raises(orc.OracleError):
        c.scalar_chain(0, [(0, 0)], 0, 4)          # a step into a primitive array
    with pytest.raises(orc.OracleError):
        c.scalar_chain(0, [], 20, 8)               # past the 24-byte struct
    with pytest.raises(orc.OracleError):
        c.scalar_chain(0, [(1, 0), (1, 0), (1, 0)], 0, 4)  # null at the last level


# ---- GPU -----------------------------------------------------------------------------


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.gpu
def test_gpu_declare_md_counts():
    torch = _gpu()
    from tests.test_gpu_parity import Copy
    from paper_1906_01128_amd import dc
    ctx = dc.Context(0)
    t = fx.md(seed=22, nsims=50, cells_lo=1, cells_hi=40, mean_atoms=9)
    c = Copy(ctx, t)
    rng = random.Random(9)
    refs = []
    for _ in range(3000):
        i = rng.randrange(50)
        ncells = int.from_bytes(_host_scalar(t, i, [], 0, 8), "little")
        refs.append((i, [(0, rng.randrange(ncells))], 0, 8))
    refs.append((3, [], 0, 8))   # a member of the root itself
    temps = torch.full((len(refs),), -1, dtype=torch.int64, device="cuda")
    c.tree.scalar_declare(refs, temps)
    got = temps.cpu().numpy().view(np.uint64)
    want = [int.from_bytes(_oracle_scalar(c.oracle, *r), "little") for r in refs]
    assert list(got) == want


@pytest.mark.gpu
@pytest.mark.parametrize("seed", range(6))
def test_gpu_update_random_tags(seed):
    torch = _gpu()
    from tests.test_gpu_parity import Copy, assert_same_bytes
    from paper_1906_01128_amd import dc
    ctx = dc.Context(0)
    t = fx.random_tree(seed, max_objects=14, nroots=3)
    c = Copy(ctx, t)
    refs, seen = [], set()
    for root in range(3):
        chain = []
        for _ in range(6):
            try:
                a = c.oracle.scalar_chain(root, chain, 32, 8)
            except orc.OracleError:
                break
            if a not in seen:
                seen.add(a)
                refs.append((root, list(chain), 32, 8))
            chain.append((1, 0))
    # a 4-byte scalar too: the count na of each root
    for root in range(3):
        refs.append((root, [], 0, 4))
    temps = torch.zeros(len(refs), dtype=torch.int64, device="cuda")
    c.tree.scalar_declare(refs, temps)
    vals = temps.cpu().numpy().copy()
    # the "region": new values for every temporary
    new = np.array([0x1111111100000000 + 7 * i for i in range(len(refs))], dtype=np.int64)
    for i, r in enumerate(refs):
        if r[3] == 4:
            new[i] = (int(vals[i]) + 5) & 0x7FFFFFFF     # keep the count sane on the host side
    temps.copy_(torch.from_numpy(new))
    c.tree.scalar_update(refs, temps)
    ar = c.oracle.arena()
    for i, (root, chain, off, nb) in enumerate(refs):
        a = c.oracle.scalar_chain(root, chain, off, nb) - c.base
        ar[a:a + nb] = np.frombuffer(int(new[i]).to_bytes(8, "little", signed=True)[:nb], np.uint8)
    assert_same_bytes(c.device_arena(), ar, "arena after scalar update")
    # the scalar copy back takes the new values to the host structure
    tags_host_before = [_host_scalar(t, r[0], r[1], r[2], r[3]) for r in refs]
    assert any(tags_host_before[i] != int(new[i]).to_bytes(8, "little", signed=True)[:refs[i][3]]
               for i in range(len(refs)))
    c.tree.copy_back(scalars=True)
    for i, r in enumerate(refs):
        assert _host_scalar(t, *r) == int(new[i]).to_bytes(8, "little", signed=True)[:r[3]]


@pytest.mark.gpu
def test_gpu_scalar_errors():
    _gpu()
    import torch
    from tests.test_gpu_parity import Copy
    from paper_1906_01128_amd import dc
    ctx = dc.Context(0)
    t = fx.linear(k=3, n=10, scheme=1)
    c = Copy(ctx, t)
    temps = torch.zeros(4, dtype=torch.int64, device="cuda")
    for bad in [(0, [(1, 1)], 0, 4), (0, [(0, 0)], 0, 4), (0, [], 20, 8), (0, [], 8, 8), (0, [], 4, 8),
                (0, [(1, 0), (1, 0), (1, 0)], 0, 4), (5, [], 0, 4), (0, [], 0, 2)]:
        with pytest.raises(dc.DcError):
            c.tree.scalar_declare([bad], temps)
    with pytest.raises(dc.DcError):      # misaligned temporaries
        c.tree.scalar_declare([(0, [], 0, 4)], temps.view(torch.uint8)[4:12])
    c.tree.scalar_declare([(0, [(1, 0), (1, 0)], 0, 4)], temps)
    assert int(temps[0]) == 10
    c.tree.detach()
    with pytest.raises(dc.DcError):      # detached: host pointers in the arena
        c.tree.scalar_declare([(0, [], 0, 4)], temps)
