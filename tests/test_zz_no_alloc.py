"""The deep copy that allocates nothing (dc_deep_copy_to_device_noalloc),
through the C ABI, against the ordinary deep copy into a caller scratch
buffer: same arena bytes after the copy, after a pass over every leaf and
after a per-access pass over one chain, and the same host tree after the
copy back. Two calls in a row, the second with a smaller tree, so the fixed
array holds the first call's tables when the second begins."""
import ctypes

import numpy as np
import pytest

import fixtures as fx
import oracle as orc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_1906_01128_amd import dc
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return dc.Context(0)


def _leaf_bytes(t, plan):
    """Every FP32/FP64 array of the host tree, in plan order, as bytes."""
    objs = plan.objects()
    return b"".join(ctypes.string_at(int(o["host"]), int(o["bytes"]))
                    for o in objs if o["kind"] in (1, 2) and o["bytes"])


def _one(ctx, t, plan, arena, noalloc, chain):
    """Deep copy, one pass over every leaf, two per-access passes over one
    chain, copy back; the arena after each step and the host leaves after."""
    from paper_1906_01128_amd import dc
    scratch = None
    if noalloc:
        tree = dc.Tree.noalloc(ctx, plan, arena)
    else:
        scratch = torch.empty(plan.scratch_bytes, dtype=torch.uint8, device="cuda")
        tree = dc.Tree(ctx, plan, arena, scratch)
    snaps = []
    torch.cuda.synchronize()
    snaps.append(arena[: plan.arena_bytes].cpu().numpy().copy())
    tree.run_kernel(mode="resolved", select="all", iters=1, a=1.0001, b=0.5)
    torch.cuda.synchronize()
    snaps.append(arena[: plan.arena_bytes].cpu().numpy().copy())
    tree.run_kernel(mode="deref_each", select="chain", chain=chain, iters=2, a=0.9999, b=-0.25)
    torch.cuda.synchronize()
    snaps.append(arena[: plan.arena_bytes].cpu().numpy().copy())
    tree.check()
    tree.copy_back()
    host = _leaf_bytes(t, plan)
    tree.release()
    return snaps, host


@pytest.mark.parametrize("first,second", [(dict(nsims=120), dict(nsims=7, cells_lo=1, cells_hi=9))])
def test_noalloc_matches_the_scratch_copy_twice(ctx, first, second):
    from paper_1906_01128_amd import dc
    for k, shape in enumerate((first, second)):
        # the same tree built twice from one seed: one per entry point, since
        # the copy back writes the host leaves
        ta = fx.md(seed=700 + k, **shape)
        tb = fx.md(seed=700 + k, **shape)
        schema = dc.Schema(ta.types)
        pa = dc.Plan(schema, ta.root_type, ta.roots)
        pb = dc.Plan(schema, tb.root_type, tb.roots)
        assert pa.scratch_bytes <= dc.NOALLOC_SCRATCH_BYTES
        arena = torch.empty(pa.arena_bytes, dtype=torch.uint8, device="cuda")
        chain = [(0, 3), (2, 0)] if k == 0 else [(0, 0), (2, 0)]   # the small tree's first sim may hold one cell
        print(f"[gpu] noalloc call {k}: {len(ta.roots)} sims, arena {pa.arena_bytes} B, tables {pa.scratch_bytes} B",
              flush=True)
        want, want_host = _one(ctx, ta, pa, arena, False, chain)
        got, got_host = _one(ctx, tb, pb, arena, True, chain)
        for step, (g, w) in enumerate(zip(got, want)):
            bad = np.nonzero(g != w)[0]
            assert bad.size == 0, f"call {k} step {step}: {bad.size} arena bytes differ, first at {bad[:6]}"
        assert got_host == want_host, f"call {k}: copied-back leaves differ"
        # and both equal the oracle's copy at this arena address after the same passes
        tc = fx.md(seed=700 + k, **shape)
        ref = orc.OracleCopy(tc.types, tc.root_type, tc.roots, 64, arena.data_ptr())
        assert np.array_equal(ref.arena(), want[0]), f"call {k}: deep copy differs from the oracle"
        ref.free()


def test_noalloc_refusals(ctx):
    from paper_1906_01128_amd import dc
    t = fx.md(seed=711, nsims=20, cells_lo=2, cells_hi=20)
    schema = dc.Schema(t.types)
    plan = dc.Plan(schema, t.root_type, t.roots)
    arena = torch.empty(plan.arena_bytes, dtype=torch.uint8, device="cuda")
    tree = dc.Tree.noalloc(ctx, plan, arena)
    # one tree at a time holds the fixed array
    with pytest.raises(dc.DcError) as e:
        dc.Tree.noalloc(ctx, plan, arena)
    assert e.value.name == "STATE"
    tree.release()
    tree = dc.Tree.noalloc(ctx, plan, arena)   # free again after the release
    tree.check()
    tree.release()
    # an arena too small
    small = torch.empty(plan.arena_bytes // 2 + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(dc.DcError) as e:
        dc.Tree.noalloc(ctx, plan, small)
    assert e.value.name == "RANGE"
    # tables larger than the fixed array: refused before anything is copied
    big = fx.md(seed=712, nsims=1500)
    bplan = dc.Plan(schema, big.root_type, big.roots)
    assert bplan.scratch_bytes > dc.NOALLOC_SCRATCH_BYTES
    with pytest.raises(dc.DcError) as e:
        dc.Tree.noalloc(ctx, bplan, arena)
    assert e.value.name == "RANGE"
    # the refusals left the array free
    tree = dc.Tree.noalloc(ctx, plan, arena)
    tree.release()
