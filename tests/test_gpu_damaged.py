"""A damaged arena is reported, not followed: pointer members overwritten
from the host with addresses outside the arena make every kernel that walks
them skip the work and record the error, which dc_tree_check returns. Every
load the kernels issue stays inside the arena (each slot is checked before
it is read), so these runs exit normally."""
import numpy as np
import pytest

import fixtures as fx
from tests.test_gpu_parity import Copy, ctx  # noqa: F401

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

K, N = 8, 5000
CHAIN = [(1, 0)] * (K - 1) + [(0, 0)]


def _damaged(ctx, node, slot_off, value):
    t = fx.linear(seed=fx.SEED_BASE + 61, k=K, n=N, scheme=1)
    c = Copy(ctx, t)
    torch.cuda.synchronize()
    v = value(c) if callable(value) else value
    c.arena[64 * node + slot_off: 64 * node + slot_off + 8] = torch.tensor(
        np.frombuffer(int(v).to_bytes(8, "little"), np.uint8).copy(), device="cuda")
    torch.cuda.synchronize()
    return c


WILD = [0x10, 0xFFFF000000000000, lambda c: c.base + c.plan.arena_bytes + 4096]


@pytest.mark.parametrize("wild", range(len(WILD)))
def test_deref_each_stops_at_a_wild_slot(ctx, wild):
    from paper_1906_01128_amd import dc
    c = _damaged(ctx, 3, 16, WILD[wild])          # node 3's next-level member
    leaf_off = int(c.oracle.objects()[-1]["off"])
    before = c.arena[leaf_off: leaf_off + 8 * N].clone()
    c.tree.run_kernel(mode="deref_each", select="chain", chain=CHAIN, iters=2, a=2.0, b=1.0)
    torch.cuda.synchronize()
    with pytest.raises(dc.DcError):
        c.tree.check()
    assert torch.equal(c.arena[leaf_off: leaf_off + 8 * N], before), "no element was written"


@pytest.mark.parametrize("wild", range(len(WILD)))
def test_resolved_chain_reports_the_mismatch(ctx, wild):
    from paper_1906_01128_amd import dc
    c = _damaged(ctx, 3, 16, WILD[wild])
    c.tree.run_kernel(mode="resolved", select="chain", chain=CHAIN, iters=1, a=2.0, b=1.0)
    torch.cuda.synchronize()
    with pytest.raises(dc.DcError):
        c.tree.check()


@pytest.mark.parametrize("mode", ["resolved", "deref_each"])
def test_all_leaves_skip_a_wild_leaf(ctx, mode):
    from paper_1906_01128_amd import dc
    c = _damaged(ctx, K - 1, 8, 0xFFFF000000000000)   # the last level's data member
    leaf_off = int(c.oracle.objects()[-1]["off"])
    before = c.arena[leaf_off: leaf_off + 8 * N].clone()
    c.tree.run_kernel(mode=mode, select="all", iters=1, a=2.0, b=1.0)
    torch.cuda.synchronize()
    with pytest.raises(dc.DcError):
        c.tree.check()
    assert torch.equal(c.arena[leaf_off: leaf_off + 8 * N], before)


@pytest.mark.parametrize("launches", [0, 1, 2, 3])
def test_batched_forms_skip_a_wild_slot(ctx, launches):
    """In every batched form (per-unit persistent, three launches, three-phase
    persistent, fused), a leaf whose member was overwritten with an address
    outside the arena is neither attached nor computed, the error is
    reported, and nothing past the arena is written."""
    from paper_1906_01128_amd import dc
    t = fx.md(seed=fx.SEED_BASE + 62, nsims=20, cells_lo=2, cells_hi=6, mean_atoms=8)
    schema = dc.Schema(t.types)
    plan = dc.Plan(schema, t.root_type, t.roots)
    guard = 1 << 16
    arena = torch.zeros(plan.arena_bytes + guard, dtype=torch.uint8, device="cuda")
    scratch = torch.empty(plan.scratch_bytes, dtype=torch.uint8, device="cuda")
    tree = dc.Tree(ctx, plan, arena, scratch, relocate=False)
    torch.cuda.synchronize()
    objs = plan.objects()
    cells = [o for o in objs if o["kind"] == 0 and o["type"] == 1][3]
    slot = int(cells["off"]) + 32 + 8                      # cell 1's position member
    host = int.from_bytes(bytes(arena[slot: slot + 8].cpu().numpy()), "little")
    leaf = [o for o in objs if int(o["host"]) == host][0]
    lo, hi = int(leaf["off"]), int(leaf["off"]) + int(leaf["bytes"])
    arena[slot: slot + 8] = torch.tensor(np.frombuffer((0xFFFF000000000000).to_bytes(8, "little"), np.uint8).copy(),
                                         device="cuda")
    before = arena[lo:hi].clone()
    print(f"[gpu] wild slot at {slot}, batched form {launches}", flush=True)
    tree.batch_run(a=2.0, b=1.0, attach=True, detach=True, tune=dict(tile_chunks=1024, launches=launches))
    torch.cuda.synchronize()
    with pytest.raises(dc.DcError):
        tree.check()
    assert torch.equal(arena[lo:hi], before), "the leaf behind the wild member was computed"
    assert int(arena[plan.arena_bytes:].count_nonzero()) == 0, "bytes past the arena were written"
    tree.release()
