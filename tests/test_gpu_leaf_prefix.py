"""GPU parity of the leaves' 16-byte-chunk prefix that the deep copy computes
on the device (the sizing step of Algorithm 1, for the leaves): read from the
caller's scratch buffer and compared word for word with the prefix derived
from the oracle's layout. Covers no leaves, one scan block, several blocks
with a ragged tail, zero-length and odd-sized FP32 leaves; the full MD
workload (more than a thousand scan blocks, so the block offsets are taken
in several rounds) is in test_gpu_batch.py."""
import numpy as np
import pytest

import fixtures as fx
import oracle as orc
from tests.test_gpu_parity import Copy, ctx  # noqa: F401

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def expected_leaf_prefix(objs):
    """From the oracle's object table: the FP32/FP64 arrays with at least one
    element, in arena order, each rounded up to whole 16-byte chunks; the
    exclusive prefix of those counts, then their total."""
    objs = np.sort(objs, order="off")
    leaves = objs[((objs["kind"] == 1) | (objs["kind"] == 2)) & (objs["count"] > 0)]
    chunks = (leaves["bytes"].astype(np.uint64) + np.uint64(15)) // np.uint64(16)
    out = np.zeros(len(leaves) + 1, np.uint64)
    np.cumsum(chunks, out=out[1:])
    return out


def device_leaf_prefix(plan, scratch):
    info = plan.info()
    lo = int(info.leaf_prefix_offset)
    n = int(info.nleaves) + 1
    assert lo % 8 == 0 and lo + 8 * n <= int(info.scratch_bytes)
    torch.cuda.synchronize()
    return scratch[lo: lo + 8 * n].cpu().numpy().view(np.uint64)


CASES = {
    "no leaves": lambda: fx.linear(k=3, n=0),
    "plain, one block": lambda: fx.plain(),
    "random graphs, zero-length arrays": lambda: fx.random_tree(11, max_objects=4000, nroots=300),
    "wide, odd FP32 lengths, 3 blocks": lambda: fx.wide(f1=8, f2=300, lo=1, hi=300),
    "md, 5 blocks ragged": lambda: fx.md(seed=3, nsims=40, cells_lo=8, cells_hi=64, mean_atoms=5),
    "wide, exactly 2 full blocks": lambda: fx.wide(f1=8, f2=256, lo=1, hi=100),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("relocate", [True, False])
def test_leaf_prefix_matches_oracle_layout(ctx, name, relocate):
    t = CASES[name]()
    c = Copy(ctx, t, relocate=relocate)
    want = expected_leaf_prefix(c.oracle.objects())
    assert int(c.plan.info().nleaves) + 1 == len(want)
    got = device_leaf_prefix(c.plan, c.scratch)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{name}: {bad.size} words differ, first at {bad[:8]}"
    c.tree.check()


def test_leaf_prefix_rewritten_by_each_copy(ctx):
    """Scratch filled with ones first: every word is written by the copy."""
    t = fx.md(seed=9, nsims=30, cells_lo=8, cells_hi=80, mean_atoms=4)
    c = Copy(ctx, t)
    c.scratch.fill_(0xFF)
    from paper_1906_01128_amd import dc
    tree = dc.Tree(ctx, c.plan, c.arena, c.scratch)
    got = device_leaf_prefix(c.plan, c.scratch)
    assert np.array_equal(got, expected_leaf_prefix(c.oracle.objects()))
    tree.check()
    tree.release()
