"""The RESOLVED leaf pass follows each leaf's relocated parent slot (the
resolved address of Section 3), not the plan: it starts loading a leaf at
its planned address while the slot is still being read, and whatever the
slot turns out to hold is what is computed. Here one leaf's member is
pointed, on the device, at another leaf of the same size and kind, and the
out-of-place image must show the other leaf's values in the first leaf's
place (an in-place pass would update the other leaf twice, racing). The
kick-drift kernel is checked the same way, with two cells' position members
swapped."""
import numpy as np
import pytest

import fixtures as fx
from tests.test_gpu_parity import Copy, assert_same_bytes, ctx  # noqa: F401

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _image_offsets(objs, align):
    """Offsets of the leaves in the out-of-place image (arena order, each at the
    next multiple of the alignment after the previous one's end) and its size
    (the last end, aligned)."""
    offs, end, first = {}, 0, True
    for k in np.argsort(objs["off"], kind="stable"):
        o = objs[k]
        if o["kind"] not in (1, 2):
            continue
        off = 0 if first else -(-end // align) * align
        end = off + max(int(o["bytes"]), 1)
        first = False
        offs[int(o["off"])] = off
    return offs, -(-end // align) * align


def _slot_of(c, leaf_off):
    """Arena offset of the 8-byte member that holds the leaf's device address."""
    a = c.device_arena()
    words = a[: len(a) // 8 * 8].view(np.uint64)
    hits = np.nonzero(words == np.uint64(c.base + leaf_off))[0]
    assert hits.size == 1, hits
    return int(hits[0]) * 8


CASES = {
    # small MD leaves: the redirected leaf lies within its tile's first round
    "md": lambda: fx.md(seed=fx.SEED_BASE + 71, nsims=30, cells_lo=2, cells_hi=6, mean_atoms=8),
    # 40 KB leaves: several tiles and several rounds per leaf
    "wide": lambda: fx.wide(seed=fx.SEED_BASE + 72, f1=3, f2=4, lo=5000, hi=5000),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_resolved_pass_follows_a_redirected_member(ctx, case):
    t = CASES[case]()
    c = Copy(ctx, t)
    objs = c.oracle.objects()
    f64 = [o for o in objs if o["kind"] == 2 and o["count"]]
    by_size = {}
    for o in f64:
        by_size.setdefault(int(o["bytes"]), []).append(o)
    pair = next(v for v in by_size.values() if len(v) >= 2)
    A, B = pair[0], pair[-1]
    n = c.tree.out_bytes(select="all")
    offs, end = _image_offsets(objs, 64)
    assert end == n == c.oracle.out_bytes("all")
    want = np.zeros(n, np.uint8)
    c.oracle.run_kernel(1.0001, 0.5, select="all", out=want)
    ia, ib, nb = offs[int(A["off"])], offs[int(B["off"])], int(A["bytes"])
    want[ia: ia + nb] = want[ib: ib + nb]
    slot = _slot_of(c, int(A["off"]))
    c.arena[slot: slot + 8] = torch.tensor(
        np.frombuffer(int(c.base + int(B["off"])).to_bytes(8, "little"), np.uint8).copy(), device="cuda")
    before = c.device_arena()
    out = torch.zeros(n, dtype=torch.uint8, device="cuda")
    print(f"[gpu] {case}: member at {slot} redirected from {int(A['off'])} to {int(B['off'])}", flush=True)
    c.tree.run_kernel(select="all", a=1.0001, b=0.5, out=out)
    torch.cuda.synchronize()
    c.tree.check()
    assert_same_bytes(out.cpu().numpy(), want, "image with the redirected member")
    assert_same_bytes(c.device_arena(), before, "arena unchanged")


def test_kick_drift_follows_swapped_members(ctx):
    """Two cells of the same length have their position members swapped on
    the device: each cell's drift lands in the other's position array, with
    its own kicked velocity (the kernel follows the relocated members)."""
    import oracle as orc
    t = fx.md(seed=fx.SEED_BASE + 73, nsims=6, cells_lo=3, cells_hi=9, mean_atoms=6)
    c = Copy(ctx, t)
    cell, size = 1, t.types[1].size          # the MD cell: natoms@0, pos@8, vel@16, force@24
    before = c.device_arena()
    word = lambda buf, off: int.from_bytes(buf[off: off + 8].tobytes(), "little")
    objs = c.oracle.objects()
    nbytes = {int(o["off"]): int(o["bytes"]) for o in objs}
    by_len = {}
    for o in objs:
        if o["kind"] == 0 and o["type"] == cell:
            for e in range(int(o["count"])):
                el = int(o["off"]) + e * size
                arrays = [word(before, el + m) - c.base for m in (8, 16, 24)]
                by_len.setdefault(nbytes[arrays[0]], []).append((el, arrays))
    (ea, A), (eb, B) = next(v for k, v in sorted(by_len.items()) if k > 0 and len(v) >= 2)[:2]
    n = nbytes[A[0]] // 8
    dt, dtm = 1e-3, 1e-3 / 39.948
    c.oracle.kick_drift(cell, 0, 1, 2, dt, dtm)
    want = c.oracle.arena().copy()
    f64 = lambda buf, off: buf[off: off + 8 * n].view(np.float64)
    # the cell whose member now points at the other's positions drifts them with its own velocity
    for pos, vel in ((B[0], A[1]), (A[0], B[1])):
        x0, v1 = f64(before, pos).copy(), f64(want, vel)
        f64(want, pos)[:] = [orc.fma64(float(v), dt, float(x)) for v, x in zip(v1, x0)]
    for el, target in ((ea, B[0]), (eb, A[0])):
        b = np.frombuffer(int(c.base + target).to_bytes(8, "little"), np.uint8).copy()
        want[el + 8: el + 16] = b
        c.arena[el + 8: el + 16] = torch.tensor(b, device="cuda")
    torch.cuda.synchronize()
    print(f"[gpu] cells at {ea} and {eb} ({n} doubles) swap their position members", flush=True)
    c.tree.kick_drift(cell, 0, 1, 2, dt, dtm, steps=1)
    torch.cuda.synchronize()
    c.tree.check()
    assert_same_bytes(c.device_arena(), want, "kick-drift with swapped members")
