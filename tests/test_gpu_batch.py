"""GPU parity of the batched form: every structure's relocation and leaf
kernel in one persistent launch, its HIP-graph replays, and the autotuner.
Results must not depend on the tile shape."""
import ctypes

import numpy as np
import pytest

import fixtures as fx
import oracle as orc
from tests.test_gpu_parity import Copy, assert_same_bytes, ctx  # noqa: F401

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _staged_after_kernel(c, iters):
    """The staged image (host pointers in the slots) with every leaf advanced
    by `iters` oracle passes."""
    ref = orc.OracleCopy(c.t.types, c.t.root_type, c.t.roots, c.oracle.align, c.base)
    ref.run_kernel(1.0001, 0.5, iters=iters, select="all")
    img = c.raw_image()
    ar = ref.arena()
    for o in ref.objects():
        if o["kind"] in (1, 2) and o["bytes"]:
            lo, hi = int(o["off"]), int(o["off"]) + int(o["bytes"])
            img[lo:hi] = ar[lo:hi]
    return img


def test_batch_md_attach(ctx):
    t = fx.md(nsims=100)
    c = Copy(ctx, t, relocate=False)
    assert_same_bytes(c.device_arena(), c.raw_image(), "staged")
    c.tree.batch_run(a=1.0001, b=0.5, attach=True, detach=False)
    c.oracle.run_kernel(1.0001, 0.5, iters=1, select="all")
    assert_same_bytes(c.device_arena(), c.oracle.arena(), "batched attach+compute")
    c.tree.check()
    # the tree is attached now: plain kernels and chains work on it
    assert c.tree.resolve_chain([(0, 3), (2, 0)], root_index=7) == c.oracle.resolve_chain(7, [(0, 3), (2, 0)])


SHAPES = [None,
          # one persistent launch, one relocation unit per item
          dict(block=256, wg_per_cu=8, launches=0), dict(block=512, wg_per_cu=4, launches=0),
          dict(block=1024, wg_per_cu=2, launches=0), dict(block=256, wg_per_cu=1, launches=0),
          # one persistent launch in three phases
          dict(block=256, wg_per_cu=2, tile_chunks=1024, launches=2),
          dict(block=512, wg_per_cu=4, tile_chunks=4096, launches=2),
          dict(block=1024, wg_per_cu=1, tile_chunks=65536, launches=2),
          dict(block=256, wg_per_cu=4, tile_chunks=1 << 20, launches=2),
          # three launches
          dict(tile_chunks=1024, launches=1), dict(tile_chunks=4096, launches=1),
          # one fused launch: tiles relocate their own leaves' slots
          dict(tile_chunks=512, launches=3), dict(tile_chunks=1024, launches=3), dict(tile_chunks=65536, launches=3),
          # the fused launch's items in a persistent grid fed by device queues
          dict(block=256, wg_per_cu=8, tile_chunks=512, launches=4),
          dict(block=256, wg_per_cu=4, tile_chunks=1024, launches=4),
          dict(block=256, wg_per_cu=1, tile_chunks=65536, launches=4)]


@pytest.mark.parametrize("tune", SHAPES)
def test_batch_attach_detach_any_tile_shape(ctx, tune):
    t = fx.md(seed=5, nsims=60, cells_lo=1, cells_hi=40, mean_atoms=5)
    c = Copy(ctx, t, relocate=False)
    assert c.plan.info().unit_leaves == 1
    want = _staged_after_kernel(c, 1)
    c.tree.batch_run(a=1.0001, b=0.5, attach=True, detach=True, tune=tune)
    assert_same_bytes(c.device_arena(), want, f"batched attach+compute+detach {tune}")
    c.tree.check()


@pytest.mark.parametrize("launches", [0, 1, 2, 3, 4])
def test_batch_each_flag_combination(ctx, launches):
    """ATTACH alone, then neither (compute on the attached tree), then DETACH
    alone, each compared with the oracle's arena at that point: attached and
    advanced one pass, two passes, then staged again after three."""
    t = fx.md(seed=15, nsims=80, cells_lo=1, cells_hi=60, mean_atoms=7)
    c = Copy(ctx, t, relocate=False)
    tune = dict(block=256 if launches == 4 else 512, wg_per_cu=2, tile_chunks=2048, launches=launches)
    ref = c.oracle
    c.tree.batch_run(a=1.0001, b=0.5, attach=True, detach=False, tune=tune)
    ref.run_kernel(1.0001, 0.5, iters=1, select="all")
    assert_same_bytes(c.device_arena(), ref.arena(), f"attach only, launches {launches}")
    c.tree.batch_run(a=1.0001, b=0.5, attach=False, detach=False, tune=tune)
    ref.run_kernel(1.0001, 0.5, iters=1, select="all")
    assert_same_bytes(c.device_arena(), ref.arena(), f"compute only, launches {launches}")
    c.tree.batch_run(a=1.0001, b=0.5, attach=False, detach=True, tune=tune)
    assert_same_bytes(c.device_arena(), _staged_after_kernel(c, 3), f"detach only, launches {launches}")
    c.tree.check()


@pytest.mark.parametrize("launches", [0, 2, 3])
def test_batch_units_not_contiguous(ctx, launches):
    """A 16-way Dense tree: its relocation units do not own contiguous leaf
    runs, so the persistent launch runs in three phases either way."""
    t = fx.dense(seed=44, q=16, n=10, D=3)
    c = Copy(ctx, t, relocate=False)
    assert c.plan.info().unit_leaves == 0
    want = _staged_after_kernel(c, 1)
    c.tree.batch_run(a=1.0001, b=0.5, attach=True, detach=True, tune=dict(block=256, wg_per_cu=4, launches=launches))
    assert_same_bytes(c.device_arena(), want, f"dense q=16 launches {launches}")
    c.tree.check()


@pytest.mark.parametrize("tune", [dict(block=256, wg_per_cu=1, launches=0),
                                  dict(block=256, wg_per_cu=1, tile_chunks=4096, launches=2),
                                  dict(block=256, wg_per_cu=1, tile_chunks=1024, launches=4)])
def test_batch_many_items_per_workgroup(ctx, tune):
    """600 simulations (~0.7 GB) on one 256-thread workgroup per compute unit:
    every workgroup takes several relocation units (per-unit form), or, in
    three phases, several relocation units and then some twenty batches of
    two compute tiles each, with its phase waits contended by every other
    workgroup, or (persistent fused) some 170 tiles from its queue. The whole
    arena is compared with the oracle."""
    fx.set_threads(0)
    t = fx.md(seed=21, nsims=600)
    c = Copy(ctx, t, relocate=False)
    info = c.plan.info()
    print(f"[md 600] objects {info.nobjects} units {info.nsegments} arena {info.arena_bytes} {tune}", flush=True)
    want = _staged_after_kernel(c, 1)
    c.tree.batch_run(a=1.0001, b=0.5, attach=True, detach=True, tune=tune)
    assert_same_bytes(c.device_arena(), want, f"md 600 sims {tune}")
    c.tree.check()


SMALL = {
    "no leaves": lambda: fx.linear(k=3, n=0),
    "one leaf of one element": lambda: fx.linear(k=2, n=1),
    "plain, 16 leaves": lambda: fx.plain(),
}


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("tune", [dict(tile_chunks=512, launches=3),
                                  dict(block=256, wg_per_cu=8, tile_chunks=512, launches=4),
                                  dict(block=256, wg_per_cu=1, tile_chunks=1024, launches=4)],
                         ids=["fused", "persistent8", "persistent1"])
def test_fused_forms_on_small_trees(ctx, name, tune):
    """Trees with fewer items than the persistent grid has queues or
    workgroups (most queues hand out nothing), no leaves at all, a single
    one-element leaf: attach + pass + detach, then attach + pass, each
    compared with the oracle."""
    t = SMALL[name]()
    c = Copy(ctx, t, relocate=False)
    want = _staged_after_kernel(c, 1)
    c.tree.batch_run(a=1.0001, b=0.5, attach=True, detach=True, tune=tune)
    assert_same_bytes(c.device_arena(), want, f"{name} attach+detach {tune}")
    c.tree.batch_run(a=1.0001, b=0.5, attach=True, detach=False, tune=tune)
    c.oracle.run_kernel(1.0001, 0.5, iters=2, select="all")
    assert_same_bytes(c.device_arena(), c.oracle.arena(), f"{name} attach {tune}")
    c.tree.check()


@pytest.mark.parametrize("tune", [None, dict(tile_chunks=1024, launches=1),
                                  dict(block=256, wg_per_cu=4, tile_chunks=512, launches=4)],
                         ids=["default", "three", "persistent"])
def test_batch_wide_and_out_of_place(ctx, tune):
    t = fx.wide(seed=81, f1=16, f2=16, lo=1, hi=5000)
    c = Copy(ctx, t, relocate=False)
    n = c.plan.info().out_bytes
    out = torch.zeros(n, dtype=torch.uint8, device="cuda")
    c.tree.batch_run(a=0.9999, b=-0.25, attach=True, detach=False, out=out, tune=tune)
    want = np.zeros(n, np.uint8)
    c.oracle.run_kernel(0.9999, -0.25, iters=1, select="all", out=want)
    torch.cuda.synchronize()
    assert_same_bytes(out.cpu().numpy(), want, "batched out-of-place image")
    assert_same_bytes(c.device_arena(), c.oracle.arena(), "arena relocated, leaves untouched")


@pytest.mark.parametrize("launches", [0, 1, 3, 4])
def test_graph_replays(ctx, launches):
    t = fx.md(seed=6, nsims=40, cells_lo=2, cells_hi=30, mean_atoms=8)
    c = Copy(ctx, t, relocate=False)
    g = c.tree.graph(a=1.0001, b=0.5, tune=dict(tile_chunks=1024, launches=launches))
    x = torch.ones(1 << 20, device="cuda")
    for r in range(1, 4):
        g.launch()
        torch.cuda.synchronize()
        assert_same_bytes(c.device_arena(), _staged_after_kernel(c, r), f"graph replay {r}")
        x.mul_(1.5).add_(1.0)  # eager work between replays
        torch.cuda.synchronize()
    c.tree.check()
    g.close()


@pytest.mark.parametrize("launches", [0, 1, 4])
def test_graph_replay_after_another_tile_size(ctx, launches):
    """A graph replays the tile count it was captured with: calls with other
    tile sizes in between rebuild the tree's tile list, and the replay must
    restore its own before it runs."""
    t = fx.md(seed=9, nsims=40, cells_lo=2, cells_hi=30, mean_atoms=8)
    c = Copy(ctx, t, relocate=False)
    g = c.tree.graph(a=1.0001, b=0.5, tune=dict(tile_chunks=1024, launches=launches))
    passes = 0
    for other in (4096, 512, 1 << 16):
        c.tree.batch_run(a=1.0001, b=0.5, attach=True, detach=True, tune=dict(tile_chunks=other, launches=launches))
        g.launch()
        passes += 2
        torch.cuda.synchronize()
        assert_same_bytes(c.device_arena(), _staged_after_kernel(c, passes), f"replay after tiles of {other}")
    c.tree.check()
    g.close()


def test_graph_with_upload_restarts_from_image(ctx):
    t = fx.md(seed=7, nsims=30, cells_lo=2, cells_hi=20, mean_atoms=8)
    c = Copy(ctx, t, relocate=False)
    want = _staged_after_kernel(c, 1)
    g = c.tree.graph(a=1.0001, b=0.5, upload=True, download=True)
    for r in range(3):
        g.launch()
        torch.cuda.synchronize()
        assert_same_bytes(c.device_arena(), want, f"uploaded replay {r}")
    g.close()


@pytest.mark.parametrize("nsims", [30, 500])
@pytest.mark.parametrize("tune", [dict(tile_chunks=1024, launches=3),
                                  dict(block=256, wg_per_cu=8, tile_chunks=1024, launches=4)],
                         ids=["fused", "persistent"])
def test_graph_whole_job_in_and_out(ctx, nsims, tune):
    """The whole job in one graph: the staged image in, attach + pass +
    detach, the arena out (Algorithm 2's transfer, kernel, transfer back).
    Every replay restarts from the staged image, so the image brought back
    and the device arena are, each time, the staged image with every leaf
    advanced one pass by the oracle."""
    from paper_1906_01128_amd import dc
    fx.set_threads(0)
    t = fx.md(seed=41, nsims=nsims)
    c = Copy(ctx, t, relocate=False)
    print(f"[gpu] whole-job graph: {c.plan.arena_bytes} B {tune}", flush=True)
    want = _staged_after_kernel(c, 1)
    g = c.tree.graph(a=1.0001, b=0.5, tune=tune, upload=True, download=True)
    for r in range(3):
        g.launch()
        torch.cuda.synchronize()
        assert_same_bytes(g.image(), want, f"image brought back, replay {r}")
        assert_same_bytes(c.device_arena(), want, f"device arena, replay {r}")
    c.tree.check()
    g.close()
    g2 = c.tree.graph(a=1.0001, b=0.5, tune=tune)
    with pytest.raises(dc.DcError) as e:
        g2.image()
    assert e.value.name == "STATE"
    g2.close()


def test_autotune_then_parity(ctx, tmp_path, monkeypatch):
    monkeypatch.setenv("DC_TUNE_CACHE", str(tmp_path / "tune.json"))
    t = fx.md(seed=8, nsims=200, cells_lo=4, cells_hi=64, mean_atoms=16)
    c = Copy(ctx, t, relocate=False)
    choice = c.tree.autotune(reps=1)
    assert choice["block"] in (256, 512, 1024) and choice["launches"] in (0, 1, 2, 3, 4)
    table = c.tree.autotune_results()
    assert len(table) >= 8 and choice in [tu for tu, _ in table]
    assert all(tu["block"] * tu["wg_per_cu"] <= 2048 for tu, _ in table if tu["launches"] in (0, 2))
    assert any(tu["launches"] == 3 for tu, _ in table)
    assert all(tu["block"] == 256 and tu["wg_per_cu"] <= 8 for tu, _ in table if tu["launches"] == 4)
    assert {tu["wg_per_cu"] for tu, _ in table if tu["launches"] == 4} == {4, 6, 8}
    assert any(tu["block"] == 1024 for tu, _ in table)
    assert (tmp_path / "tune.json").exists()
    # the autotuner changed leaf values; copy again and run with the cached choice
    t2 = fx.md(seed=8, nsims=200, cells_lo=4, cells_hi=64, mean_atoms=16)
    c2 = Copy(ctx, t2, relocate=False)
    c2.tree.batch_run(a=1.0001, b=0.5, attach=True)
    c2.oracle.run_kernel(1.0001, 0.5, iters=1, select="all")
    assert_same_bytes(c2.device_arena(), c2.oracle.arena(), "after autotune")


@pytest.fixture(scope="module")
def md_full(ctx):
    """The full MD workload, planned once, with device buffers and the
    oracle's copy at the same arena address advanced by one pass: every
    full-size case stages the tree again into the same buffers."""
    from paper_1906_01128_amd import dc
    fx.set_threads(0)
    t = fx.md()
    schema = dc.Schema(t.types)
    plan = dc.Plan(schema, t.root_type, t.roots)
    arena = torch.empty(plan.arena_bytes, dtype=torch.uint8, device="cuda")
    scratch = torch.empty(plan.scratch_bytes, dtype=torch.uint8, device="cuda")
    ref = orc.OracleCopy(t.types, t.root_type, t.roots, 64, arena.data_ptr())
    ref.run_kernel(1.0001, 0.5, iters=1, select="all")
    yield t, schema, plan, arena, scratch, ref
    ref.free()
    del arena, scratch


@pytest.mark.slow
@pytest.mark.parametrize("tune", [dict(block=1024, wg_per_cu=2, launches=0),
                                  dict(block=1024, wg_per_cu=2, tile_chunks=16384, launches=2),
                                  dict(tile_chunks=1024, launches=1),
                                  dict(tile_chunks=1024, launches=3),
                                  dict(block=256, wg_per_cu=8, tile_chunks=1024, launches=4),
                                  dict(block=256, wg_per_cu=4, tile_chunks=2048, launches=4)])
def test_batch_md_full_size(ctx, md_full, tune):
    """10,000 simulations, ~7.8 M arrays, ~12 GB, in each batched form with
    an explicit shape (the per-unit persistent launch, the three-phase
    persistent launch in the shape the bench measures, three launches),
    attached and advanced one pass, compared with the oracle over the whole
    arena."""
    from paper_1906_01128_amd import dc
    t, schema, plan, arena, scratch, ref = md_full
    info = plan.info()
    print(f"[md full] objects {info.nobjects} slots {info.nslots_nonnull} arena {info.arena_bytes} {tune}", flush=True)
    tree = dc.Tree(ctx, plan, arena, scratch, relocate=False)
    tree.batch_run(a=1.0001, b=0.5, attach=True, tune=tune)
    torch.cuda.synchronize()
    got = arena[: plan.arena_bytes].cpu().numpy()
    want = ref.arena()
    step = 1 << 30
    for lo in range(0, len(want), step):
        assert np.array_equal(got[lo:lo + step], want[lo:lo + step]), f"md full arena differs in GiB {lo >> 30} {tune}"
    tree.check()
    tree.release()


@pytest.mark.slow
def test_leaf_prefix_md_full_size(ctx, md_full):
    """The device's leaf chunk prefix for 7.7 M leaves (more than a thousand
    scan blocks: block offsets in several rounds), word for word against the
    prefix derived from the oracle's layout."""
    from paper_1906_01128_amd import dc
    from tests.test_gpu_leaf_prefix import device_leaf_prefix, expected_leaf_prefix
    t, schema, plan, arena, scratch, ref = md_full
    assert plan.info().nleaves > 1024 * 1024
    tree = dc.Tree(ctx, plan, arena, scratch, relocate=False)
    got = device_leaf_prefix(plan, scratch)
    want = expected_leaf_prefix(ref.objects())
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} words differ, first at {bad[:8]}"
    tree.check()
    tree.release()


def test_forced_wait_bound_is_reported_and_the_launch_ends(ctx):
    """The persistent launch's waits are bounded. Forced (from the host) to
    wait for one item more than each phase has, every wait ends at a small
    bound, the launch ends, and the next check of the tree reports the error;
    a fresh copy then runs exactly as before."""
    from paper_1906_01128_amd import dc
    t = fx.md(seed=5, nsims=60, cells_lo=1, cells_hi=40, mean_atoms=5)
    c = Copy(ctx, t, relocate=False)
    tune = dict(block=256, wg_per_cu=1, tile_chunks=1024, launches=0, spin_limit=64)
    print(f"[gpu] forced wait bound: {tune}", flush=True)
    c.tree.batch_run(a=1.0001, b=0.5, attach=True, detach=True, tune=tune, force_wait_bound=True)
    torch.cuda.synchronize()
    with pytest.raises(dc.DcError) as e:
        c.tree.check()
    assert e.value.name == "STATE" and "wait bound" in str(e.value)
    c2 = Copy(ctx, t, relocate=False)
    # three launches and the fused ones have no waits to force
    for bad in (dict(tile_chunks=1024, launches=1), dict(tile_chunks=1024, launches=3),
                dict(block=256, wg_per_cu=4, tile_chunks=1024, launches=4)):
        with pytest.raises(dc.DcError) as e:
            c2.tree.batch_run(attach=True, detach=True, tune=bad, force_wait_bound=True)
        assert e.value.name == "INVAL"
    want = _staged_after_kernel(c2, 1)
    c2.tree.batch_run(a=1.0001, b=0.5, attach=True, detach=True, tune=dict(tune, spin_limit=0))
    assert_same_bytes(c2.device_arena(), want, "persistent launch after a forced wait bound")
    c2.tree.check()


def test_persistent_fused_shape_is_checked(ctx):
    """The persistent fused launch takes 256-thread workgroups, at most eight
    per compute unit (all resident at once); other shapes are refused before
    anything is enqueued, and the tree then runs as before."""
    from paper_1906_01128_amd import dc
    t = fx.md(seed=5, nsims=20, cells_lo=1, cells_hi=20, mean_atoms=5)
    c = Copy(ctx, t, relocate=False)
    for bad in (dict(block=512, wg_per_cu=2, tile_chunks=1024, launches=4),
                dict(block=256, wg_per_cu=9, tile_chunks=1024, launches=4),
                dict(block=256, wg_per_cu=4, tile_chunks=1024, launches=5)):
        with pytest.raises(dc.DcError) as e:
            c.tree.batch_run(a=1.0001, b=0.5, attach=True, detach=True, tune=bad)
        assert e.value.name == "INVAL", bad
    want = _staged_after_kernel(c, 1)
    c.tree.batch_run(a=1.0001, b=0.5, attach=True, detach=True,
                     tune=dict(block=256, wg_per_cu=8, tile_chunks=1024, launches=4))
    assert_same_bytes(c.device_arena(), want, "persistent fused after refused shapes")
    c.tree.check()


def test_autotune_and_graph_right_after_staging(ctx, tmp_path, monkeypatch):
    """The autotuner and the graph capture run on streams of their own; called
    right after staging, with the staging copies still in flight on the
    caller's stream, they must wait for them (a ~0.6 GB tree, as the bench's
    500-simulation comparison stages just before autotuning)."""
    from paper_1906_01128_amd import dc
    monkeypatch.setenv("DC_TUNE_CACHE", str(tmp_path / "tune.json"))
    fx.set_threads(0)
    t = fx.md(seed=31, nsims=500)
    schema = dc.Schema(t.types)
    plan = dc.Plan(schema, t.root_type, t.roots)
    arena = torch.empty(plan.arena_bytes, dtype=torch.uint8, device="cuda")
    scratch = torch.empty(plan.scratch_bytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    print(f"[gpu] stage then autotune at once: {plan.arena_bytes} B", flush=True)
    tree = dc.Tree(ctx, plan, arena, scratch, relocate=False)
    tree.autotune(reps=1)
    tree.check()
    tree.release()
    # stage again and capture with the image upload at once: the captured
    # image must be the staged one
    tree = dc.Tree(ctx, plan, arena, scratch, relocate=False)
    g = tree.graph(a=1.0001, b=0.5, tune=dict(tile_chunks=1024, launches=1), upload=True)
    g.launch()
    torch.cuda.synchronize()
    ref = orc.OracleCopy(t.types, t.root_type, t.roots, 64, arena.data_ptr())
    ref.run_kernel(1.0001, 0.5, iters=1, select="all")
    img = ref.arena().copy()
    for o in ref.objects():    # staged again after the replay's detach: host pointers in the slots
        if o["kind"] == 0 and o["bytes"]:
            lo, hi = int(o["off"]), int(o["off"]) + int(o["bytes"])
            img[lo:hi] = np.frombuffer(ctypes.string_at(int(o["host"]), int(o["bytes"])), np.uint8)
    assert_same_bytes(arena[: plan.arena_bytes].cpu().numpy(), img, "graph captured right after staging")
    tree.check()
    g.close()
    tree.release()
    ref.free()


FUSED = [dict(tile_chunks=512, launches=3), dict(block=256, wg_per_cu=2, tile_chunks=512, launches=4)]


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("detach", [False, True])
@pytest.mark.parametrize("fused", FUSED, ids=["fused", "persistent"])
def test_fused_random_graphs(ctx, seed, detach, fused):
    """The fused launch on random pointer graphs: null members, arrays reached
    twice (the second slot is translated apart from the tiles), cycles,
    zero-length arrays and struct arrays, several roots; 512-chunk tiles so
    that long leaves span several tiles."""
    t = fx.random_tree(5100 + seed, max_objects=80, nroots=1 + seed % 3)
    c = Copy(ctx, t, align=[16, 64, 256][seed % 3], relocate=False)
    ref = c.oracle
    c.tree.batch_run(a=1.0001, b=0.5, attach=True, detach=detach, tune=fused)
    ref.run_kernel(1.0001, 0.5, iters=1, select="all")
    if detach:
        assert_same_bytes(c.device_arena(), _staged_after_kernel(c, 1), f"fused attach+detach seed {seed}")
    else:
        assert_same_bytes(c.device_arena(), ref.arena(), f"fused attach seed {seed}")
        # and detach alone afterwards, with one more pass
        c.tree.batch_run(a=1.0001, b=0.5, attach=False, detach=True, tune=fused)
        assert_same_bytes(c.device_arena(), _staged_after_kernel(c, 2), f"fused detach seed {seed}")
    c.tree.check()


@pytest.mark.parametrize("fused", FUSED, ids=["fused", "persistent"])
def test_fused_selective_and_long_leaves(ctx, fused):
    """A selective copy (unfollowed members are zeroed, apart from the
    tiles) and leaves of up to 40,000 elements spread over many 512-chunk
    tiles, compared with the oracle after attach, and after attach + detach."""
    t = fx.wide(seed=91, f1=6, f2=9, lo=1, hi=40000)
    follow = [0b1, 0b1, 0b01]   # the leaf structs follow their f32 member only
    c = Copy(ctx, t, relocate=False, follow=follow)
    c.tree.batch_run(a=0.9999, b=-0.25, attach=True, detach=False, tune=fused)
    c.oracle.run_kernel(0.9999, -0.25, iters=1, select="all")
    assert_same_bytes(c.device_arena(), c.oracle.arena(), f"fused selective attach {fused}")
    c.tree.check()
