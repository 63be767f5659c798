"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit
for bit. Layouts, offsets and relocated pointers are compared as raw arena
bytes (the oracle lays its buffer out as if at the device arena's address);
leaf values are compared with a tolerance of 0 ulp."""
import ctypes
import os

import numpy as np
import pytest

import fixtures as fx
import oracle as orc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def ctx():
    _need_gpu()
    from paper_1906_01128_amd import dc
    print(f"[gpu] libdc {dc.version()} on {torch.cuda.get_device_name(0)}", flush=True)
    return dc.Context(0)


def _alloc(n):
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device="cuda")


class Copy:
    """A tree deep-copied by libdc, plus the oracle's copy at the same base."""

    def __init__(self, ctx, t, align=64, relocate=True, follow=None):
        from paper_1906_01128_amd import dc
        self.t = t
        self.schema = dc.Schema(t.types)
        self.plan = dc.Plan(self.schema, t.root_type, t.roots, align=align, follow=follow)
        self.arena = _alloc(self.plan.arena_bytes)
        self.scratch = _alloc(self.plan.scratch_bytes)
        self.tree = dc.Tree(ctx, self.plan, self.arena, self.scratch, relocate=relocate)
        self.base = self.arena.data_ptr()
        self.oracle = orc.OracleCopy(t.types, t.root_type, t.roots, align, self.base, follow=follow)

    def device_arena(self):
        torch.cuda.synchronize()
        return self.arena[: self.plan.arena_bytes].cpu().numpy()

    def raw_image(self):
        """What the arena holds before relocation: every object's host bytes
        at the oracle's offsets, zeros between."""
        img = np.zeros(self.oracle.arena_bytes, np.uint8)
        for o in self.oracle.objects():
            if o["bytes"]:
                img[int(o["off"]): int(o["off"]) + int(o["bytes"])] = np.frombuffer(
                    ctypes.string_at(int(o["host"]), int(o["bytes"])), np.uint8)
        return img


def assert_same_bytes(got, want, what):
    assert got.shape == want.shape, f"{what}: {got.shape} vs {want.shape}"
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{what}: {bad.size} bytes differ, first at {bad[:8]}"


def leaf_views(objs, arena):
    out = []
    for o in objs:
        if o["kind"] in (1, 2) and o["count"]:
            dt = np.float32 if o["kind"] == 1 else np.float64
            out.append(arena[int(o["off"]): int(o["off"]) + int(o["bytes"])].view(dt))
    return out


# ---- the plain workload (16 children x 1024 FP64), end to end -------------------------------

def test_plain_deep_copy_kernel_copy_back(ctx):
    t = fx.plain()
    t_ref = fx.plain()  # the same seed builds the same values
    c = Copy(ctx, t)
    assert_same_bytes(c.device_arena(), c.oracle.arena(), "arena after relocation")
    c.tree.run_kernel(mode="resolved", select="all", iters=1, a=1.0001, b=0.5)
    c.oracle.run_kernel(1.0001, 0.5, iters=1, select="all")
    assert_same_bytes(c.device_arena(), c.oracle.arena(), "arena after kernel")
    c.tree.copy_back()
    ro = orc.OracleCopy(t_ref.types, t_ref.root_type, t_ref.roots, 64, c.base)
    ro.run_kernel(1.0001, 0.5, iters=1, select="all")
    ro.copy_back()
    for a, b in zip(t.snapshot(), t_ref.snapshot()):
        assert a == b
    # host pointers untouched
    assert int.from_bytes(ctypes.string_at(t.roots[0] + 8, 8), "little") == t.allocs[1].base


@pytest.mark.parametrize("mode", ["resolved", "deref_each"])
def test_plain_chain_kernels(ctx, mode):
    t = fx.plain()
    c = Copy(ctx, t)
    for i in (0, 7, 15):
        chain = [(0, i), (0, 0)]
        assert c.tree.resolve_chain(chain) == c.oracle.resolve_chain(0, chain)
        c.tree.run_kernel(mode=mode, select="chain", chain=chain, iters=3, a=0.9999, b=-0.25)
        c.oracle.run_kernel(0.9999, -0.25, iters=3, select="chain", chain=chain)
    assert_same_bytes(c.device_arena(), c.oracle.arena(), f"arena after chain kernels ({mode})")


# ---- the Linear chain: 8 nodes, 2^24 FP64, 100 passes --------------------------------------

@pytest.mark.parametrize("mode", ["resolved", "deref_each"])
def test_linear_chain_100_passes(ctx, mode):
    t = fx.linear()
    c = Copy(ctx, t)
    chain = [(1, 0)] * 7 + [(0, 0)]
    addr, n, kind = c.tree.resolve_chain(chain)
    assert (addr, n, kind) == (c.base + 512, 1 << 24, "f64")
    c.tree.run_kernel(mode=mode, select="chain", chain=chain, iters=100, a=1.0001, b=0.5)
    c.oracle.run_kernel(1.0001, 0.5, iters=100, select="chain", chain=chain)
    assert_same_bytes(c.device_arena(), c.oracle.arena(), f"linear arena after 100 passes ({mode})")
    c.tree.copy_back()
    got = np.frombuffer(ctypes.string_at(t.allocs[-1].base, 8 << 24), np.uint64)
    want = c.oracle.arena()[512:512 + (8 << 24)].view(np.uint64)
    assert np.array_equal(got, want)


# ---- the wide tree: 64 x 64 leaves, FP32 and FP64, ~0.28 GB ---------------------------------

def test_wide_all_leaves(ctx):
    t = fx.wide()
    c = Copy(ctx, t)
    assert_same_bytes(c.device_arena(), c.oracle.arena(), "wide arena after relocation")
    c.tree.run_kernel(mode="resolved", select="all", iters=1, a=1.0001, b=0.5)
    c.oracle.run_kernel(1.0001, 0.5, iters=1, select="all")
    assert_same_bytes(c.device_arena(), c.oracle.arena(), "wide arena after kernel")


@pytest.mark.slow
def test_wide_1g_all_leaves(ctx):
    """The wide-1G variant (leaf lengths up to 2^18, ~0.96 GB), whole arena."""
    t = fx.wide(hi=1 << 18)
    c = Copy(ctx, t)
    c.tree.run_kernel(mode="resolved", select="all", iters=1, a=1.0001, b=0.5)
    c.oracle.run_kernel(1.0001, 0.5, iters=1, select="all")
    assert_same_bytes(c.device_arena(), c.oracle.arena(), "wide-1G arena after kernel")


def test_wide_deref_each_small(ctx):
    t = fx.wide(f1=6, f2=5, lo=1, hi=300)
    c = Copy(ctx, t)
    c.tree.run_kernel(mode="deref_each", select="all", iters=2, a=0.9999, b=-0.25)
    c.oracle.run_kernel(0.9999, -0.25, iters=2, select="all")
    assert_same_bytes(c.device_arena(), c.oracle.arena(), "wide arena after deref kernel")


# ---- edge cases ------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_random_graphs_attach_detach(ctx, seed):
    t = fx.random_tree(3000 + seed, max_objects=80, nroots=1 + seed % 3)
    c = Copy(ctx, t, align=[16, 64, 256][seed % 3], relocate=False)
    raw = c.raw_image()
    assert_same_bytes(c.device_arena(), raw, "staged image")
    c.tree.attach()
    assert_same_bytes(c.device_arena(), c.oracle.arena(), "after attach")
    c.tree.run_kernel(select="all", a=1.0001, b=0.5, iters=2)
    c.oracle.run_kernel(1.0001, 0.5, iters=2, select="all")
    assert_same_bytes(c.device_arena(), c.oracle.arena(), "after kernel")
    c.tree.detach()
    after = c.device_arena()
    # detached: host pointers back in every slot, leaf values kept
    c.tree.attach()
    assert_same_bytes(c.device_arena(), c.oracle.arena(), "after detach + attach")
    c.tree.check()
    assert after.shape == raw.shape


def test_ragged_and_empty_leaves(ctx):
    # leaf lengths 0..40 elements of both kinds: every tail shape of a 16-byte chunk
    t = fx.wide(seed=77, f1=3, f2=41, lo=1, hi=41)
    c = Copy(ctx, t)
    for it in range(3):
        c.tree.run_kernel(select="all", a=1.0001, b=0.5)
        c.oracle.run_kernel(1.0001, 0.5, select="all")
    assert_same_bytes(c.device_arena(), c.oracle.arena(), "ragged leaves")
    # a tree with no leaves at all
    t2 = fx.linear(k=3, n=0)
    c2 = Copy(ctx, t2)
    c2.tree.run_kernel(select="all", a=1.0001, b=0.5)
    assert_same_bytes(c2.device_arena(), c2.oracle.arena(), "no leaves")


def test_out_of_place(ctx):
    t = fx.wide(seed=78, f1=4, f2=9, lo=1, hi=2000)
    c = Copy(ctx, t)
    n = c.tree.out_bytes(select="all")
    assert n == c.oracle.out_bytes("all")
    out = torch.zeros(n, dtype=torch.uint8, device="cuda")
    before = c.device_arena()
    c.tree.run_kernel(select="all", a=0.9999, b=0.5, iters=2, out=out)
    want = np.zeros(n, np.uint8)
    c.oracle.run_kernel(0.9999, 0.5, iters=2, select="all", out=want)
    torch.cuda.synchronize()
    assert_same_bytes(out.cpu().numpy(), want, "out-of-place image")
    assert_same_bytes(c.device_arena(), before, "arena unchanged")


def test_fp32_double_rounding_case(ctx):
    # x = a = 1 + 2^-12, b = 2^-80: fma in binary32 differs from rounding via binary64
    t = fx.wide(seed=79, f1=1, f2=1, lo=8, hi=8)
    x = np.float32(1 + 2.0 ** -12)
    leaf = [a for a in t.allocs if a.kind == "f32"][0]
    ctypes.memmove(leaf.base, np.full(8, x, np.float32).tobytes(), 32)
    c = Copy(ctx, t)
    c.tree.run_kernel(select="all", a=float(x), b=2.0 ** -80, af=float(x), bf=2.0 ** -80)
    got = c.device_arena()[int(c.oracle.objects()["off"][-1]):][:32].view(np.float32)
    assert np.all(got == np.float32(1 + 2.0 ** -11 + 2.0 ** -23))


def test_errors(ctx):
    from paper_1906_01128_amd import dc
    t = fx.linear(k=4, n=10)
    c = Copy(ctx, t, relocate=False)
    with pytest.raises(dc.DcError) as e:
        c.tree.run_kernel(select="all")
    assert e.value.name == "STATE"
    with pytest.raises(dc.DcError) as e:
        c.tree.detach()
    assert e.value.name == "STATE"
    c.tree.attach()
    with pytest.raises(dc.DcError) as e:  # L0.A is null
        c.tree.resolve_chain([(0, 0)])
    assert e.value.name == "RANGE"
    with pytest.raises(dc.DcError) as e:
        c.tree.resolve_chain([(1, 1), (0, 0)])
    assert e.value.name == "RANGE"
    with pytest.raises(dc.DcError) as e:
        c.tree.resolve_chain([(5, 0)])
    assert e.value.name == "INVAL"
    with pytest.raises(dc.DcError) as e:
        dc.Tree(ctx, c.plan, _alloc(16), c.scratch)
    assert e.value.name == "RANGE"
    # a host pointer changed after planning: the device check catches it
    t2 = fx.plain(nchild=2, leaf_len=4)
    from paper_1906_01128_amd import dc as _dc
    schema = _dc.Schema(t2.types)
    plan = _dc.Plan(schema, t2.root_type, t2.roots)
    arena, scratch = _alloc(plan.arena_bytes), _alloc(plan.scratch_bytes)
    child = t2.allocs[1].base
    old = ctypes.string_at(child + 8, 8)
    ctypes.memmove(child + 8, (int.from_bytes(old, "little") + 8).to_bytes(8, "little"), 8)
    tree = _dc.Tree(ctx, plan, arena, scratch)
    with pytest.raises(_dc.DcError) as e:
        tree.check()
    assert e.value.name == "STATE"
    ctypes.memmove(child + 8, old, 8)


def test_tree_objects_are_device_addresses(ctx):
    t = fx.random_tree(7, max_objects=10, nroots=2)
    c = Copy(ctx, t)
    objs = c.tree.objects()
    want = c.oracle.objects()          # offsets relative to the arena start
    assert len(objs) == len(want)
    assert np.array_equal(objs["off"].astype(np.uint64), want["off"].astype(np.uint64) + np.uint64(c.base))
    for name in ("host", "bytes", "count", "kind"):
        assert np.array_equal(objs[name], want[name]), name
    # every relocated pointer in the arena names one of these addresses
    starts = set(int(x) for x in objs["off"])
    ar = c.device_arena()
    for o in want:
        if o["kind"] == 0:
            ty = t.types[int(o["type"])]
            for e in range(int(o["count"])):
                for f in ty.fields:
                    at = int(o["off"]) + e * ty.size + f.offset
                    p = int(ar[at:at + 8].view(np.uint64)[0])
                    assert p == 0 or p in starts


def _many_types_tree(seed=5):
    """64 struct types (the schema's limit) in a chain: T_i holds a pointer to
    an array of T_{i+1} (two elements every 16 levels, else one) and an FP64
    leaf; the last type has 16 pointer members (the most a type may have),
    each to an FP64 leaf."""
    n = 64
    types = []
    for i in range(n - 1):
        types.append(fx.Type(f"T{i}", 8 * (2 + i % 4), 8,
                             [fx.Field(0, "struct", i + 1, fixed_count=2 if i % 16 == 0 else 1),
                              fx.Field(8, "f64", fixed_count=3 + i % 7)]))
    types.append(fx.Type(f"T{n - 1}", 128, 8, [fx.Field(8 * j, "f64", fixed_count=1 + j) for j in range(16)]))
    t = fx.Tree()
    t.types = types
    t.root_type = 0
    rng = np.random.default_rng(seed)

    def leaf(cnt):
        buf = (ctypes.c_double * cnt)(*rng.uniform(-1, 1, cnt))
        t._keep.append(buf)
        return ctypes.addressof(buf)

    def array(i, cnt):
        ty = types[i]
        buf = ctypes.create_string_buffer(ty.size * cnt)
        t._keep.append(buf)
        base = ctypes.addressof(buf)
        for e in range(cnt):
            for f in ty.fields:
                p = array(f.type, f.fixed_count) if f.kind == "struct" else leaf(f.fixed_count)
                ctypes.c_uint64.from_address(base + e * ty.size + f.offset).value = p
        return base

    t.roots = [array(0, 1)]
    return t


@pytest.mark.parametrize("persistent", [False, True])
def test_many_types_relocate(ctx, persistent):
    """Relocation with the largest type table the schema allows (the
    relocation kernel stages the plan's types in LDS), by the relocation
    kernel and by the persistent batch kernel."""
    t = _many_types_tree()
    c = Copy(ctx, t, relocate=False)
    assert len(t.types) == 64
    assert_same_bytes(c.device_arena(), c.raw_image(), "staged image")
    if persistent:
        c.tree.batch_run(a=1.0001, b=0.5, attach=True, detach=False,
                         tune=dict(block=256, wg_per_cu=2, tile_chunks=1024))
        c.oracle.run_kernel(1.0001, 0.5, select="all")
    else:
        c.tree.attach()
        assert_same_bytes(c.device_arena(), c.oracle.arena(), "after attach")
        c.tree.run_kernel(select="all", a=1.0001, b=0.5)
        c.oracle.run_kernel(1.0001, 0.5, select="all")
    assert_same_bytes(c.device_arena(), c.oracle.arena(), "after kernel")
    c.tree.detach()
    c.tree.attach()
    assert_same_bytes(c.device_arena(), c.oracle.arena(), "after detach + attach")
    c.tree.check()
