"""The served form: jobs of mixed sizes admitted by budget, structures kept
resident, work of several jobs overlapping on the device. Every job's result
must be the same alone and in the mix, and equal to the oracle's."""
import ctypes
import random

import numpy as np
import pytest

import fixtures as fx
import oracle as orc
from tests.test_gpu_parity import ctx  # noqa: F401

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

AB = [(1.0001, 0.5), (1.0001, -0.25), (0.9999, 0.5), (0.9999, -0.25)]


def _structures(n, bytes_hi, seed=0):
    return [fx.broom(seed=9000 + seed + i, bytes_lo=64, bytes_hi=bytes_hi) for i in range(n)]


def _expected(t, a, b):
    c = orc.OracleCopy(t.types, t.root_type, t.roots, 64, 0)
    out = np.zeros(c.out_bytes("all"), np.uint8)
    c.run_kernel(a, b, iters=1, select="all", out=out)
    return out


def _run(srv, jobs, structs):
    """Submits every job, waits for all; returns outputs and results."""
    outs, ids = [], []
    for (si, key, ab) in jobs:
        t = structs[si]
        exp_n = orc.OracleCopy(t.types, t.root_type, t.roots, 64, 0).out_bytes("all")
        buf = np.zeros(max(exp_n, 1), np.uint8)
        outs.append(buf)
        ids.append(srv.submit(t.root_type, t.roots[0], buf.ctypes.data, buf.nbytes, *AB[ab], key=key))
    res = [srv.wait(i, timeout=120.0) for i in ids]
    return outs, res


def test_alone_equals_mix_equals_oracle(ctx):
    from paper_1906_01128_amd import dc
    structs = _structures(8, 1 << 20)
    schema = dc.Schema(structs[0].types)
    rng = random.Random(1)
    jobs = [(rng.randrange(8), 0, rng.randrange(4)) for _ in range(24)]
    jobs = [(si, (si + 1) if k % 2 == 0 else 0, ab) for k, (si, _, ab) in enumerate(jobs)]
    # alone: a fresh server per job
    alone = []
    for j in jobs:
        srv = dc.Server(ctx, schema, budget_bytes=1 << 30, max_inflight=4, nstreams=2)
        o, r = _run(srv, [j], structs)
        srv.close()
        alone.append(o[0])
    # mixed: all submitted at once, structures reused through keys
    srv = dc.Server(ctx, schema, budget_bytes=1 << 30, max_inflight=6, nstreams=4)
    mixed, res = _run(srv, jobs, structs)
    st = srv.stats()
    srv.close()
    assert st.completed == len(jobs) and st.reused > 0
    for k, (j, a, m) in enumerate(zip(jobs, alone, mixed)):
        want = _expected(structs[j[0]], *AB[j[2]])
        assert np.array_equal(a, want), f"job {k} alone differs from the oracle"
        assert np.array_equal(m, want), f"job {k} in the mix differs from the oracle"
    assert all(r.status == 0 for r in res)
    assert all(r.t_done >= r.t_admit >= r.t_submit for r in res)


def test_budget_admission_and_eviction(ctx):
    from paper_1906_01128_amd import dc
    structs = _structures(5, 4 << 20, seed=100)
    schema = dc.Schema(structs[0].types)
    sizes = []
    for t in structs:
        p = dc.Plan(schema, t.root_type, t.roots)
        sizes.append(p.arena_bytes + p.scratch_bytes + p.info().out_bytes)
    budget = max(2 * max(sizes), 8 << 20)
    srv = dc.Server(ctx, schema, budget_bytes=budget, max_inflight=3, nstreams=2)
    jobs = [(i % 5, i % 5 + 1, i % 4) for i in range(15)]  # every structure keyed, cycled
    outs, res = _run(srv, jobs, structs)
    st = srv.stats()
    assert st.peak_bytes <= budget
    assert st.evictions > 0
    for (si, _, ab), o in zip(jobs, outs):
        assert np.array_equal(o, _expected(structs[si], *AB[ab]))
    # a job that can never fit
    small = dc.Server(ctx, schema, budget_bytes=1 << 20, max_inflight=2, nstreams=1)
    big = max(range(5), key=lambda i: sizes[i])
    if sizes[big] > (1 << 20):
        need = orc.OracleCopy(structs[big].types, structs[big].root_type, structs[big].roots, 64, 0).out_bytes("all")
        buf = np.zeros(max(need, 1), np.uint8)
        with pytest.raises(dc.DcError) as e:
            small.submit(structs[big].root_type, structs[big].roots[0], buf.ctypes.data, buf.nbytes, 1.0, 0.0)
        assert e.value.name == "BUDGET"
    small.close()
    srv.close()


def test_wait_timeout_and_unknown_id(ctx):
    """A wait that times out reports DC_E_STATE and leaves the job running;
    waiting again returns its result. An id never issued is DC_E_INVAL."""
    from paper_1906_01128_amd import dc
    t = fx.broom(seed=9300, d_lo=4, d_hi=4, f_lo=16, f_hi=16, bytes_lo=16 << 20, bytes_hi=32 << 20)
    schema = dc.Schema(t.types)
    srv = dc.Server(ctx, schema, budget_bytes=4 << 30, max_inflight=2, nstreams=1)
    need = orc.OracleCopy(t.types, t.root_type, t.roots, 64, 0).out_bytes("all")
    buf = np.zeros(need, np.uint8)
    rid = srv.submit(t.root_type, t.roots[0], buf.ctypes.data, buf.nbytes, *AB[0])
    # hundreds of MB in and out cannot be done at once
    with pytest.raises(dc.DcError) as e:
        srv.wait(rid, timeout=0.0)
    assert e.value.name == "STATE"
    res = srv.wait(rid, timeout=120.0)
    assert res.status == 0
    assert np.array_equal(buf, _expected(t, *AB[0]))
    with pytest.raises(dc.DcError) as e:
        srv.wait(rid + 1000, timeout=0.0)
    assert e.value.name == "INVAL"
    srv.close()


@pytest.mark.slow
def test_served_full_size_whole_images(ctx):
    """The served workload's full distribution (leaf bytes up to 256 MiB, fan-out
    up to 64, depth up to 8): 12 jobs on 6 structures, the second job on each
    reusing the resident copy, all in flight together under the 200 GB budget.
    Every job's whole leaf image (padding between leaves included, which must
    stay as the caller left it) equals the oracle's, byte for byte."""
    from paper_1906_01128_amd import dc
    fx.set_threads(0)
    structs = [fx.broom(seed=190601132 + i, bytes_lo=4096, bytes_hi=256 << 20) for i in range(6)]
    schema = dc.Schema(structs[0].types)
    rng = random.Random(5)
    # every job names its structure's key: the second job on a structure finds it resident
    jobs = [(i % 6, i % 6 + 1, rng.randrange(4)) for i in range(12)]
    srv = dc.Server(ctx, schema, budget_bytes=200 * 10 ** 9, max_inflight=16, nstreams=4)
    outs, ids = [], []
    for si, key, ab in jobs:
        t = structs[si]
        n = orc.OracleCopy(t.types, t.root_type, t.roots, 64, 0).out_bytes("all")
        buf = np.zeros(max(n, 1), np.uint8)
        outs.append(buf)
        ids.append(srv.submit(t.root_type, t.roots[0], buf.ctypes.data, buf.nbytes, *AB[ab], key=key))
    res = [srv.wait(i, timeout=600.0) for i in ids]
    st = srv.stats()
    srv.close()
    assert all(r.status == 0 for r in res)
    assert st.reused == 6
    print(f"[served full] {sum(o.nbytes for o in outs)} output bytes over {len(jobs)} jobs", flush=True)
    for k, (buf, (si, _, ab)) in enumerate(zip(outs, jobs)):
        want = _expected(structs[si], *AB[ab])
        assert buf.nbytes == max(want.nbytes, 1)
        assert np.array_equal(buf[: want.nbytes], want), f"job {k} on structure {si} differs from the oracle"


def test_failed_admission_is_not_kept(ctx):
    """The admission of a new structure fails after its deep copy (forced from
    the host): that job reports the error, the structure is not kept resident,
    and the next job with the same key copies it again and gets the oracle's
    result; the other structure stays resident and is reused."""
    from paper_1906_01128_amd import dc
    structs = _structures(2, 4 << 20, seed=300)
    schema = dc.Schema(structs[0].types)
    srv = dc.Server(ctx, schema, budget_bytes=1 << 30, max_inflight=1, nstreams=2, fail_copy_at=2)
    jobs = [(0, 1, 0), (1, 2, 1), (1, 2, 2), (0, 1, 3)]
    outs, ids = [], []
    for si, key, ab in jobs:
        t = structs[si]
        n = orc.OracleCopy(t.types, t.root_type, t.roots, 64, 0).out_bytes("all")
        buf = np.zeros(max(n, 1), np.uint8)
        outs.append(buf)
        ids.append(srv.submit(t.root_type, t.roots[0], buf.ctypes.data, buf.nbytes, *AB[ab], key=key))
    ok0 = srv.wait(ids[0], timeout=120.0)
    with pytest.raises(dc.DcError) as e:
        srv.wait(ids[1], timeout=120.0)
    assert "injected" in str(e.value)
    ok2 = srv.wait(ids[2], timeout=120.0)
    ok3 = srv.wait(ids[3], timeout=120.0)
    st = srv.stats()
    srv.close()
    assert ok0.status == ok2.status == ok3.status == 0
    assert ok2.reused == 0 and ok3.reused == 1
    for k in (0, 2, 3):
        si, _, ab = jobs[k]
        assert np.array_equal(outs[k], _expected(structs[si], *AB[ab])), f"job {k}"


def test_pinned_outputs_equal_pageable_and_oracle(ctx):
    """Jobs whose output buffers are page-locked receive every leaf by a direct
    copy; the whole image (the bytes between leaves left as the caller set
    them) equals the oracle's and the pageable path's."""
    from paper_1906_01128_amd import dc
    structs = _structures(6, 8 << 20, seed=400)
    schema = dc.Schema(structs[0].types)
    jobs = [(i % 6, (i % 6) + 1 if i % 2 else 0, i % 4) for i in range(12)]
    srv = dc.Server(ctx, schema, budget_bytes=2 << 30, max_inflight=4, nstreams=2)
    pinned, ids = [], []
    for si, key, ab in jobs:
        t = structs[si]
        n = orc.OracleCopy(t.types, t.root_type, t.roots, 64, 0).out_bytes("all")
        buf = torch.full((max(n, 1),), 0, dtype=torch.uint8, pin_memory=True)
        pinned.append(buf)
        ids.append(srv.submit(t.root_type, t.roots[0], buf.data_ptr(), buf.numel(), *AB[ab], key=key))
    res = [srv.wait(i, timeout=120.0) for i in ids]
    assert all(r.status == 0 for r in res)
    pageable, _ = _run(srv, jobs, structs)
    srv.close()
    for k, (si, _, ab) in enumerate(jobs):
        want = _expected(structs[si], *AB[ab])
        got = pinned[k].numpy()
        assert np.array_equal(got[: want.nbytes], want), f"job {k}: pinned output differs from the oracle"
        assert np.array_equal(pageable[k][: want.nbytes], want), f"job {k}: pageable output differs from the oracle"
