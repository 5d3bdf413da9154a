"""Batched decomposition (one launch per wave of work items plus one launch
for the small coarse levels) against per-field decompositions on the GPU and
against the CPU oracle.

The batch runs the same device code as the per-field path, with the same
arithmetic in the same order, so its results are compared bit for bit; a
few fields are also checked against the FP64 oracle at the usual tolerance
(max |gpu - oracle| / max |x|: 1e-12 in float64, 2e-5 in float32).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2007_04457_amd as mgr
from paper_2007_04457_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {torch.float64: 1e-12, torch.float32: 2e-5}

MIXED = [
    # shape, nonuniform
    ((33, 17, 65), False),
    ((65, 65, 65), True),
    ((129, 129), False),
    ((17, 9, 33), True),
    ((257,), False),
    ((9, 9, 9), False),
    ((513, 257), True),
    ((5, 5, 9), False),
    ((129, 33, 65), False),
    ((1025, 9), True),
]


def make_fields(cases, dtype, seed0):
    xs, coords = [], []
    for i, (shape, nu) in enumerate(cases):
        u, c = synth.sinusoid_field(shape, seed0 + i, nonuniform=nu)
        xs.append(torch.from_numpy(u).to(dtype).to(DEV))
        coords.append(c)
    return xs, coords


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_batch_equals_per_field(dtype):
    xs, coords = make_fields(MIXED, dtype, 500)
    plan = mgr.BatchPlan([x.shape for x in xs], dtype, coords)
    ys = plan.decompose(xs)
    torch.cuda.synchronize()
    for i, (x, c) in enumerate(zip(xs, coords)):
        want = mgr.decompose(x, c)
        torch.cuda.synchronize()
        assert torch.equal(ys[i], want), (i, MIXED[i])
    # and against the oracle on a few fields
    for i in (1, 3, 6):
        xd = xs[i].double().cpu().numpy()
        ref = oracle.decompose(xd, coords[i])
        err = float(np.max(np.abs(ys[i].double().cpu().numpy() - ref))) / float(np.max(np.abs(xd)))
        assert err <= TOL[dtype], (i, err)
    plan.close()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_batch_long_contiguous_fibres(dtype):
    """Fibres along the contiguous dimension longer than a batch work item
    stages (coarse rows of 4097) go through the three-phase partitioned
    solve as separate waves of items; the per-field path stages them whole,
    so the two agree to rounding and both match the oracle."""
    cases = [((8193,), False), ((9, 8193), True), ((17, 9, 33), False)]
    print(f"\n[batch] long fibres {dtype}", flush=True)
    xs, coords = make_fields(cases, dtype, 900)
    plan = mgr.BatchPlan([x.shape for x in xs], dtype, coords)
    ys = plan.decompose(xs)
    torch.cuda.synchronize()
    for i, (x, c) in enumerate(zip(xs, coords)):
        xd = x.double().cpu().numpy()
        scale = float(np.max(np.abs(xd)))
        ref = oracle.decompose(xd, c)
        got = ys[i].double().cpu().numpy()
        assert float(np.max(np.abs(got - ref))) / scale <= TOL[dtype], (i, cases[i])
        per_field = mgr.decompose(x, c).double().cpu().numpy()
        assert float(np.max(np.abs(got - per_field))) / scale <= TOL[dtype], (i, cases[i])
    plan.close()


def test_batch_repeated_calls_and_levels():
    """Second call with other inputs and partial level counts; every counter
    and the queue start from zero again."""
    cases = [((65, 33, 17), False), ((129, 65), True), ((33, 33, 33), False)]
    nl = [2, 3, 1]
    xs, coords = make_fields(cases, torch.float64, 600)
    plan = mgr.BatchPlan([x.shape for x in xs], torch.float64, coords, nl)
    for rep in range(2):
        if rep:
            xs = [torch.randn_like(x) for x in xs]
        ys = plan.decompose(xs)
        torch.cuda.synchronize()
        for i, x in enumerate(xs):
            assert torch.equal(ys[i], mgr.decompose(x, coords[i], nl[i])), (rep, i)
    plan.close()


def test_batch_config_and_autotune():
    xs, coords = make_fields(MIXED[:6], torch.float32, 700)
    plan = mgr.BatchPlan([x.shape for x in xs], torch.float32, coords)
    want = [mgr.decompose(x, c) for x, c in zip(xs, coords)]
    for chunk in (2, 5, 128):
        plan.set_config(chunk)
        assert plan.config()[0] == chunk
        ys = plan.decompose(xs)
        torch.cuda.synchronize()
        for i in range(len(xs)):
            assert torch.equal(ys[i], want[i]), (chunk, i)
    dsts = [torch.empty_like(x) for x in xs]
    chunk, launches, items = plan.autotune(xs, dsts, top_k=2)
    assert chunk in (2, 4, 8, 16, 32, 64, 128) and launches > 1 and items > 0
    # the model constants were fitted to timed probe runs of both launch forms
    form, model = plan.tuning()
    assert form in (0, 1) and plan.tile() in (False, True)
    for m in (model["waves"], model["persistent"]):
        assert len(m) == 4 and all(v >= 0.0 for v in m) and any(v != 0.0 for v in m)
    ys = plan.decompose(xs)
    plan.check()
    for i in range(len(xs)):
        assert torch.equal(ys[i], want[i]), ("tuned", i)
    with pytest.raises(mgr.MgrError):
        plan.set_config(1 << 30)
    plan.close()


def test_batch_rejects_in_place_and_bad_shapes():
    x = torch.zeros(33, 33, device=DEV)
    plan = mgr.BatchPlan([x.shape], torch.float32)
    with pytest.raises(mgr.MgrError):
        mgr._lib.check(mgr._lib.load().mgr_batch_decompose(plan._h, plan._ptrs([x]), plan._ptrs([x]), None))
    plan.close()
    with pytest.raises(mgr.MgrError):
        mgr.BatchPlan([(33, 34)], torch.float32)


def test_batch_graph_replay():
    """The batch captured into a HIP graph: every replay, with eager calls of
    the same plan on other tensors and synchronisation between replays,
    writes the captured call's outputs from the captured call's inputs, and
    the eager calls' outputs stay correct."""
    xs, coords = make_fields(MIXED[:5], torch.float32, 800)
    others, _ = make_fields(MIXED[:5], torch.float32, 850)
    plan = mgr.BatchPlan([x.shape for x in xs], torch.float32, coords)
    dsts = [torch.empty_like(x) for x in xs]
    plan.decompose(xs, dsts)  # warm-up outside the capture
    torch.cuda.synchronize()
    want = [mgr.decompose(x, c) for x, c in zip(xs, coords)]
    want_o = [mgr.decompose(x, c) for x, c in zip(others, coords)]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for d in dsts:
            d.zero_()
        with torch.cuda.graph(g, stream=s):
            plan.decompose(xs, dsts)
    torch.cuda.synchronize()
    for rep in range(3):
        for d in dsts:
            d.fill_(float(rep + 7))
        # an eager call of the same plan with other tensors before the replay
        odst = [torch.full_like(x, -1.0) for x in others]
        plan.decompose(others, odst)
        torch.cuda.synchronize()
        for i in range(len(xs)):
            assert torch.equal(odst[i], want_o[i]), ("eager", rep, i)
            assert torch.equal(dsts[i], torch.full_like(dsts[i], float(rep + 7))), ("untouched", rep, i)
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(xs)):
            assert torch.equal(dsts[i], want[i]), (rep, i)
            assert torch.equal(odst[i], want_o[i]), ("eager after replay", rep, i)
        _ = [mgr.decompose(x, c) for x, c in zip(xs, coords)]  # per-field work between replays
    del g
    plan.close()


def test_batch_plan_survives_finalize():
    """A batch plan owns its tables: mgr_finalize (which frees the per-field
    cache) leaves it working, with the same results as before."""
    xs, coords = make_fields(MIXED[:4], torch.float64, 870)
    plan = mgr.BatchPlan([x.shape for x in xs], torch.float64, coords)
    before = plan.decompose(xs)
    torch.cuda.synchronize()
    mgr.mgr_finalize()
    after = plan.decompose(xs)
    plan.set_config(4)
    again = plan.decompose(xs)
    torch.cuda.synchronize()
    for i in range(len(xs)):
        assert torch.equal(before[i], after[i]), i
        assert torch.equal(before[i], again[i]), i
        assert torch.equal(before[i], mgr.decompose(xs[i], coords[i])), i
    plan.close()


def test_batch_full_workload_96_fields():
    """The 96-field float32 workload (80 3-D fields of 2^k+1 per axis, k in
    [5, 8], and 16 2-D fields, k in [9, 12]) against per-field calls."""
    shapes = [s for s, _ in synth.batched_shapes()]
    print(f"\n[batch] {len(shapes)} fields", flush=True)
    xs = [torch.from_numpy(synth.batched_field(i)).to(torch.float32).to(DEV) for i in range(len(shapes))]
    plan = mgr.BatchPlan(shapes, torch.float32)
    ys = plan.decompose(xs)
    torch.cuda.synchronize()
    for i, x in enumerate(xs):
        assert torch.equal(ys[i], mgr.decompose(x)), (i, shapes[i])
    # a sample against the FP64 oracle: the largest 2-D and 3-D fields, the
    # smallest field, and a few more picked by a fixed draw
    sizes = [int(np.prod(s)) for s in shapes]
    big2 = max(range(80, len(shapes)), key=lambda i: sizes[i])
    big3 = max(range(80), key=lambda i: sizes[i])
    small = min(range(len(shapes)), key=lambda i: sizes[i])
    extra = np.random.default_rng(96).choice(len(shapes), 3, replace=False)
    for i in sorted({big2, big3, small, *[int(e) for e in extra]}):
        print(f"[batch] field {i} {shapes[i]} vs oracle", flush=True)
        xd = xs[i].double().cpu().numpy()
        ref = oracle.decompose(xd)
        err = float(np.max(np.abs(ys[i].double().cpu().numpy() - ref))) / float(np.max(np.abs(xd)))
        assert err <= TOL[torch.float32], (i, shapes[i], err)
    plan.close()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_batch_tile_geometry(dtype):
    """Both tile geometries of the 3-D streaming items (a tuned parameter)
    give the per-field results bit for bit, in both launch forms; the
    setting is kept across set_config and rejected outside 0/1."""
    xs, coords = make_fields(MIXED, dtype, 540)
    plan = mgr.BatchPlan([x.shape for x in xs], dtype, coords)
    assert plan.tile() == (dtype == torch.float64)
    want = [mgr.decompose(x, c) for x, c in zip(xs, coords)]
    for wide in (True, False):
        plan.set_tile(wide)
        assert plan.tile() == wide
        for persistent in (False, True):
            plan.set_mode(persistent)
            for chunk in (4, 32):
                print(f"\n[batch-tile] {dtype} wide {wide} persistent {persistent} chunk {chunk}", flush=True)
                plan.set_config(chunk)
                assert plan.tile() == wide
                ys = plan.decompose(xs)
                plan.check()
                for i in range(len(xs)):
                    assert torch.equal(ys[i], want[i]), (wide, persistent, chunk, i, MIXED[i])
    with pytest.raises(mgr.MgrError):
        mgr._lib.check(mgr._lib.load().mgr_batch_set_tile(plan._h, 2))
    assert plan.tile() is False  # unchanged by the rejected call
    plan.close()


# ---- persistent form: one launch, items taken from per-XCD queues ----------
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_batch_persistent_equals_per_field(dtype):
    """The persistent launch runs the same item functions as the wave
    launches, so its results are those of the per-field path bit for bit, for
    several chunk lengths (item counts)."""
    xs, coords = make_fields(MIXED, dtype, 520)
    plan = mgr.BatchPlan([x.shape for x in xs], dtype, coords)
    plan.set_mode(True)
    want = [mgr.decompose(x, c) for x, c in zip(xs, coords)]
    for chunk in (8, 32, 2):
        print(f"\n[batch-queue] {dtype} chunk {chunk}", flush=True)
        plan.set_config(chunk)
        ys = plan.decompose(xs)
        plan.check()
        for i in range(len(xs)):
            assert torch.equal(ys[i], want[i]), (chunk, i, MIXED[i])
    plan.close()


def test_batch_persistent_full_workload_and_graph():
    """The 96-field workload through the persistent launch, eagerly and as
    replays of a captured graph (with eager calls of the plan on other
    tensors between the replays), against the wave launches."""
    shapes = [s for s, _ in synth.batched_shapes()]
    print(f"\n[batch-queue] {len(shapes)} fields", flush=True)
    xs = [torch.from_numpy(synth.batched_field(i)).to(torch.float32).to(DEV) for i in range(len(shapes))]
    plan = mgr.BatchPlan(shapes, torch.float32)
    want = plan.decompose(xs)
    plan.set_mode(True)
    got = plan.decompose(xs)
    plan.check()
    for i in range(len(xs)):
        assert torch.equal(got[i], want[i]), (i, shapes[i])
    others = [torch.flip(x, dims=[0]).contiguous() for x in xs[:len(xs)]]
    want_o = [mgr.decompose(x) for x in others]
    dsts = [torch.empty_like(x) for x in xs]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.decompose(xs, dsts)
    torch.cuda.synchronize()
    for rep in range(3):
        for d in dsts:
            d.fill_(float(rep))
        odst = plan.decompose(others)
        plan.check()
        g.replay()
        plan.check()
        for i in range(len(xs)):
            assert torch.equal(dsts[i], want[i]), (rep, i)
            assert torch.equal(odst[i], want_o[i]), ("eager", rep, i)
    del g
    plan.close()


def test_batch_persistent_timeout_is_reported_and_recovers():
    """Every dependency wait of the persistent launch is bounded: with a
    bound of one poll the waits run out, the launch aborts and ends, and
    mgr_batch_check reports it; with the default bound the next call is
    correct again (the queue words are reset per call)."""
    xs, coords = make_fields(MIXED[:6], torch.float32, 540)
    plan = mgr.BatchPlan([x.shape for x in xs], torch.float32, coords)
    plan.set_mode(True, poll_limit=1)
    plan.decompose(xs)
    with pytest.raises(mgr.MgrError) as e:
        plan.check()
    assert "timed out" in str(e.value)
    plan.set_mode(True)
    ys = plan.decompose(xs)
    plan.check()
    for i, (x, c) in enumerate(zip(xs, coords)):
        assert torch.equal(ys[i], mgr.decompose(x, c)), i
    # an aborted run, then new tables (set_config reallocates them, possibly
    # on the memory that held the aborted run's queue words) and wave
    # launches only: the check reports no stale abort
    plan.set_mode(True, poll_limit=1)
    plan.decompose(xs)
    with pytest.raises(mgr.MgrError):
        plan.check()
    plan.set_mode(False)
    for chunk in (4, 16, 64):
        plan.set_config(chunk)
        ys = plan.decompose(xs)
        plan.check()
    for i, (x, c) in enumerate(zip(xs, coords)):
        assert torch.equal(ys[i], mgr.decompose(x, c)), ("waves after abort", i)
    plan.close()
