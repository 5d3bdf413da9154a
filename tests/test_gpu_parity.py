"""GPU (HIP, gfx950) path against the CPU FP64 oracle, element by element.

Tolerances (max |gpu - oracle| / max |input|): 1e-12 in float64, 2e-5 in
float32; the oracle always runs in FP64 on the input as rounded to the GPU
dtype.  Shapes span several tiles with ragged tails, uneven dimensions,
nonuniform coordinates, partial and maximal level counts, and in-place
calls.  Every call goes through the C ABI (libmgr.so).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2007_04457_amd as mgr
from paper_2007_04457_amd import synth

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 2e-5}
DEV = "cuda:0"


def field(shape, seed, nonuniform, dtype):
    u, coords = synth.sinusoid_field(shape, seed, nonuniform=nonuniform)
    x = torch.from_numpy(u).to(dtype)
    return x, x.double().numpy(), coords


def rel_err(got, want, scale):
    return float(np.max(np.abs(got - want))) / max(scale, 1e-300)


def step_scaled_err(got, want, gd, coords, L):
    """Error of the recomposition's transpose, per class, relative to the
    size of what the class's step computes with.  R^T runs fine to coarse;
    step k reads the level-k grid G_k (the input after steps 0..k-1, which
    collects the transposed interpolation of every finer level: up to 2^d
    per level) and writes class L - k as G_k at the fine nodes minus
    E^T M P M_c^{-1} applied to the coarse nodes.  Where that difference is
    far smaller than G_k (in 1-D at 32769 nodes, class 8 is 900 times smaller
    than G_6), rounding of the step's inputs and products sets the error, so
    each class is measured against max(max|G_k|, max|class|) (class 0:
    G_L, the class itself)."""
    shape = gd.shape
    cm = oracle.class_map(shape, L)
    worst = 0.0
    for c in range(L + 1):
        m = cm == c
        scale = float(np.max(np.abs(want[m])))
        if c > 0:
            k = L - c
            Gk = oracle.recompose_adjoint(gd, coords, k)[tuple(slice(None, None, 2 ** k) for _ in shape)]
            scale = max(scale, float(np.max(np.abs(Gk))))
        worst = max(worst, float(np.max(np.abs(got[m] - want[m]))) / max(scale, 1e-300))
    return worst


CASES = [
    # shape, dtype, nonuniform, nlevels
    ((129,), torch.float64, False, -1),
    ((257,), torch.float32, True, -1),
    ((3,), torch.float64, False, 1),
    ((65, 33), torch.float64, True, -1),
    ((33, 65), torch.float32, False, 2),
    ((129, 129), torch.float32, True, -1),
    ((5, 9), torch.float64, False, 2),
    ((33, 17, 65), torch.float64, False, -1),
    ((17, 33, 9), torch.float64, True, -1),
    ((65, 65, 65), torch.float64, False, -1),
    ((33, 33, 33), torch.float32, True, -1),
    ((9, 9, 9), torch.float64, False, 3),
    ((3, 5, 9), torch.float32, False, 1),
    ((65, 9, 129), torch.float32, False, 3),
    ((17, 17, 17), torch.float64, True, 0),
    ((1025, 33), torch.float64, True, -1),
    ((33, 1025), torch.float32, True, -1),
    ((129, 65, 257), torch.float32, True, -1),
    ((257, 17, 33), torch.float64, False, -1),
    # extreme aspect ratios: one long dimension beside minimal ones
    ((3, 3, 1025), torch.float32, False, 1),
    ((1025, 3, 5), torch.float64, True, 1),
    ((5, 1025, 3), torch.float32, True, 1),
    ((2049,), torch.float32, True, -1),
    ((8193,), torch.float64, False, -1),
    # fibres longer than one workgroup stages (three-phase partitioned
    # solve): along the contiguous dimension, and along a strided one
    ((16385,), torch.float64, True, -1),
    ((32769,), torch.float32, False, -1),
    ((2049, 3, 3), torch.float32, True, 1),
]


@pytest.fixture(params=["tail", "notail"])
def tail_mode(request):
    """Runs a test with the small coarse levels in the combined single-
    workgroup launch (default) and with every level on the large-level
    kernels."""
    prev = mgr.mgr_set_tail_max_nodes(0 if request.param == "notail" else 5000)
    yield request.param
    mgr.mgr_set_tail_max_nodes(prev)


def case_id(c):
    shape, dt, nu, L = c
    return f"{'x'.join(map(str, shape))}-{str(dt).split('.')[-1]}-{'nonuni' if nu else 'uni'}-L{L}"


@pytest.mark.parametrize("case", CASES, ids=[case_id(c) for c in CASES])
def test_decompose_matches_oracle(case, tail_mode):
    shape, dt, nu, L = case
    x, xd, coords = field(shape, 100 + len(shape), nu, dt)
    want = oracle.decompose(xd, coords, L)
    y = mgr.decompose(x.to(DEV), coords, L)
    torch.cuda.synchronize()
    err = rel_err(y.double().cpu().numpy(), want, np.max(np.abs(xd)))
    assert err <= TOL[dt], err


@pytest.mark.parametrize("case", CASES, ids=[case_id(c) for c in CASES])
def test_recompose_matches_oracle(case, tail_mode):
    shape, dt, nu, L = case
    x, xd, coords = field(shape, 200 + len(shape), nu, dt)
    refac = torch.from_numpy(oracle.decompose(xd, coords, L)).to(dt)
    rd = refac.double().numpy()
    want = oracle.recompose(rd, coords, L)
    r = mgr.recompose(refac.to(DEV), coords, L)
    torch.cuda.synchronize()
    err = rel_err(r.double().cpu().numpy(), want, np.max(np.abs(rd)))
    assert err <= TOL[dt], err


@pytest.mark.parametrize("case", CASES, ids=[case_id(c) for c in CASES])
def test_adjoint_matches_oracle(case):
    shape, dt, nu, L = case
    g, gd, coords = field(shape, 300 + len(shape), nu, dt)
    want = oracle.decompose_adjoint(gd, coords, L)
    a = mgr.decompose_adjoint(g.to(DEV), coords, L)
    torch.cuda.synchronize()
    # normalised by the input's scale, max|g|, as for every other direction
    err = rel_err(a.double().cpu().numpy(), want, np.max(np.abs(gd)))
    assert err <= TOL[dt], err


@pytest.mark.parametrize("case", CASES, ids=[case_id(c) for c in CASES])
def test_recompose_adjoint_matches_oracle(case):
    shape, dt, nu, L = case
    g, gd, coords = field(shape, 400 + len(shape), nu, dt)
    want = oracle.recompose_adjoint(gd, coords, L)
    a = mgr.recompose_adjoint(g.to(DEV), coords, L)
    torch.cuda.synchronize()
    Lf = oracle.max_levels(shape) if L < 0 else L
    err = step_scaled_err(a.double().cpu().numpy(), want, gd, coords, Lf)
    assert err <= TOL[dt], err


@pytest.mark.parametrize("shape,dt", [((65, 33, 17), torch.float64), ((129, 65), torch.float32),
                                      ((257,), torch.float64)])
def test_in_place_equals_out_of_place(shape, dt, tail_mode):
    x, _, coords = field(shape, 7, True, dt)
    xg = x.to(DEV)
    for fn in (mgr.mgr_decompose, mgr.mgr_recompose, mgr.mgr_decompose_adjoint, mgr.mgr_recompose_adjoint):
        out = torch.empty_like(xg)
        fn(xg, out, coords)
        inp = xg.clone()
        fn(inp, inp, coords)
        torch.cuda.synchronize()
        assert torch.equal(out, inp), fn.__name__


@pytest.mark.parametrize("shape", [(33, 17, 65), (129, 33), (257,)])
def test_multilinear_input_exact_zero_layout(shape):
    """Layout check, bitwise: integer data on the stride-2^j grid,
    multilinearly interpolated, decompose to exact zeros exactly at the
    classes finer than the data's level, and their coarse values pass
    through the first steps unchanged."""
    rng = np.random.default_rng(1)
    L = oracle.max_levels(shape)
    for j in (1, 2):
        s = 2 ** j
        coarse = rng.integers(-8, 9, tuple((n - 1) // s + 1 for n in shape)).astype(np.float64)
        # multilinear interpolation of dyadic data is exact in float64
        u = coarse
        for d in range(len(shape)):
            idx = np.arange(shape[d]) / s
            lo = np.minimum(np.floor(idx).astype(int), u.shape[d] - 1)
            hi = np.minimum(lo + 1, u.shape[d] - 1)
            fr = idx - np.floor(idx)
            u = (np.take(u, lo, axis=d) * np.expand_dims(1 - fr, tuple(e for e in range(len(shape)) if e != d))
                 + np.take(u, hi, axis=d) * np.expand_dims(fr, tuple(e for e in range(len(shape)) if e != d)))
        cls = oracle.class_map(shape, L)
        for dt in (torch.float64, torch.float32):
            y = mgr.decompose(torch.from_numpy(u).to(dt).to(DEV), None, L).double().cpu().numpy()
            assert np.all(y[cls > L - j] == 0.0), (j, dt)
            part = mgr.decompose(torch.from_numpy(u).to(dt).to(DEV), None, j).double().cpu().numpy()
            sl = tuple(slice(None, None, s) for _ in shape)
            assert np.array_equal(part[sl], u[sl]), (j, dt)


def test_autograd_function():
    shape = (17, 9, 33)
    x, xd, coords = field(shape, 11, True, torch.float64)
    xg = x.to(DEV).requires_grad_(True)
    y = mgr.Decompose.apply(xg, coords, -1)
    w = torch.from_numpy(np.power(2.0, oracle.class_map(shape))).to(DEV)
    loss = (w * y * y).sum()
    loss.backward()
    d = oracle.decompose(xd, coords)
    want = oracle.decompose_adjoint(2.0 * np.power(2.0, oracle.class_map(shape)) * d, coords)
    err = rel_err(xg.grad.cpu().numpy(), want, np.max(np.abs(want)))
    assert err <= 1e-12, err


def test_autograd_through_recompose():
    """x = R y with R the recomposition; the gradient of sum(w * x^2) with
    respect to y is R^T (2 w x), through the recomposition's adjoint."""
    shape = (17, 9, 33)
    y0, yd, coords = field(shape, 13, True, torch.float64)
    yg = y0.to(DEV).requires_grad_(True)
    x = mgr.Recompose.apply(yg, coords, -1)
    w = torch.from_numpy(np.linspace(0.5, 2.0, int(np.prod(shape))).reshape(shape)).to(DEV)
    (w * x * x).sum().backward()
    xr = oracle.recompose(yd, coords)
    want = oracle.recompose_adjoint(2.0 * w.cpu().numpy() * xr, coords)
    err = rel_err(yg.grad.cpu().numpy(), want, np.max(np.abs(want)))
    assert err <= 1e-12, err
    # decompose then recompose is the identity, and so is its gradient
    xg = torch.from_numpy(yd).to(DEV).requires_grad_(True)
    out = mgr.Recompose.apply(mgr.Decompose.apply(xg, coords, -1), coords, -1)
    (w * out).sum().backward()
    assert float((xg.grad - w).abs().max()) <= 1e-12 * float(w.abs().max())


def test_prepare_and_repeat_calls_are_deterministic():
    shape = (65, 33, 33)
    x, _, coords = field(shape, 12, True, torch.float32)
    mgr.mgr_prepare(torch.float32, shape, coords)
    xg = x.to(DEV)
    a = mgr.decompose(xg, coords)
    b = mgr.decompose(xg, coords)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_bench_copy_and_timing():
    src = torch.arange(1 << 20, dtype=torch.float32, device=DEV)
    dst = torch.empty_like(src)
    mgr.mgr_timing_enable("bench_copy", 0)
    mgr.mgr_bench_copy(src, dst)
    ms, n = mgr.mgr_timing_read()
    mgr.mgr_timing_disable()
    assert torch.equal(src, dst)
    assert n == 1 and ms > 0.0
