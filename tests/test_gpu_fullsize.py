"""GPU path against the CPU FP64 oracle at the full workload sizes, element
by element, in the launch configuration the benchmark times (out of place,
default level count and combined coarse-level launch):

* 513^3 uniform, float32 sinusoid-plus-noise and float64 Gaussian blobs;
* 8193^2 float64 and 1025x1025x257 float32 on nonuniform coordinates;
* the 257^3 float32 Gaussian-blob field through the adjoint, and the
  gradient of the level-weighted loss through the autograd function;
* the adjoint in float64 against central finite differences of the loss
  (17^3) and against the explicit dense transposed operator (9^3).

The oracle is single-threaded C; each full-size case costs a few seconds of
CPU time and a few GiB of host memory.
"""
import numpy as np
import pytest
import torch

import dense_ref
import oracle
import paper_2007_04457_amd as mgr
from paper_2007_04457_amd import synth

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 2e-5}
DEV = "cuda:0"


def rel_err(got, want, scale):
    return float(np.max(np.abs(got - want))) / max(scale, 1e-300)


FULL = [
    # shape, dtype, generator, seed, nonuniform
    ((513, 513, 513), torch.float32, synth.sinusoid_field, 1, False),
    ((513, 513, 513), torch.float64, synth.blob_field, 2, False),
    ((8193, 8193), torch.float64, synth.sinusoid_field, 3, True),
    ((1025, 1025, 257), torch.float32, synth.sinusoid_field, 4, True),
]


def full_id(c):
    return f"{'x'.join(map(str, c[0]))}-{str(c[1]).split('.')[-1]}-{c[2].__name__}"


@pytest.mark.parametrize("case", FULL, ids=[full_id(c) for c in FULL])
def test_full_size_decompose_recompose(case):
    shape, dt, gen, seed, nu = case
    print(f"\n[full] {full_id(case)} seed {seed}", flush=True)
    u, coords = gen(shape, seed, nonuniform=nu)
    x = torch.from_numpy(u).to(dt)
    del u
    xd = x.double().numpy()
    scale = float(np.max(np.abs(xd)))

    xg = x.to(DEV)
    yg = mgr.decompose(xg, coords)
    torch.cuda.synchronize()
    got = yg.double().cpu().numpy()
    want = oracle.decompose(xd, coords)
    err = rel_err(got, want, scale)
    assert err <= TOL[dt], ("decompose", err)
    del got

    # recompose the oracle's refactored array (rounded to the dtype)
    refac = torch.from_numpy(want).to(dt)
    del want
    rd = refac.double().numpy()
    want_r = oracle.recompose(rd, coords)
    rg = mgr.recompose(refac.to(DEV), coords)
    torch.cuda.synchronize()
    err = rel_err(rg.double().cpu().numpy(), want_r, float(np.max(np.abs(rd))))
    assert err <= TOL[dt], ("recompose", err)

    # and the GPU round trip returns the input
    rt = mgr.recompose(yg, coords)
    torch.cuda.synchronize()
    err = float((rt - xg).abs().max().item()) / scale
    assert err <= TOL[dt], ("roundtrip", err)


def test_full_size_adjoint_257_blobs():
    shape = (257, 257, 257)
    print("\n[full] adjoint 257^3 float32 blobs seed 5", flush=True)
    u, _ = synth.blob_field(shape, 5)
    g = torch.from_numpy(u).to(torch.float32)
    gd = g.double().numpy()
    want = oracle.decompose_adjoint(gd)
    a = mgr.decompose_adjoint(g.to(DEV))
    torch.cuda.synchronize()
    err = rel_err(a.double().cpu().numpy(), want, np.max(np.abs(gd)))
    assert err <= TOL[torch.float32], err


def test_full_size_loss_gradient_257_blobs():
    """Gradient of sum_l 2^l ||class l||^2 through the autograd function,
    checked as its two float32 stages, each at the float32 gate relative to
    its own input: the forward y = D x against the oracle (scale max|x|), and
    the backward D^T g, for the upstream gradient g = 2 w y that torch formed
    from the GPU's y, against the oracle adjoint of that same g (scale
    max|g|)."""
    shape = (257, 257, 257)
    print("\n[full] loss gradient 257^3 float32 blobs seed 6", flush=True)
    u, _ = synth.blob_field(shape, 6)
    x = torch.from_numpy(u).to(torch.float32)
    xd = x.double().numpy()
    w = torch.from_numpy(np.power(2.0, oracle.class_map(shape)).astype(np.float32)).to(DEV)
    xg = x.to(DEV).requires_grad_(True)
    y = mgr.Decompose.apply(xg, None, -1)
    y.retain_grad()
    loss = (w * y * y).sum()
    loss.backward()
    torch.cuda.synchronize()
    err = rel_err(y.detach().double().cpu().numpy(), oracle.decompose(xd), float(np.max(np.abs(xd))))
    assert err <= TOL[torch.float32], ("forward", err)
    g = y.grad.double().cpu().numpy()  # the upstream gradient 2 w y, as the backward received it
    want = oracle.decompose_adjoint(g)
    err = rel_err(xg.grad.double().cpu().numpy(), want, float(np.max(np.abs(g))))
    assert err <= TOL[torch.float32], ("backward", err)


def test_adjoint_finite_difference_17cubed_gpu():
    """The loss is quadratic in x, so its float64 central difference along a
    direction e equals <grad, e> up to rounding."""
    rng = np.random.default_rng(61)
    shape = (17, 17, 17)
    L = mgr.mgr_max_levels(shape)
    w = torch.from_numpy(np.power(2.0, mgr.mgr_class_map(shape, L))).to(DEV)
    x = torch.from_numpy(rng.standard_normal(shape)).to(DEV)

    def loss(v):
        d = mgr.decompose(v, None, L)
        return float((w * d * d).sum().item())

    xg = x.clone().requires_grad_(True)
    y = mgr.Decompose.apply(xg, None, L)
    (w * y * y).sum().backward()
    for t in range(6):
        e = torch.from_numpy(rng.standard_normal(shape)).to(DEV)
        eps = 1e-3
        fd = (loss(x + eps * e) - loss(x - eps * e)) / (2 * eps)
        an = float((xg.grad * e).sum().item())
        assert abs(fd - an) <= 1e-9 * abs(an), (t, fd, an)


def test_adjoint_equals_dense_transpose_9cubed_gpu():
    """D^T g on the GPU (float64) against the transpose of the explicit
    decomposition matrix assembled from the L2 projections."""
    rng = np.random.default_rng(62)
    for shape, nonuni in [((9, 9, 9), False), ((9, 9, 9), True)]:
        coords = synth.draw_coords(rng, shape) if nonuni else None
        L = mgr.mgr_max_levels(shape)
        D = dense_ref.decompose_matrix(shape, coords, L)
        g = rng.standard_normal(shape)
        got = mgr.decompose_adjoint(torch.from_numpy(g).to(DEV), coords, L).cpu().numpy()
        want = (D.T @ g.reshape(-1)).reshape(shape)
        assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want)), shape


def test_recompose_adjoint_equals_dense_inverse_transpose_9cubed_gpu():
    """R^T g on the GPU (float64) against (D^{-1})^T g with D the explicit
    decomposition matrix."""
    rng = np.random.default_rng(63)
    for shape, nonuni in [((9, 9, 9), False), ((9, 5, 9), True)]:
        coords = synth.draw_coords(rng, shape) if nonuni else None
        L = mgr.mgr_max_levels(shape)
        D = dense_ref.decompose_matrix(shape, coords, L)
        g = rng.standard_normal(shape)
        got = mgr.recompose_adjoint(torch.from_numpy(g).to(DEV), coords, L).cpu().numpy()
        want = (np.linalg.inv(D).T @ g.reshape(-1)).reshape(shape)
        assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want)), shape


def test_full_size_recompose_adjoint_257_blobs():
    shape = (257, 257, 257)
    print("\n[full] recompose adjoint 257^3 float32 blobs seed 5", flush=True)
    u, _ = synth.blob_field(shape, 5)
    g = torch.from_numpy(u).to(torch.float32)
    gd = g.double().numpy()
    want = oracle.recompose_adjoint(gd)
    a = mgr.recompose_adjoint(g.to(DEV))
    torch.cuda.synchronize()
    # per class, against the size of what the class's step computes with:
    # the classes of R^T g span 0.4 (finest) to 5.8e4 (coarsest) times
    # max|g| here, so float32 rounding of the coarsest outputs alone is
    # ~2e-3 of max|g| (see step_scaled_err)
    from test_gpu_parity import step_scaled_err
    prev = oracle.set_threads(8)  # the oracle's output does not depend on it
    err = step_scaled_err(a.double().cpu().numpy(), want, gd, None, oracle.max_levels(shape))
    oracle.set_threads(prev)
    assert err <= TOL[torch.float32], err
