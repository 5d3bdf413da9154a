"""Class-packed layout and progressive recomposition on the GPU against the
CPU oracle.

Packing is a permutation, so the GPU layout is compared bit for bit with the
oracle's (class 0 first, each class in C order of its nodes).  Progressive
recomposition is compared with the oracle's recomposition from the classes
0..l (finer classes zeroed) at the level-l nodes, at the usual tolerance
(max |gpu - oracle| / max |input|: 1e-12 float64, 2e-5 float32), from both
layouts; the class-packed call gets only the prefix it needs.
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

CASES = [
    # shape, dtype, nonuniform, nlevels
    ((129,), torch.float64, True, -1),
    ((65, 33), torch.float32, False, -1),
    ((33, 65), torch.float64, True, 3),
    ((33, 17, 65), torch.float32, True, -1),
    ((65, 65, 65), torch.float64, False, -1),
    ((17, 9, 33), torch.float64, False, 2),
    ((3, 5, 9), torch.float32, False, 1),
    ((129, 129, 129), torch.float32, True, -1),
]


def cid(c):
    return f"{'x'.join(map(str, c[0]))}-{str(c[1]).split('.')[-1]}-{'nu' if c[2] else 'u'}-L{c[3]}"


@pytest.mark.parametrize("case", CASES, ids=[cid(c) for c in CASES])
def test_pack_unpack_bitwise(case):
    shape, dt, nu, L = case
    y = torch.from_numpy(synth.sinusoid_field(shape, 70, nonuniform=nu)[0]).to(dt)
    want = oracle.pack_classes(y.double().numpy(), L)
    p = mgr.pack_classes(y.to(DEV), L)
    torch.cuda.synchronize()
    assert np.array_equal(p.double().cpu().numpy(), want)
    back = mgr.unpack_classes(p, shape, L)
    torch.cuda.synchronize()
    assert torch.equal(back.cpu(), y)


@pytest.mark.parametrize("case", CASES, ids=[cid(c) for c in CASES])
def test_recompose_level_matches_oracle(case):
    shape, dt, nu, L = case
    u, coords = synth.sinusoid_field(shape, 71, nonuniform=nu)
    yd = oracle.decompose(torch.from_numpy(u).to(dt).double().numpy(), coords, L)
    y = torch.from_numpy(yd).to(dt)
    yd = y.double().numpy()
    scale = float(np.max(np.abs(yd)))
    full = oracle.max_levels(shape) if L < 0 else L
    off = oracle.class_offsets(shape, L)
    yg = y.to(DEV)
    pg = mgr.pack_classes(yg, L)
    for lev in range(full + 1):
        want = oracle.recompose_level(yd, lev, coords, L)
        got = mgr.recompose_level(yg, lev, shape, coords, L).double().cpu().numpy()
        assert got.shape == want.shape
        assert float(np.max(np.abs(got - want))) / scale <= TOL[dt], ("in-place", lev)
        prefix = pg[: int(off[lev + 1])].clone()  # only the classes 0..lev
        gotp = mgr.recompose_level(prefix, lev, shape, coords, L, packed=True)
        torch.cuda.synchronize()
        assert np.array_equal(gotp.double().cpu().numpy(), got), ("packed", lev)


def test_full_size_pack_and_progressive_513():
    """513^3 float32 sinusoid field: the GPU class-packed layout equals the
    oracle's bit for bit, and recomposition to levels 4..8 from the packed
    prefixes matches the oracle's progressive recomposition."""
    shape = (513, 513, 513)
    print("\n[packed] 513^3 float32", flush=True)
    prev = oracle.set_threads(8)  # the oracle's output does not depend on it
    u, _ = synth.sinusoid_field(shape, 1)
    x = torch.from_numpy(u).to(torch.float32)
    del u
    yg = mgr.decompose(x.to(DEV))
    torch.cuda.synchronize()
    yd = yg.double().cpu().numpy()
    pg = mgr.pack_classes(yg)
    torch.cuda.synchronize()
    assert np.array_equal(pg.cpu().numpy(), oracle.pack_classes(yg.cpu().numpy()))
    off = oracle.class_offsets(shape)
    scale = float(np.max(np.abs(yd)))
    for lev in (4, 6, 7, 8):
        print(f"[packed] level {lev}", flush=True)
        got = mgr.recompose_level(pg[: int(off[lev + 1])].clone(), lev, shape, None, -1, packed=True)
        want = oracle.recompose_level(yd, lev)
        err = float(np.max(np.abs(got.double().cpu().numpy() - want))) / scale
        assert err <= TOL[torch.float32], (lev, err)
    oracle.set_threads(prev)
