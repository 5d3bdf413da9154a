"""Seeded synthetic input fields.

These stand in for the Gray-Scott simulation output used in the paper's
evaluation (Sec. IV-A), which is not available; the paper notes that the
refactoring cost does not depend on the data values.  This module holds no
arithmetic of the refactoring method: it only draws inputs, which the GPU
path and the CPU oracle then both receive.

Recipe (all draws from ``numpy.random.default_rng(seed)`` in this order):
  1. nonuniform coordinates (only when requested), axis by axis: n-1 spacings
     U(0.5, 1.5), x = [0, cumsum] / sum, last node pinned to 1;
  2. sinusoid field: 8 plane waves a_m sin(2 pi k_m . x + phi_m) with integer
     wave vector k_m uniform in [1, 6] per axis, a_m ~ U(0.1, 1),
     phi_m ~ U(0, 2 pi); then Gaussian noise N(0, 1e-3) per node (C order);
     or blob field: 16 Gaussian blobs, centre U(0, 1)^d, width U(0.02, 0.1),
     amplitude U(-1, 1).
Node positions are the coordinates in [0, 1] (uniform grids: i / (n - 1)).
Values are produced in float64; callers round to float32 where needed.
"""
import numpy as np


def nonuniform_axis(rng, n):
    h = rng.uniform(0.5, 1.5, n - 1)
    x = np.concatenate([[0.0], np.cumsum(h)])
    x = x / x[-1]
    x[-1] = 1.0
    return x


def draw_coords(rng, shape):
    return [nonuniform_axis(rng, n) for n in shape]


def _positions(shape, coords):
    if coords is None:
        return [np.arange(n, dtype=np.float64) / (n - 1) for n in shape]
    return [np.asarray(c, dtype=np.float64) for c in coords]


def _add_plane_wave(out, xs, amp, kvec, phase):
    """out += amp * sin(2 pi k.x + phase), evaluated as
    sin(A + B) = sin A cos B + cos A sin B with B the last-axis term so the
    full-size work is two multiply-adds per node."""
    nd = len(xs)
    lead = np.full(tuple(len(x) for x in xs[:-1]), phase, dtype=np.float64)
    for d in range(nd - 1):
        sh = [1] * (nd - 1)
        sh[d] = len(xs[d])
        lead = lead + (2.0 * np.pi * kvec[d] * xs[d]).reshape(sh)
    b = 2.0 * np.pi * kvec[-1] * xs[-1]
    sa, ca = np.sin(lead)[..., None], np.cos(lead)[..., None]
    sb, cb = amp * np.sin(b), amp * np.cos(b)
    if out.ndim > 1:
        # slab by slab along axis 0 to bound temporaries
        for i in range(out.shape[0]):
            out[i] += sa[i] * cb + ca[i] * sb
    else:
        out += sa[..., 0] * cb + ca[..., 0] * sb


def sinusoid_field(shape, seed, nonuniform=False):
    """Returns (field float64, coords or None)."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(n) for n in shape)
    coords = draw_coords(rng, shape) if nonuniform else None
    xs = _positions(shape, coords)
    nd = len(shape)
    waves = []
    for _ in range(8):
        k = rng.integers(1, 7, nd)
        a = rng.uniform(0.1, 1.0)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        waves.append((a, k, phi))
    out = np.zeros(shape, dtype=np.float64)
    for a, k, phi in waves:
        _add_plane_wave(out, xs, a, k, phi)
    out += rng.normal(0.0, 1e-3, shape)
    return out, coords


def blob_field(shape, seed, nonuniform=False):
    """Returns (field float64, coords or None): 16 separable Gaussian blobs."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(n) for n in shape)
    coords = draw_coords(rng, shape) if nonuniform else None
    xs = _positions(shape, coords)
    nd = len(shape)
    out = np.zeros(shape, dtype=np.float64)
    for _ in range(16):
        c = rng.uniform(0.0, 1.0, nd)
        sigma = rng.uniform(0.02, 0.1)
        amp = rng.uniform(-1.0, 1.0)
        factors = [np.exp(-((xs[d] - c[d]) ** 2) / (2.0 * sigma * sigma)) for d in range(nd)]
        lead = np.full(tuple(shape[:-1]), amp, dtype=np.float64)
        for d in range(nd - 1):
            sh = [1] * (nd - 1)
            sh[d] = shape[d]
            lead = lead * factors[d].reshape(sh)
        if nd > 1:
            for i in range(shape[0]):
                out[i] += lead[i][..., None] * factors[-1]
        else:
            out += amp * factors[-1]
    return out, coords


def batched_shapes(nfields=96, n3d=80, seed_base=1000):
    """Per-field (shape, seed) for the batched workload: fields i < n3d are 3D
    with per-axis sizes 2^k+1, k uniform in [5, 8]; the rest are 2D with
    k uniform in [9, 12].  The exponents are the first draws of the field's
    own generator (seed seed_base + i)."""
    out = []
    for i in range(nfields):
        seed = seed_base + i
        rng = np.random.default_rng(seed)
        if i < n3d:
            ks = rng.integers(5, 9, 3)
        else:
            ks = rng.integers(9, 13, 2)
        out.append((tuple(int(2 ** k + 1) for k in ks), seed))
    return out


def batched_field(i, nfields=96, n3d=80, seed_base=1000):
    """Field i of the batched workload: sinusoid-plus-noise on its own shape.
    The generator state after the shape draw continues into the field draw."""
    seed = seed_base + i
    rng = np.random.default_rng(seed)
    if i < n3d:
        ks = rng.integers(5, 9, 3)
    else:
        ks = rng.integers(9, 13, 2)
    shape = tuple(int(2 ** k + 1) for k in ks)
    # derive the field seed from the same stream so one seed fixes both
    field_seed = int(rng.integers(0, 2 ** 63 - 1))
    f, _ = sinusoid_field(shape, field_seed)
    return f
