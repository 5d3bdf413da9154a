"""Pins of the CPU oracle to things other than itself (CPU only).

Each test names the passage or the mathematics it checks.  A plausible
mistake anywhere in the oracle (a dropped term, a swapped interpolation
weight, a wrong boundary row, a transposed operand, a wrong sweep order)
fails at least one of them:
  - dense L2 projections (every output element, tiny grids),
  - exact zero coefficients for multilinear input (bitwise, dyadic data),
  - the paper's 1D quadratic example (closed form),
  - 1D closed forms of the load-vector stencil and the correction solve,
  - recompose(decompose(x)) = x and progressive recomposition,
  - scale invariance of the coordinates (bitwise),
  - the adjoint against the explicit dense transpose, a dot-product test and
    exact central finite differences of a quadratic loss.
"""
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import dense_ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_coords(rng, shape):
    out = []
    for n in shape:
        h = rng.uniform(0.5, 1.5, n - 1)
        x = np.concatenate([[0.0], np.cumsum(h)])
        out.append(x / x[-1])
    return out


TINY = [(9,), (17,), (33,), (9, 9), (17, 9), (5, 17), (5, 5, 5), (9, 5, 9), (9, 9, 9)]


@pytest.mark.parametrize("shape", TINY)
@pytest.mark.parametrize("nonuniform", [False, True])
def test_matches_dense_l2_projection(shape, nonuniform):
    """Eq. (1)-(2): coarsest = Q_0 u, class l = (I - Pi_{l-1}) Q_l u."""
    rng = np.random.default_rng(hash((shape, nonuniform)) % 2**32)
    coords = rand_coords(rng, shape) if nonuniform else None
    u = rng.standard_normal(shape)
    full = oracle.max_levels(shape)
    for L in sorted({1, full, full + 1}):
        if L < 1:
            continue
        got = oracle.decompose(u, coords, L)
        want = dense_ref.decompose_dense(u, coords, L)
        assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(u)), (shape, L)


def test_dense_reference_is_an_l2_projection():
    """Orthogonality (Sec. II-A.2): the detail Q_l u - Q_{l-1} u is
    M-orthogonal to V_{l-1}; checks the dense reference itself."""
    rng = np.random.default_rng(11)
    shape = (9, 5)
    coords = rand_coords(rng, shape)
    u = rng.standard_normal(shape)
    L = 2
    xs = [c for c in coords]
    M_L = dense_ref.kron_all([dense_ref.fe_mass_1d(x) for x in xs])
    for l in (1, 2):
        q = dense_ref.projection_values(u, coords, L, l)
        qc = dense_ref.projection_values(u, coords, L, l - 1)
        Bl = dense_ref.kron_all([dense_ref.hat_eval_1d(x, x[:: 2 ** (L - l)]) for x in xs])
        Bc = dense_ref.kron_all([dense_ref.hat_eval_1d(x, x[:: 2 ** (L - l + 1)]) for x in xs])
        detail = Bl @ q.reshape(-1) - Bc @ qc.reshape(-1)
        # orthogonal to every coarse basis function
        assert np.max(np.abs(Bc.T @ (M_L @ detail))) < 1e-13
        # and u - Q_l u orthogonal to V_l
        r = u.reshape(-1) - Bl @ q.reshape(-1)
        assert np.max(np.abs(Bl.T @ (M_L @ r))) < 1e-13


@pytest.mark.parametrize("shape", [(33,), (17, 9), (9, 17, 5), (17, 17, 17)])
def test_multilinear_input_gives_exact_zero_classes(shape):
    """Sec. II-A.1: coefficients vanish where u is already multilinear.  With
    integer coarse data on a uniform grid the arithmetic is exact, so classes
    finer than the data's level are zero bitwise and the values at the data's
    nodes pass through unchanged."""
    rng = np.random.default_rng(3)
    L = oracle.max_levels(shape)
    for j in range(1, L + 1):  # data live on the grid of stride 2^j
        s = 2 ** j
        coarse = rng.integers(-8, 9, tuple((n - 1) // s + 1 for n in shape)).astype(np.float64)
        # multilinear interpolant on the finest grid, by repeated 1D averaging
        u = coarse
        for d in range(len(shape)):
            for _ in range(j):
                m = u.shape[d]
                new_shape = list(u.shape)
                new_shape[d] = 2 * m - 1
                v = np.zeros(new_shape)
                sl_even = [slice(None)] * len(shape)
                sl_even[d] = slice(0, None, 2)
                v[tuple(sl_even)] = u
                lo = [slice(None)] * len(shape)
                hi = [slice(None)] * len(shape)
                od = [slice(None)] * len(shape)
                lo[d], hi[d], od[d] = slice(0, m - 1), slice(1, m), slice(1, None, 2)
                v[tuple(od)] = 0.5 * (u[tuple(lo)] + u[tuple(hi)])
                u = v
        out = oracle.decompose(u, None, L)
        cls = oracle.class_map(shape, L)
        assert np.all(out[cls > L - j] == 0.0), (shape, j)
        # the first L-j levels leave the stride-2^j values untouched
        part = oracle.decompose(u, None, j)
        sl = tuple(slice(None, None, s) for _ in shape)
        assert np.array_equal(part[sl], u[sl])


def test_paper_quadratic_example():
    """Sec. II-A.1, Fig. 2: y = x^2 - 5x + 6; finest coefficients = -h^2."""
    data = np.loadtxt(os.path.join(GOLDEN, "fig2_quadratic_1d.txt"))
    x, y, c = data[:, 0], data[:, 1], data[:, 2]
    out = oracle.decompose(y, [x], 3)
    odd = ~np.isnan(c)
    assert np.array_equal(out[odd], c[odd])
    # one step only: the level step of the finest grid gives the same values
    one = oracle.decompose(y, [x], 1)
    assert np.array_equal(one[odd], c[odd])


def test_load_vector_uniform_stencil():
    """Sec. III-A.2: on a uniform grid (h = 1) R M applied to a unit value at
    an odd node 2i+1 gives 3 at coarse nodes i and i+1; at an interior even
    fine node (possible only in >= 2D, so tested via the 1D operator on the
    even-node coefficient-free pattern) the merged stencil is (1/2, 3, 5, 3,
    1/2).  Here the 1D load vector of single odd spikes is checked."""
    n = 17
    for j in range(1, n, 2):
        u = np.zeros(n)
        u[j] = 1.0
        f = oracle.load_vector_level(u, 0)
        want = np.zeros((n + 1) // 2)
        i = (j - 1) // 2
        want[i] = 3.0
        want[i + 1] = 3.0
        assert np.array_equal(f, want), j


def test_load_vector_2d_even_row_stencil():
    """Along an axis, R M maps a unit value at an even interior node 2i to
    (1/2, 5, 1/2) at coarse nodes (i-1, i, i+1) (uniform h = 1); in 2D a
    value at (odd, even) therefore gives the outer product of (3, 3) and
    (1/2, 5, 1/2)."""
    shape = (9, 17)
    u = np.zeros(shape)
    u[3, 8] = 1.0
    f = oracle.load_vector_level(u, 0)
    want = np.zeros((5, 9))
    want[1:3, 3:6] = np.outer([3.0, 3.0], [0.5, 5.0, 0.5])
    assert np.array_equal(f, want)


@pytest.mark.parametrize("nonuniform", [False, True])
def test_correction_is_textbook_banded_solve(nonuniform):
    """Sec. II-A.2: z solves M_{l-1} z = f; compare with scipy's banded LU on
    the finite-element mass matrix (scaled by 6) of the coarse coordinates."""
    rng = np.random.default_rng(5)
    n = 33
    coords = rand_coords(rng, (n,)) if nonuniform else None
    x = coords[0] if nonuniform else np.arange(n, dtype=np.float64)
    for k in range(0, 4):
        xc = x[:: 2 ** (k + 1)]
        f = rng.standard_normal(len(xc))
        z = oracle.correction_level(f, (n,), k, coords)
        M = 6.0 * dense_ref.fe_mass_1d(xc)
        ab = np.zeros((3, len(xc)))
        ab[0, 1:] = np.diag(M, 1)
        ab[1] = np.diag(M)
        ab[2, :-1] = np.diag(M, -1)
        want = scipy.linalg.solve_banded((1, 1), ab, f)
        assert np.max(np.abs(z - want)) <= 1e-13 * np.max(np.abs(want))


@pytest.mark.parametrize("shape", [(65,), (33, 17), (17, 9, 33), (33, 33, 33)])
@pytest.mark.parametrize("nonuniform", [False, True])
def test_roundtrip(shape, nonuniform):
    """Sec. II-A: recomposition is the exact inverse of decomposition."""
    rng = np.random.default_rng(7)
    coords = rand_coords(rng, shape) if nonuniform else None
    u = rng.standard_normal(shape)
    for L in (1, oracle.max_levels(shape), oracle.max_levels(shape) + 1):
        d = oracle.decompose(u, coords, L)
        r = oracle.recompose(d, coords, L)
        assert np.max(np.abs(r - u)) <= 1e-13 * np.max(np.abs(u))


@pytest.mark.parametrize("shape", [(17,), (9, 17), (9, 5, 9)])
def test_progressive_recomposition(shape):
    """Sec. I and II-A: recomposing from the classes 0..l0 only returns the
    projection Q_{l0} u, interpolated to the finest nodes."""
    rng = np.random.default_rng(9)
    coords = rand_coords(rng, shape)
    u = rng.standard_normal(shape)
    L = oracle.max_levels(shape)
    d = oracle.decompose(u, coords, L)
    cls = oracle.class_map(shape, L)
    for l0 in range(0, L + 1):
        trunc = np.where(cls <= l0, d, 0.0)
        r = oracle.recompose(trunc, coords, L)
        want = dense_ref.progressive_dense(u, coords, L, l0)
        assert np.max(np.abs(r - want)) <= 1e-12 * np.max(np.abs(u)), l0


def test_scale_invariance_bitwise():
    """Only coordinate ratios enter the method: scaling all coordinates by a
    power of two, or replacing None by i * 2^-k, changes no bit."""
    rng = np.random.default_rng(13)
    shape = (17, 9, 33)
    u = rng.standard_normal(shape)
    coords = rand_coords(rng, shape)
    a = oracle.decompose(u, coords)
    b = oracle.decompose(u, [c * 8.0 for c in coords])
    assert np.array_equal(a, b)
    c = oracle.decompose(u, None)
    e = oracle.decompose(u, [np.arange(n) / (n - 1) for n in shape])
    assert np.array_equal(c, e)
    f = oracle.decompose(u, [None, np.arange(9) * 0.25, None])
    assert np.array_equal(c, f)


def test_class_map_definition():
    """Class of a node: 0 for the coarsest nodes, else L minus the smallest
    2-adic valuation of its indices (brute force)."""
    shape = (17, 9, 5)
    L = 2
    cm = oracle.class_map(shape, L)
    for idx in np.ndindex(*shape):
        v = L
        for i in idx:
            if i == 0:
                continue
            t = 0
            while i % 2 == 0:
                i //= 2
                t += 1
            v = min(v, t)
        assert cm[idx] == (0 if v >= L else L - v)


def test_adjoint_equals_dense_transpose():
    """The transposed map equals the transpose of the dense decomposition
    matrix built from the L2 projections (9x9x9 grid, 729 unit vectors)."""
    rng = np.random.default_rng(17)
    for shape, nonuni in [((9, 9, 9), False), ((9, 5, 9), True), ((17, 9), True), ((33,), True)]:
        coords = rand_coords(rng, shape) if nonuni else None
        L = oracle.max_levels(shape)
        D = dense_ref.decompose_matrix(shape, coords, L)
        g = rng.standard_normal(shape)
        got = oracle.decompose_adjoint(g, coords, L)
        want = (D.T @ g.reshape(-1)).reshape(shape)
        assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want)), shape


@pytest.mark.parametrize("shape", [(17, 17, 17), (33, 9, 17), (65, 33)])
def test_adjoint_dot_product(shape):
    """<D x, g> = <x, D^T g> for random x, g."""
    rng = np.random.default_rng(19)
    coords = rand_coords(rng, shape)
    x = rng.standard_normal(shape)
    g = rng.standard_normal(shape)
    lhs = np.sum(oracle.decompose(x, coords) * g)
    rhs = np.sum(x * oracle.decompose_adjoint(g, coords))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.sqrt(x.size))


def test_adjoint_finite_difference_17cubed():
    """Loss = sum_l 2^l ||class l||^2 is quadratic in x, so its central
    difference is exact up to rounding; compare with <grad, e> where
    grad = D^T (2 w * D x)."""
    rng = np.random.default_rng(6)
    shape = (17, 17, 17)
    x = rng.standard_normal(shape)
    L = oracle.max_levels(shape)
    w = np.power(2.0, oracle.class_map(shape, L))

    def loss(v):
        d = oracle.decompose(v, None, L)
        return np.sum(w * d * d)

    grad = oracle.decompose_adjoint(2.0 * w * oracle.decompose(x, None, L), None, L)
    for t in range(4):
        e = rng.standard_normal(shape)
        eps = 1e-3
        fd = (loss(x + eps * e) - loss(x - eps * e)) / (2 * eps)
        an = np.sum(grad * e)
        assert abs(fd - an) <= 1e-9 * abs(an), t


@pytest.mark.parametrize("shape,k", [((17,), 0), ((33,), 2), ((9, 17), 0), ((17, 9), 1), ((9, 5, 9), 0),
                                     ((17, 9, 17), 1), ((9, 9, 9), 2)])
@pytest.mark.parametrize("nonuniform", [False, True])
def test_coefficients_level_is_u_minus_interpolant(shape, k, nonuniform):
    """The coefficient stage alone (Sec. II-A.1) at level step k equals
    u - Pi u at the level grid's fine-only nodes, with Pi assembled densely
    from hat functions; every other node is unchanged."""
    rng = np.random.default_rng(hash((shape, k, nonuniform)) % 2**32)
    coords = rand_coords(rng, shape) if nonuniform else None
    u = rng.standard_normal(shape)
    got = oracle.coefficients_level(u, k, coords)
    want = dense_ref.coefficients_dense(u, coords, k)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(u)), (shape, k)
    off = np.ones(shape, dtype=bool)
    off[tuple(slice(None, None, 2 ** k) for _ in shape)] = False
    assert np.array_equal(got[off], u[off])


def test_error_codes():
    u = np.zeros((9, 9))
    with pytest.raises(oracle.OracleError, match="shape"):
        oracle.decompose(np.zeros((2, 9)))
    with pytest.raises(oracle.OracleError, match="levels"):
        oracle.decompose(np.zeros((10, 9)), None, 5)  # 10 -> 6 -> 4 -> 3 -> 2: four steps at most
    with pytest.raises(oracle.OracleError, match="levels"):
        oracle.decompose(u, None, 4)
    with pytest.raises(oracle.OracleError, match="coordinates"):
        oracle.decompose(u, [np.array([0, 1, 2, 3, 3, 5, 6, 7, 8.0]), None])
    assert oracle.max_levels((9, 9)) == 2
    assert oracle.max_levels((513, 513, 513)) == 8
    assert oracle.max_levels((1025, 1025, 257)) == 7
    assert oracle.max_levels((10, 9)) == 2 and oracle.max_levels((100, 37)) == 5 and oracle.max_levels((3, 7)) == 0
    # nlevels = 0 is the identity
    v = np.arange(81.0).reshape(9, 9)
    assert np.array_equal(oracle.decompose(v, None, 0), v)


@pytest.mark.parametrize("shape", [(65, 33, 17), (129, 65), (257,)])
def test_thread_count_does_not_change_results(shape):
    """The oracle's loops over independent fibres and nodes give bitwise the
    same output with 1 and with several threads (decompose, recompose)."""
    rng = np.random.default_rng(23)
    coords = rand_coords(rng, shape)
    u = rng.standard_normal(shape)
    prev = oracle.set_threads(1)
    try:
        d1 = oracle.decompose(u, coords)
        r1 = oracle.recompose(d1, coords)
        oracle.set_threads(4)
        d4 = oracle.decompose(u, coords)
        r4 = oracle.recompose(d1, coords)
    finally:
        oracle.set_threads(prev)
    assert np.array_equal(d1, d4)
    assert np.array_equal(r1, r4)



@pytest.mark.parametrize("shape,L", [((9,), -1), ((17, 9), -1), ((9, 5, 9), -1), ((17, 9, 17), 2), ((5, 5, 5), 0)])
def test_class_packed_layout_by_brute_force(shape, L):
    """Class-packed layout: walking the nodes in C order and appending each
    value to its class's list, then concatenating the lists class 0 first,
    gives pack_classes; segment lengths follow the nested level grids
    (class 0: the coarsest grid, class l: level grid l minus level grid
    l - 1); unpacking inverts it."""
    rng = np.random.default_rng(31)
    y = rng.standard_normal(shape)
    full = oracle.max_levels(shape) if L < 0 else L
    lists = [[] for _ in range(full + 1)]
    for idx in np.ndindex(*shape):
        v = full
        for i in idx:
            if i == 0:
                continue
            t = 0
            while i % 2 == 0:
                i //= 2
                t += 1
            v = min(v, t)
        lists[0 if v >= full else full - v].append(y[idx])
    want = np.array([x for lst in lists for x in lst])
    got = oracle.pack_classes(y, L)
    assert np.array_equal(got, want)
    sizes = [int(np.prod([(n - 1) // 2 ** (full - l) + 1 for n in shape])) for l in range(full + 1)]
    counts = [sizes[0]] + [sizes[l] - sizes[l - 1] for l in range(1, full + 1)]
    assert np.array_equal(oracle.class_offsets(shape, L), np.concatenate([[0], np.cumsum(counts)]))
    assert np.array_equal(oracle.unpack_classes(got, shape, L), y)


@pytest.mark.parametrize("shape", [(17,), (9, 17), (9, 5, 9)])
@pytest.mark.parametrize("nonuniform", [False, True])
def test_recompose_level_is_the_projection(shape, nonuniform):
    """Recomposition from the classes 0..l alone returns the nodal values of
    the L2 projection Q_l u at the level-l nodes (dense reference), for every
    l; at l = L it is the input."""
    rng = np.random.default_rng(37)
    coords = rand_coords(rng, shape) if nonuniform else None
    u = rng.standard_normal(shape)
    L = oracle.max_levels(shape)
    y = oracle.decompose(u, coords, L)
    for l in range(L + 1):
        got = oracle.recompose_level(y, l, coords, L)
        s = 2 ** (L - l)
        want = dense_ref.progressive_dense(u, coords, L, l)[tuple(slice(None, None, s) for _ in shape)]
        assert got.shape == want.shape
        assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(u)), l
    assert np.max(np.abs(oracle.recompose_level(y, L, coords, L) - u)) <= 1e-13 * np.max(np.abs(u))



def test_recompose_adjoint_equals_dense_inverse_transpose():
    """The recomposition's transpose equals (D^-1)^T, with D the dense
    decomposition matrix built from the L2 projections."""
    rng = np.random.default_rng(41)
    for shape, nonuni in [((9, 9, 9), False), ((9, 5, 9), True), ((17, 9), True), ((33,), True)]:
        coords = rand_coords(rng, shape) if nonuni else None
        L = oracle.max_levels(shape)
        D = dense_ref.decompose_matrix(shape, coords, L)
        g = rng.standard_normal(shape)
        got = oracle.recompose_adjoint(g, coords, L)
        want = (np.linalg.inv(D).T @ g.reshape(-1)).reshape(shape)
        assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want)), shape


@pytest.mark.parametrize("shape", [(17, 17, 17), (33, 9, 17), (65, 33), (129,)])
def test_recompose_adjoint_identities(shape):
    """<R y, g> = <y, R^T g> for random y, g, and R^T D^T g = (D R)^T g = g."""
    rng = np.random.default_rng(43)
    coords = rand_coords(rng, shape)
    y = rng.standard_normal(shape)
    g = rng.standard_normal(shape)
    ry = oracle.recompose(y, coords)
    lhs = np.sum(ry * g)
    rhs = np.sum(y * oracle.recompose_adjoint(g, coords))
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(ry * g))
    back = oracle.recompose_adjoint(oracle.decompose_adjoint(g, coords), coords)
    assert np.max(np.abs(back - g)) <= 1e-12 * np.max(np.abs(g))


# ---- quantisation of the classes (Sec. V, lossy compression) ----------------
# Reading: per-class uniform scalar quantiser, round half to even in the data's
# precision, codes clamped to +-(2^31 - 1).  Pins: exact multiples and ties of
# power-of-two bins (decided exactly by the definition), the half-bin bound in
# exact rational arithmetic, the class used per element (revealed through
# bins 2^-c), clamping, and the recomposed max-norm bound of the bin rule.


def _brute_class(idx, L):
    v = L
    for i in idx:
        if i == 0:
            continue
        t = 0
        while i % 2 == 0:
            i //= 2
            t += 1
        v = min(v, t)
    return 0 if v >= L else L - v


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_quantize_exact_multiples_and_ties(dt):
    shape, L = (9, 17), 3
    bins = np.array([2.0 ** -c for c in range(L + 1)]) * 0.25
    rng = np.random.default_rng(41)
    k = rng.integers(-1000, 1000, size=shape)
    cls = np.array([_brute_class(i, L) for i in np.ndindex(*shape)]).reshape(shape)
    b = bins[cls]
    q, nc = oracle.quantize((k * b).astype(dt), bins, L)
    assert nc == 0 and np.array_equal(q, k)
    # exact ties k + 1/2 go to the even neighbour
    q, _ = oracle.quantize(((k + 0.5) * b).astype(dt), bins, L)
    want = np.where(k % 2 == 0, k, k + 1)
    assert np.array_equal(q, want)
    y = oracle.dequantize(k.astype(np.int32), bins, dt, L)
    assert y.dtype == dt and np.array_equal(y, (k * b).astype(dt))


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_quantize_half_bin_bound_exact(dt):
    from fractions import Fraction
    shape, L = (17, 9), 2
    rng = np.random.default_rng(42)
    y = rng.standard_normal(shape).astype(dt)
    bins = np.array([0.013, 0.0071, 0.0029])
    q, _ = oracle.quantize(y, bins, L)
    for idx in list(np.ndindex(*shape))[::7]:
        b = Fraction(float(dt(bins[_brute_class(idx, L)])))
        err = abs(Fraction(float(y[idx])) - q[idx] * b)
        # the quotient is rounded to the data's precision before rounding to
        # an integer, which can add one unit of its last place
        slack = Fraction(float(abs(y[idx]))) * Fraction(2 * float(np.finfo(dt).eps))
        assert err <= b / 2 + slack, (idx, err, b)


@pytest.mark.parametrize("packed", [False, True])
def test_quantize_class_per_element(packed):
    """With bins 2^-c and unit values the code is 2^c: the class that each
    element was quantised with, against the brute-force class definition
    (in-place layout) or the class segments of the packed layout."""
    shape, L = (9, 5, 17), 2
    bins = np.array([2.0 ** -c for c in range(L + 1)])
    ones = np.ones(int(np.prod(shape)) if packed else shape)
    q, _ = oracle.quantize(ones, bins, L, packed=packed, shape=shape)
    got = np.log2(q.astype(np.float64)).astype(int).reshape(-1)
    if packed:
        sizes = [int(np.prod([(n - 1) // 2 ** (L - l) + 1 for n in shape])) for l in range(L + 1)]
        counts = [sizes[0]] + [sizes[l] - sizes[l - 1] for l in range(1, L + 1)]
        want = np.concatenate([np.full(c, l) for l, c in enumerate(counts)])
    else:
        want = np.array([_brute_class(i, L) for i in np.ndindex(*shape)])
    assert np.array_equal(got, want)


def test_quantize_clamps_and_counts():
    shape, L = (5, 5), 1
    y = np.zeros(shape)
    y[0, 1], y[1, 1], y[2, 3] = 1e300, -1e300, np.nan
    y[3, 0] = 2147483646.0  # representable, not clamped
    q, nc = oracle.quantize(y, np.ones(L + 1), L)
    assert nc == 3
    assert q[0, 1] == 2147483647 and q[1, 1] == -2147483647 and q[2, 3] == 0 and q[3, 0] == 2147483646
    y32 = np.zeros(shape, dtype=np.float32)
    y32[4, 4] = 2.0 ** 31  # rounds to 2^31 in float32: clamped
    q, nc = oracle.quantize(y32, np.ones(L + 1), L)
    assert nc == 1 and q[4, 4] == 2147483647


def test_one_dimensional_projection_max_norm_at_most_three():
    """The bin rule assumes |Q| <= 3 per dimension for the nodal matrix of
    the L2 projection onto the next coarser piecewise-linear space (largest
    row sum), on any mesh; checked on random meshes with spacings spread over
    five orders of magnitude."""
    rng = np.random.default_rng(43)
    worst = 0.0
    for t in range(120):
        m = 2 ** int(rng.integers(1, 6)) + 1
        h = np.exp(rng.uniform(-6, 6, m - 1)) if t % 2 else rng.uniform(0.5, 1.5, m - 1)
        x = np.concatenate([[0.0], np.cumsum(h)])
        xc = x[::2]
        P = dense_ref.hat_eval_1d(x, xc)
        Q = np.linalg.solve(dense_ref.fe_mass_1d(xc), P.T @ dense_ref.fe_mass_1d(x))
        worst = max(worst, float(np.abs(P @ Q).sum(axis=1).max()))
    assert worst <= 3.0


@pytest.mark.parametrize("shape", [(257,), (33, 65), (17, 9, 33)])
@pytest.mark.parametrize("nonuniform", [False, True])
@pytest.mark.parametrize("tol", [1e-1, 1e-3])
def test_quant_bins_bound_recomposition_error(shape, nonuniform, tol):
    """Recomposing the dequantised classes stays within tol of the field
    (max norm), for the bin widths of quant_bins."""
    rng = np.random.default_rng(44)
    coords = rand_coords(rng, shape) if nonuniform else None
    u = rng.standard_normal(shape)
    L = oracle.max_levels(shape)
    bins = oracle.quant_bins(len(shape), L, tol)
    q, nc = oracle.quantize(oracle.decompose(u, coords, L), bins, L)
    assert nc == 0
    r = oracle.recompose(oracle.dequantize(q, bins, np.float64, L), coords, L)
    assert np.max(np.abs(r - u)) <= tol


# ---- sizes other than 2^k + 1 ---------------------------------------------
# Reading (the paper's grids are all 2^k + 1 per dimension): the level grid of
# a dimension of n nodes keeps the multiples of 2^step and the last node.
# Pinned by the dense nested-grid L2 projection written from those sets alone
# (dense_ref.decompose_dense_nested), which equals dense_ref.decompose_dense
# on 2^k + 1 sizes.

ANY = [(10,), (7,), (4,), (12, 6), (9, 10), (6, 9, 5), (4, 5, 6), (5, 4, 3, 6), (3, 7, 4, 5)]


@pytest.mark.parametrize("shape", ANY)
@pytest.mark.parametrize("nonuniform", [False, True])
def test_any_size_matches_dense_nested_projection(shape, nonuniform):
    rng = np.random.default_rng(abs(hash((shape, nonuniform, "any"))) % 2**32)
    coords = rand_coords(rng, shape) if nonuniform else None
    u = rng.standard_normal(shape)
    full = oracle.max_levels(shape)
    assert full == dense_ref.full_levels_nested(shape)
    for L in sorted({1, full, full + 1}):
        if L < 1:
            continue
        got = oracle.decompose(u, coords, L)
        want = dense_ref.decompose_dense_nested(u, coords, L)
        assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(u)), (shape, L)
        assert np.array_equal(oracle.class_map(shape, L), dense_ref.class_map_nested(shape, L))
        back = oracle.recompose(got, coords, L)
        assert np.max(np.abs(back - u)) <= 1e-13 * np.max(np.abs(u))


def test_nested_dense_equals_dyadic_dense():
    rng = np.random.default_rng(51)
    for shape in [(9,), (5, 9), (5, 5, 9)]:
        coords = rand_coords(rng, shape)
        u = rng.standard_normal(shape)
        for L in (1, oracle.max_levels(shape)):
            a = dense_ref.decompose_dense(u, coords, L)
            b = dense_ref.decompose_dense_nested(u, coords, L)
            assert np.max(np.abs(a - b)) <= 1e-13


@pytest.mark.parametrize("shape", [(10,), (6, 7), (5, 6, 4)])
def test_any_size_multilinear_input_zero_classes(shape):
    """A field in V_k (the multilinear interpolant of values on the level-k
    grid) has zero classes above k and its coarsest values unchanged."""
    rng = np.random.default_rng(52)
    coords = rand_coords(rng, shape)
    L = oracle.max_levels(shape)
    for k in range(L):
        sets = [dense_ref.level_index_set(n, L, k) for n in shape]
        xs = [np.asarray(c) for c in coords]
        B = dense_ref.kron_all([dense_ref.hat_eval_1d(x, x[s]) for x, s in zip(xs, sets)])
        u = (B @ rng.standard_normal(int(np.prod([len(s) for s in sets])))).reshape(shape)
        y = oracle.decompose(u, coords, L)
        cm = oracle.class_map(shape, L)
        assert np.max(np.abs(y[cm > k])) <= 1e-12


@pytest.mark.parametrize("shape", [(6, 7), (5, 4, 3)])
def test_any_size_adjoints_equal_dense_transposes(shape):
    rng = np.random.default_rng(53)
    coords = rand_coords(rng, shape)
    L = oracle.max_levels(shape)
    N = int(np.prod(shape))
    D = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        D[:, j] = dense_ref.decompose_dense_nested(e.reshape(shape), coords, L).reshape(-1)
    Dinv_t = np.linalg.inv(D).T
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        got = oracle.decompose_adjoint(e.reshape(shape), coords, L).reshape(-1)
        assert np.max(np.abs(got - D[j, :])) <= 1e-12 * max(1.0, np.max(np.abs(D)))
        got = oracle.recompose_adjoint(e.reshape(shape), coords, L).reshape(-1)
        assert np.max(np.abs(got - Dinv_t[:, j])) <= 1e-11 * max(1.0, np.max(np.abs(Dinv_t)))


@pytest.mark.parametrize("shape", [(10,), (6, 9), (5, 6, 4)])
def test_any_size_progressive_is_the_projection(shape):
    rng = np.random.default_rng(54)
    coords = rand_coords(rng, shape)
    u = rng.standard_normal(shape)
    L = oracle.max_levels(shape)
    y = oracle.decompose(u, coords, L)
    for l in range(L + 1):
        want, _, _ = dense_ref.projection_values_nested(u, coords, L, l)
        got = oracle.recompose_level(y, l, coords, L)
        assert got.shape == want.shape
        assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(u))
