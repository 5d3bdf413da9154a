"""Dense linear-algebra reference for the multilevel decomposition.

This is an independent formulation of what the decomposition computes, used
to pin the CPU oracle on tiny grids.  It never forms stencils, never runs a
level recursion and never calls the oracle:

* The data define the piecewise-multilinear function u in V_L (Sec. II-A).
* Q_l u, the L2 projection onto V_l (Table I), has nodal values q_l solving
  M_l q_l = B_l^T M_L u, where M_l is the finite-element mass matrix of the
  level-l grid, assembled element by element, and B_l evaluates level-l hat
  functions at the finest nodes (np.interp of unit vectors).
* By Eq. (1) the refactored representation holds Q_0 u at the coarsest nodes
  and, for l = 1..L, the detail (I - Pi_{l-1}) Q_l u at the nodes
  N_l \\ N_{l-1}, where Pi_{l-1} is the interpolant from the level-(l-1) nodes.

Everything is assembled densely with Kronecker products, so keep the grids
tiny (a few thousand nodes at most).
"""
import numpy as np


def axis_coords(n, coords_d):
    if coords_d is None:
        return np.arange(n, dtype=np.float64)
    return np.asarray(coords_d, dtype=np.float64)


def fe_mass_1d(x):
    """Linear finite-element mass matrix int(phi_i phi_j) on nodes x."""
    n = len(x)
    M = np.zeros((n, n))
    for e in range(n - 1):
        h = x[e + 1] - x[e]
        M[e:e + 2, e:e + 2] += h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
    return M


def hat_eval_1d(x_at, x_nodes):
    """Matrix whose column j is the hat function of x_nodes[j] sampled at x_at."""
    eye = np.eye(len(x_nodes))
    return np.stack([np.interp(x_at, x_nodes, eye[:, j]) for j in range(len(x_nodes))], axis=1)


def kron_all(mats):
    out = np.ones((1, 1))
    for m in mats:
        out = np.kron(out, m)
    return out


def full_levels(shape):
    return min(int(round(np.log2(n - 1))) for n in shape) - 1


def level_coords(shape, coords, stride):
    xs = [axis_coords(n, None if coords is None else coords[d]) for d, n in enumerate(shape)]
    return [x[::stride] for x in xs], xs


def projection_values(u, coords, L, l):
    """Nodal values (on the level-l grid) of Q_l u, paper level l (L finest)."""
    shape = u.shape
    stride = 2 ** (L - l)
    xl, xs = level_coords(shape, coords, stride)
    M_L = kron_all([fe_mass_1d(x) for x in xs])
    B = kron_all([hat_eval_1d(x, y) for x, y in zip(xs, xl)])
    M_l = kron_all([fe_mass_1d(y) for y in xl])
    q = np.linalg.solve(M_l, B.T @ (M_L @ u.reshape(-1)))
    return q.reshape(tuple(len(y) for y in xl))


def decompose_dense(u, coords=None, L=None):
    """Refactored representation by Eq. (1) and the L2 projections."""
    u = np.asarray(u, dtype=np.float64)
    shape = u.shape
    if L is None or L < 0:
        L = full_levels(shape)
    out = np.zeros(shape)
    # coarsest values: Q_0 u at the level-0 nodes
    s0 = 2 ** L
    out[tuple(slice(None, None, s0) for _ in shape)] = projection_values(u, coords, L, 0)
    for l in range(1, L + 1):
        stride = 2 ** (L - l)
        q = projection_values(u, coords, L, l)
        xl, _ = level_coords(shape, coords, stride)
        xc = [y[::2] for y in xl]
        interp = kron_all([hat_eval_1d(y, yc) for y, yc in zip(xl, xc)])
        qc = q[tuple(slice(None, None, 2) for _ in shape)]
        detail = q - (interp @ qc.reshape(-1)).reshape(q.shape)
        view = out[tuple(slice(None, None, stride) for _ in shape)]
        fine = np.zeros(q.shape, dtype=bool)
        grids = np.meshgrid(*[np.arange(m) for m in q.shape], indexing="ij")
        for g in grids:
            fine |= (g % 2) == 1
        view[fine] = detail[fine]
    return out


def decompose_matrix(shape, coords=None, L=None):
    """The decomposition as an explicit N x N matrix (columns = unit inputs)."""
    N = int(np.prod(shape))
    D = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        D[:, j] = decompose_dense(e.reshape(shape), coords, L).reshape(-1)
    return D


def progressive_dense(u, coords, L, l0):
    """Q_{l0} u evaluated at the finest nodes: what recomposition from the
    classes 0..l0 alone must return (finer classes treated as zero)."""
    u = np.asarray(u, dtype=np.float64)
    shape = u.shape
    q = projection_values(u, coords, L, l0)
    xl, xs = level_coords(shape, coords, 2 ** (L - l0))
    B = kron_all([hat_eval_1d(x, y) for x, y in zip(xs, xl)])
    return (B @ q.reshape(-1)).reshape(shape)


def coefficients_dense(u, coords, k):
    """Coefficient stage of level step k (stride 2^k) alone, Sec. II-A.1:
    on the level grid, every node that is not a coarse node (some level index
    odd) becomes u - Pi u, with Pi the multilinear interpolant of the coarse
    nodes' values (the Kronecker product of 1-D hat-function evaluations);
    coarse nodes and nodes off the level grid keep their values."""
    u = np.asarray(u, dtype=np.float64)
    shape = u.shape
    out = u.copy()
    s = 2 ** k
    xl, _ = level_coords(shape, coords, s)
    xc = [y[::2] for y in xl]
    sl = tuple(slice(None, None, s) for _ in shape)
    v = u[sl]
    interp = kron_all([hat_eval_1d(y, yc) for y, yc in zip(xl, xc)])
    pi = (interp @ v[tuple(slice(None, None, 2) for _ in shape)].reshape(-1)).reshape(v.shape)
    fine = np.zeros(v.shape, dtype=bool)
    for g in np.meshgrid(*[np.arange(m) for m in v.shape], indexing="ij"):
        fine |= (g % 2) == 1
    view = out[sl]
    view[fine] = (v - pi)[fine]
    return out


# ---- any sizes ---------------------------------------------------------------
# The same definitions on nested grids of any size n >= 3 per dimension: the
# level grid l (paper numbering, L finest) along a dimension of n nodes is
# the set of indices that are multiples of 2^(L - l), together with the last
# index n - 1 (so both boundary nodes are on every level).  For n = 2^K + 1
# this is the usual stride-2^(L - l) grid.  Written from the sets alone.


def level_index_set(n, L, l):
    s = 2 ** (L - l)
    return sorted(set(range(0, n, s)) | {n - 1})


def full_levels_nested(shape):
    """Level steps until the shortest level grid has 3 nodes."""
    def steps(n):
        k = 0
        while len(level_index_set(n, k, 0)) > 3:
            k += 1
        return k
    return min(steps(n) for n in shape)


def projection_values_nested(u, coords, L, l):
    shape = u.shape
    xs = [axis_coords(n, None if coords is None else coords[d]) for d, n in enumerate(shape)]
    sets = [level_index_set(n, L, l) for n in shape]
    xl = [x[idx] for x, idx in zip(xs, sets)]
    M_L = kron_all([fe_mass_1d(x) for x in xs])
    B = kron_all([hat_eval_1d(x, y) for x, y in zip(xs, xl)])
    M_l = kron_all([fe_mass_1d(y) for y in xl])
    q = np.linalg.solve(M_l, B.T @ (M_L @ u.reshape(-1)))
    return q.reshape(tuple(len(y) for y in xl)), sets, xl


def decompose_dense_nested(u, coords=None, L=None):
    """Eq. (1) on the nested grids above: Q_0 u at the coarsest nodes, and
    (I - Pi_{l-1}) Q_l u at the nodes of level l that are not on level l - 1."""
    u = np.asarray(u, dtype=np.float64)
    shape = u.shape
    if L is None or L < 0:
        L = full_levels_nested(shape)
    out = np.zeros(shape)
    q0, sets0, _ = projection_values_nested(u, coords, L, 0)
    out[np.ix_(*sets0)] = q0
    for l in range(1, L + 1):
        q, sets, xl = projection_values_nested(u, coords, L, l)
        csets = [level_index_set(n, L, l - 1) for n in shape]
        # positions of the coarse nodes inside the level-l grid
        cpos = [[s.index(i) for i in c] for s, c in zip(sets, csets)]
        xc = [y[p] for y, p in zip(xl, cpos)]
        interp = kron_all([hat_eval_1d(y, yc) for y, yc in zip(xl, xc)])
        qc = q[np.ix_(*cpos)]
        detail = q - (interp @ qc.reshape(-1)).reshape(q.shape)
        fine = np.zeros(q.shape, dtype=bool)
        grids = np.meshgrid(*[np.array([i not in c for i in s]) for s, c in zip(sets, csets)], indexing="ij")
        for g in grids:
            fine |= g
        view = out[np.ix_(*sets)]
        view[fine] = detail[fine]
        out[np.ix_(*sets)] = view
    return out


def class_map_nested(shape, L):
    """Class of every node: 0 on the coarsest grid, else the first level l
    whose grid contains it."""
    out = np.zeros(shape, dtype=np.uint8)
    member = [[set(level_index_set(n, L, l)) for l in range(L + 1)] for n in shape]
    for idx in np.ndindex(*shape):
        c = next(l for l in range(L + 1) if all(i in member[d][l] for d, i in enumerate(idx)))
        out[idx] = c
    return out
