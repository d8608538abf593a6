"""Pins for the oracle's metrics and ghost nodes (CPU only).

Each check is against something other than the oracle's own formula: closed
forms on unit and affine grids, Gauss-Legendre quadrature of the trilinear
map's Jacobian and of the bilinear face's area element, the closed-surface
identity, and exact lattice coordinates for extrapolated / periodic ghosts.
"""
import numpy as np
import pytest

from oracle import geometry
from paper_1710_09995_amd import cases

G = 2


def _case_from_nodes(X, periodic=None, bc_kind=cases.EXTRAP):
    ni, nj, nk = X.shape[3] - 1, X.shape[2] - 1, X.shape[1] - 1
    dims = (ni, nj, nk)
    conns = []
    if periodic is not None:
        conns = cases.periodic_self_conns(0, dims, periodic)
        bcs = []
    else:
        bcs = [cases.full_bc(0, dims, f, bc_kind) for f in range(6)]
    return cases.Case("t", cases.Params(), [dims], [X], conns, bcs,
                      [np.ones((5, nk, nj, ni))])


def _affine_nodes(dims, E, origin):
    ni, nj, nk = dims
    K, J, I = np.meshgrid(np.arange(nk + 1), np.arange(nj + 1), np.arange(ni + 1), indexing="ij")
    return (origin[:, None, None, None] + E[:, 0, None, None, None] * I
            + E[:, 1, None, None, None] * J + E[:, 2, None, None, None] * K)


def test_unit_cube_metrics():
    X = cases.cartesian_nodes((4, 3, 5))
    _, S, V = geometry.build_metrics(_case_from_nodes(X), G)
    S, V = S[0], V[0]
    for d in range(3):
        e = np.zeros(3)
        e[d] = 1.0
        assert np.array_equal(S[d][:, G:-G, G:-G, G:-G], np.broadcast_to(e[:, None, None, None],
                                                                         S[d][:, G:-G, G:-G, G:-G].shape))
    assert np.array_equal(V, np.ones_like(V))   # ghosts too: extrapolated lattice is exact


def test_affine_metrics_closed_form():
    rng = np.random.default_rng(3)
    E = np.eye(3) * 0.7 + 0.2 * rng.uniform(-1, 1, (3, 3))   # columns = edge vectors e_i, e_j, e_k
    dims = (5, 4, 3)
    X = _affine_nodes(dims, E, np.array([0.3, -0.2, 1.1]))
    _, S, V = geometry.build_metrics(_case_from_nodes(X), G)
    S, V = S[0], V[0]
    e = [E[:, 0], E[:, 1], E[:, 2]]
    det = float(np.dot(e[0], np.cross(e[1], e[2])))
    assert det > 0
    for d, (a, b) in {0: (1, 2), 1: (2, 0), 2: (0, 1)}.items():
        want = np.cross(e[a], e[b])
        got = S[d].reshape(3, -1)
        assert np.max(np.abs(got - want[:, None])) < 1e-14
    assert np.max(np.abs(V - det)) < 1e-14


def _trilinear_volume_gauss(P):
    """Volume of the hexahedron with corner nodes P[a,b,c] (a=i,b=j,c=k offsets) by 2-point
    Gauss-Legendre quadrature of det(J); exact since det J is quadratic per variable."""
    gp = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    vol = 0.0
    for s in gp:
        for t in gp:
            for u in gp:
                ws = np.array([1 - s, s])
                wt = np.array([1 - t, t])
                wu = np.array([1 - u, u])
                ds = np.array([-1.0, 1.0])
                J = np.zeros((3, 3))
                for a in range(2):
                    for b in range(2):
                        for c in range(2):
                            J[:, 0] += ds[a] * wt[b] * wu[c] * P[a, b, c]
                            J[:, 1] += ws[a] * ds[b] * wu[c] * P[a, b, c]
                            J[:, 2] += ws[a] * wt[b] * ds[c] * P[a, b, c]
                vol += 0.125 * np.linalg.det(J)
    return vol


def _perturbed_nodes(dims, amp, seed):
    rng = np.random.default_rng(seed)
    X = cases.cartesian_nodes(dims)
    return X + amp * rng.uniform(-1, 1, X.shape)


def test_volume_matches_trilinear_quadrature():
    X = _perturbed_nodes((3, 3, 3), 0.25, 7)
    _, S, V = geometry.build_metrics(_case_from_nodes(X), G)
    V = V[0]
    for (i, j, k) in [(0, 0, 0), (1, 2, 0), (2, 1, 2), (1, 1, 1)]:
        P = np.empty((2, 2, 2, 3))
        for a in range(2):
            for b in range(2):
                for c in range(2):
                    P[a, b, c] = X[:, k + c, j + b, i + a]
        assert abs(V[k + G, j + G, i + G] - _trilinear_volume_gauss(P)) < 1e-14


def test_face_vector_matches_bilinear_area_integral():
    """S_d equals the integral of x_s x x_t over the bilinear face (Gauss, exact)."""
    X = _perturbed_nodes((3, 3, 3), 0.25, 11)
    _, S, _ = geometry.build_metrics(_case_from_nodes(X), G)
    S = S[0]
    gp = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    cyc = {0: (1, 2), 1: (2, 0), 2: (0, 1)}
    for d in range(3):
        t1, t2 = cyc[d]
        i, j, k = 1, 1, 1
        base = np.array([i, j, k])

        def node(o1, o2):
            idx = base.copy()
            idx[t1] += o1
            idx[t2] += o2
            return X[:, idx[2], idx[1], idx[0]]
        A = np.zeros(3)
        for s in gp:
            for t in gp:
                xs = (1 - t) * (node(1, 0) - node(0, 0)) + t * (node(1, 1) - node(0, 1))
                xt = (1 - s) * (node(0, 1) - node(0, 0)) + s * (node(1, 1) - node(1, 0))
                A += 0.25 * np.cross(xs, xt)
        assert np.max(np.abs(S[d][:, k + G, j + G, i + G] - A)) < 1e-14


def test_closed_cell_identity():
    X = _perturbed_nodes((4, 3, 5), 0.2, 5)
    _, S, _ = geometry.build_metrics(_case_from_nodes(X), G)
    S = S[0]
    tot = np.zeros_like(S[0][:, :-1, :-1, :-1])
    tot += S[0][:, :-1, :-1, 1:] - S[0][:, :-1, :-1, :-1]
    tot += S[1][:, :-1, 1:, :-1] - S[1][:, :-1, :-1, :-1]
    tot += S[2][:, 1:, :-1, :-1] - S[2][:, :-1, :-1, :-1]
    assert np.max(np.abs(tot)) < 8e-15   # a few ulp of |S| ~ 1


def test_extrapolated_ghost_nodes_continue_affine_lattice():
    rng = np.random.default_rng(1)
    E = np.eye(3) + 0.3 * rng.uniform(-1, 1, (3, 3))
    dims = (3, 4, 2)
    X = _affine_nodes(dims, E, np.zeros(3))
    Xs, _, _ = geometry.build_metrics(_case_from_nodes(X), G)
    big = _affine_nodes((3 + 2 * G, 4 + 2 * G, 2 + 2 * G), E, -G * E.sum(axis=1))
    assert np.max(np.abs(Xs[0] - big)) < 1e-13


def test_periodic_ghost_nodes_and_metrics():
    h = 0.5
    dims = (4, 3, 5)
    X = cases.cartesian_nodes(dims, h=(h, h, h))
    L = tuple(n * h for n in dims)
    Xs, S, V = geometry.build_metrics(_case_from_nodes(X, periodic=L), G)
    big = cases.cartesian_nodes(tuple(n + 2 * G for n in dims), origin=(-G * h,) * 3, h=(h, h, h))
    assert np.array_equal(Xs[0], big)
    assert np.all(V[0] == h ** 3)


@pytest.mark.parametrize("parts", [(2, 1, 1), (2, 2, 2)])
def test_split_metrics_match_parent(parts):
    """Metrics of a split periodic box equal the parent's, ghosts included."""
    c = cases.vortex_case(8, curvilinear=True)
    sc = cases.split_periodic_box(c, parts)
    _, S1, V1 = geometry.build_metrics(c, G)
    _, S2, V2 = geometry.build_metrics(sc, G)
    n = 8
    si, sj, sk = n // parts[0], n // parts[1], n // parts[2]
    b = 0
    for bk in range(parts[2]):
        for bj in range(parts[1]):
            for bi in range(parts[0]):
                for (i, j, k) in [(-2, 0, 0), (si + 1, 1, 1), (0, -1, -2), (si - 1, sj, sk + 1), (-1, -1, -1)]:
                    I = (bi * si + i) % n
                    J = (bj * sj + j) % n
                    K = (bk * sk + k) % n
                    assert abs(V2[b][k + G, j + G, i + G] - V1[0][K + G, J + G, I + G]) < 1e-14
                    for d in range(3):
                        assert np.max(np.abs(S2[b][d][:, k + G, j + G, i + G]
                                             - S1[0][d][:, K + G, J + G, I + G])) < 1e-14
                b += 1
