"""Pins of the oracle's smoothed-aggregation setup and V-cycle (CPU only).

The strength graph is rebuilt here from its definition with numpy so that the
MIS-2 / aggregation invariants are checked against an independent graph; the
MIS-2 rounds are compared with a brute-force greedy selection; the Galerkin
product with SciPy's sparse product; the coarsest LU with LAPACK (SciPy).
"""
from collections import deque

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp

import gwinputs as gi


def _strength_graph(A, eps2):
    """Symmetrised strength graph from its definition (numpy/scipy)."""
    S = A.to_scipy().tocoo()
    d = A.to_scipy().diagonal()
    i, j, v = S.row, S.col, S.data
    off = i != j
    i, j, v = i[off], j[off], v[off]
    strong = v * v > eps2 * (d[i] * d[j])
    G = sp.coo_matrix((np.ones(strong.sum()), (i[strong], j[strong])), shape=S.shape).tocsr()
    G = ((G + G.T) > 0).astype(np.int8).tocsr()
    G.sort_indices()
    return G


def _bfs_dist(G, src, cap=3):
    dist = {src: 0}
    dq = deque([src])
    while dq:
        u = dq.popleft()
        if dist[u] >= cap:
            continue
        for v in G.indices[G.indptr[u]:G.indptr[u + 1]]:
            if v not in dist:
                dist[v] = dist[u] + 1
                dq.append(v)
    return dist


def _problem(shape=(12, 10, 6), s2=2.0, seed=3):
    return gi.heterogeneous_aquifer(*shape, s2, 3, seed)


@pytest.fixture(scope="module")
def small_h(ref):
    p = _problem()
    A, b = ref.fv_assemble(p)
    H = ref.Hierarchy(A, ref.AmgParams(n_coarse=20, seed=77))
    return A, b, H


def test_mis2_equals_greedy_by_priority(ref, small_h):
    # Synchronous MIS-2 rounds with unique keys select exactly the nodes a
    # greedy pass in descending key order selects (pick a node when no picked
    # node lies within distance 2).
    A, _, H = small_h
    for l in range(H.nlevels - 1):
        L = H.level(l)
        G = _strength_graph(L.A, (0.08 * 0.08) * 0.25 ** l)
        keys = ref.mis2_keys(L.A.n, 77, l)
        removed = np.diff(G.indptr) == 0
        order = np.argsort(-keys.astype(np.float64), kind="stable")
        # exact ordering on uint64
        order = sorted(range(L.A.n), key=lambda i: int(keys[i]), reverse=True)
        picked = np.zeros(L.A.n, bool)
        blocked = np.zeros(L.A.n, bool)
        for u in order:
            if removed[u] or blocked[u]:
                continue
            picked[u] = True
            for v in _bfs_dist(G, u, 2):
                blocked[v] = True
        assert np.array_equal(picked, L.state == 2), f"level {l}"


def test_mis2_and_aggregate_invariants(ref, small_h):
    A, _, H = small_h
    for l in range(H.nlevels - 1):
        L = H.level(l)
        G = _strength_graph(L.A, (0.08 * 0.08) * 0.25 ** l)
        roots = np.flatnonzero(L.state == 2)
        removed = np.diff(G.indptr) == 0
        # roots pairwise at distance >= 3; every kept node within 2 of a root
        near = np.full(L.A.n, 99)
        for r in roots:
            for v, dv in _bfs_dist(G, r, 2).items():
                if v != r:
                    assert not (L.state[v] == 2), "two roots within distance 2"
                near[v] = min(near[v], dv)
        assert np.all(near[~removed] <= 2)
        # removed nodes have no aggregate, all others have one
        assert np.all(L.agg[removed] == -1)
        assert np.all(L.agg[~removed] >= 0)
        # aggregate ids: roots numbered by ascending node index
        assert np.array_equal(L.agg[roots], np.arange(len(roots)))
        assert L.nc == len(roots)
        # every aggregate is connected in the strength graph
        for a in range(L.nc):
            members = set(np.flatnonzero(L.agg == a).tolist())
            seen = {roots[a]}
            dq = deque([roots[a]])
            while dq:
                u = dq.popleft()
                for v in G.indices[G.indptr[u]:G.indptr[u + 1]]:
                    if v in members and v not in seen:
                        seen.add(v)
                        dq.append(v)
            assert seen == members
        # tentative prolongator column sums = aggregate sizes
        Pt = sp.csr_matrix((np.ones((~removed).sum()), (np.flatnonzero(~removed), L.agg[~removed])),
                           shape=(L.A.n, L.nc))
        assert np.array_equal(np.asarray(Pt.sum(axis=0)).ravel(), np.bincount(L.agg[~removed], minlength=L.nc))


def test_prolongator_preserves_row_sums(ref, small_h):
    # P 1 = (I - omega D_F^{-1} A_F) P_tent 1 = 1 - omega D_F^{-1} A_F 1, and
    # lumping keeps A_F 1 = A 1: rows away from the fixed-head faces have
    # A 1 = 0, so their P row sums are 1.
    A, _, H = small_h
    L = H.level(0)
    P = L.P.to_scipy()
    rs = np.asarray(P.sum(axis=1)).ravel()
    Arow = np.asarray(L.A.to_scipy().sum(axis=1)).ravel()
    zero_rows = np.abs(Arow) <= 1e-14 * L.A.to_scipy().diagonal()
    assert zero_rows.sum() > 0
    assert np.allclose(rs[zero_rows], 1.0, atol=1e-12)
    # Gershgorin weight: 7-point matrix with zero row sums -> rho <= 2
    assert 2.0 / 3.0 - 1e-12 <= L.omega_p


def test_galerkin_product_matches_scipy(ref, small_h):
    A, _, H = small_h
    for l in range(H.nlevels - 1):
        L, Lc = H.level(l), H.level(l + 1)
        P = L.P.to_scipy()
        Ac_ref = (P.T @ L.A.to_scipy() @ P).toarray()
        Ac = Lc.A.dense()
        assert np.allclose(Ac, Ac_ref, rtol=1e-12, atol=1e-13 * np.abs(Ac_ref).max())
        # symmetric up to rounding; sorted CSR with stored diagonal
        assert np.allclose(Ac, Ac.T, rtol=1e-12, atol=1e-13 * np.abs(Ac).max())
        assert ref.csr_check(Lc.A) == 0


def test_coarse_lu_matches_lapack(ref, small_h):
    A, _, H = small_h
    Ac = H.level(H.nlevels - 1).A.dense()
    lu, piv = H.coarse_lu()
    lu_ref, piv_ref = sl.lu_factor(Ac)
    assert np.array_equal(piv, piv_ref)
    assert np.allclose(lu, lu_ref, rtol=1e-11, atol=1e-12 * np.abs(lu_ref).max())


def test_vcycle_symmetric_positive(ref, small_h):
    # With equal pre/post sweeps of a diagonal smoother and R = P^T the V-cycle
    # is a symmetric positive definite operator (up to rounding).
    A, _, H = small_h
    u = gi.random_vector(A.n, 1)
    v = gi.random_vector(A.n, 2)
    Vu, Vv = H.vcycle(u), H.vcycle(v)
    assert abs(u @ Vv - v @ Vu) <= 1e-11 * abs(u @ Vv)
    assert u @ Vu > 0 and v @ Vv > 0


def test_two_level_coarse_exactness(ref):
    # Smoothing off, two levels, exact coarse solve: V(A P y) = P y.
    p = _problem((10, 9, 5))
    A, _ = ref.fv_assemble(p)
    H = ref.Hierarchy(A, ref.AmgParams(npre=0, npost=0, max_levels=2, n_coarse=1))
    assert H.nlevels == 2
    P = H.level(0).P.to_scipy()
    y = gi.random_vector(P.shape[1], 4)
    b = A.to_scipy() @ (P @ y)
    assert np.allclose(H.vcycle(b), P @ y, rtol=1e-10, atol=1e-10 * np.abs(P @ y).max())


def test_setup_is_deterministic(ref):
    p = _problem((14, 9, 5), s2=4.0, seed=9)
    A, _ = ref.fv_assemble(p)
    H1 = ref.Hierarchy(A)
    H2 = ref.Hierarchy(A)
    assert H1.nlevels == H2.nlevels
    for l in range(H1.nlevels):
        a, b = H1.level(l), H2.level(l)
        assert np.array_equal(a.A.val, b.A.val) and np.array_equal(a.A.col, b.A.col)
        if a.agg is not None:
            assert np.array_equal(a.agg, b.agg)
    # a different seed changes the aggregates but not the validity
    H3 = ref.Hierarchy(A, ref.AmgParams(seed=12345))
    assert not np.array_equal(H3.level(0).agg, H1.level(0).agg)


def test_smoother_diagonals(ref, small_h):
    A, _, H = small_h
    L = H.level(0)
    S = L.A.to_scipy()
    d = S.diagonal()
    # SPAI0: argmin over diagonal M of ||I - M A||_F gives m_i = a_ii / ||a_i||^2
    rownorm2 = np.asarray(S.multiply(S).sum(axis=1)).ravel()
    assert np.allclose(L.M, d / rownorm2, rtol=1e-14)
    HJ = ref.Hierarchy(A, ref.AmgParams(smoother=ref.JACOBI, omega=0.5, n_coarse=20))
    assert np.allclose(HJ.level(0).M, 0.5 / d, rtol=1e-15)


def test_invalid_matrix_rejected(ref):
    A = ref.Csr(np.array([0, 2, 3], np.int32), np.array([1, 0, 1], np.int32), np.array([1.0, 2.0, 3.0]))
    assert ref.csr_check(A) != 0  # unsorted row 0
    with pytest.raises(ValueError):
        ref.Hierarchy(A)
    A = ref.Csr(np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, -3.0]))
    with pytest.raises(ValueError):
        ref.Hierarchy(A)  # non-positive diagonal
