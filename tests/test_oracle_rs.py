"""Pins of the oracle's Ruge-Stueben coarsening (classical strength, PMIS
splitting, direct interpolation): defining properties checked against the
matrices themselves, closed forms in 1D, and the Galerkin product."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla

import gwinputs as gi


def _strong(A, theta):
    S = A.to_scipy().tocsr()
    n = S.shape[0]
    rows = []
    for i in range(n):
        lo, hi = S.indptr[i], S.indptr[i + 1]
        js, vs = S.indices[lo:hi], S.data[lo:hi]
        off = js != i
        mx = max([0.0] + list(-vs[off]))
        rows.append(set(js[off][-vs[off] >= theta * mx]) if mx > 0 else set())
    return rows


def _check_level(ref, H, l, theta):
    lv = H.level(l)
    A = lv.A
    S = _strong(A, theta)
    n = A.n
    cf = lv.state
    dependents = [0] * n
    for i in range(n):
        for j in S[i]:
            dependents[j] += 1
    for i in range(n):
        assert cf[i] in (ref.CF_C, ref.CF_F)
        if dependents[i] == 0:
            assert cf[i] == ref.CF_F
        if cf[i] == ref.CF_F and dependents[i] > 0:
            # an F point decided in a round depends strongly on a C point, so
            # it has something to interpolate from
            assert any(cf[j] == ref.CF_C for j in S[i]), i
    # numbering and rows of P
    P = lv.P.to_scipy().tocsr()
    c_ids = np.cumsum(cf == ref.CF_C) - 1
    Ad = A.to_scipy().tocsr()
    for i in range(n):
        cols = P.indices[P.indptr[i]:P.indptr[i + 1]]
        vals = P.data[P.indptr[i]:P.indptr[i + 1]]
        if cf[i] == ref.CF_C:
            assert list(cols) == [c_ids[i]] and list(vals) == [1.0]
            continue
        strong_c = sorted(c_ids[j] for j in S[i] if cf[j] == ref.CF_C)
        assert list(cols) == strong_c
        row = Ad.getrow(i).toarray().ravel()
        if len(cols) and abs(row.sum()) <= 1e-12 * abs(row[i]):
            # zero row sum: the weights interpolate constants exactly
            assert abs(vals.sum() - 1.0) <= 1e-12
    # Galerkin coarse operator
    Ac = H.level(l + 1).A.to_scipy()
    G = (P.T @ Ad @ P).tocsr()
    assert abs(Ac - G).max() <= 1e-12 * abs(G).max()


def test_rs_1d_closed_form(ref):
    # 1D Laplacian with zero row sums inside: an F point between two C points
    # takes 1/2 from each, one next to a single C point takes 1
    n = 64
    T = sp.diags([-np.ones(n - 1), 2.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    T = T.tolil()
    T[0, 0] = 1.0
    T[n - 1, n - 1] = 1.0
    T = (T + sp.eye(n) * 1e-3).tocsr()
    T.sort_indices()
    A = ref.Csr(T.indptr.astype(np.int32), T.indices.astype(np.int32), T.data.copy())
    H = ref.Hierarchy(A, ref.AmgParams(coarsening=ref.RS, eps_strong=0.25, n_coarse=8))
    lv = H.level(0)
    cf = lv.state
    P = lv.P.to_scipy().tocsr()
    for i in range(1, n - 1):
        if cf[i] != ref.CF_F:
            continue
        nb = [j for j in (i - 1, i + 1) if cf[j] == ref.CF_C]
        vals = P.data[P.indptr[i]:P.indptr[i + 1]]
        d = 2.0 + 1e-3
        if len(nb) == 2:
            assert np.allclose(vals, [1.0 / d, 1.0 / d], rtol=1e-14)
        elif len(nb) == 1:
            assert np.allclose(vals, [2.0 / d], rtol=1e-14)
    _check_level(ref, H, 0, 0.25)


def test_rs_properties_on_aquifer(ref):
    p = gi.heterogeneous_aquifer(16, 12, 6, 4.0, 4, 3)
    A, b = ref.fv_assemble(p)
    H = ref.Hierarchy(A, ref.AmgParams(coarsening=ref.RS, eps_strong=0.25, n_coarse=30))
    assert H.nlevels >= 3
    for l in range(H.nlevels - 1):
        _check_level(ref, H, l, 0.25)


def test_rs_pcg_converges(ref):
    p = gi.heterogeneous_aquifer(20, 16, 8, 4.0, 4, 9)
    A, b = ref.fv_assemble(p)
    exact = sla.spsolve(A.to_scipy().tocsc(), b)
    H = ref.Hierarchy(A, ref.AmgParams(coarsening=ref.RS, eps_strong=0.25, n_coarse=40))
    x, info = ref.pcg(H, b, rtol=1e-10)
    assert info.status == ref.OK and info.iters < 40
    assert np.linalg.norm(x - exact) / np.linalg.norm(exact) < 1e-7
