"""Pins of the oracle's ILU(0) smoother (Results: the relaxation used
throughout), independent of the oracle's own code: the defining property of
ILU(0), exactness where no fill can occur, symmetry, and convergence."""
import numpy as np
import scipy.linalg as la
import scipy.sparse as sp
import scipy.sparse.linalg as sla

import gwinputs as gi


def _factors(ref, A, ilu):
    S = A.to_scipy().tocsr()
    F = sp.csr_matrix((ilu, A.col, A.rowptr), shape=S.shape)
    L = sp.tril(F, -1).tocsr() + sp.eye(A.n)
    U = sp.triu(F).tocsr()
    return S, L, U


def test_ilu0_matches_a_on_its_pattern(ref):
    # ILU(0) is the factorization whose product agrees with A on A's pattern;
    # the Galerkin levels (dense rows) exercise updates of lower entries too
    p = gi.heterogeneous_aquifer(20, 16, 8, 2.0, 3, 5)
    A, _ = ref.fv_assemble(p)
    H = ref.Hierarchy(A, ref.AmgParams(smoother=ref.ILU0, n_coarse=40))
    assert H.nlevels >= 3
    for l in range(H.nlevels - 1):
        Al = H.level(l).A
        S, L, U = _factors(ref, Al, H.level_ilu(l))
        LU = (L @ U).tocsr()
        pat = S.copy()
        pat.data[:] = 1.0
        on = LU.multiply(pat)
        scale = np.abs(S.data).max()
        assert np.abs((on - S).data).max() <= 1e-12 * scale, l


def test_ilu0_is_exact_without_fill(ref):
    # a tridiagonal matrix (one row of cells) has no fill: ILU(0) = LU, so a
    # single smoothing sweep from zero solves the level's system exactly
    n = 60
    main = 2.0 + np.linspace(0.1, 0.9, n)
    T = sp.diags([-np.ones(n - 1), main, -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    T.sort_indices()
    A = ref.Csr(T.indptr.astype(np.int32), T.indices.astype(np.int32), T.data.copy())
    H = ref.Hierarchy(A, ref.AmgParams(smoother=ref.ILU0, n_coarse=10, npre=1, npost=0))
    S, L, U = _factors(ref, A, H.level_ilu(0))
    Ld = L.toarray()
    Ud = U.toarray()
    P, Ls, Us = la.lu(T.toarray())
    assert np.allclose(P, np.eye(n))
    assert np.allclose(Ld, Ls, rtol=1e-13, atol=1e-14) and np.allclose(Ud, Us, rtol=1e-13, atol=1e-14)


def test_ilu0_of_symmetric_matrix_is_ldlt(ref):
    # symmetric A with a symmetric pattern: U = D L^T, so (LU)^{-1} is a
    # symmetric smoother and the V-cycle stays a valid CG preconditioner
    p = gi.heterogeneous_aquifer(12, 10, 4, 3.0, 3, 6)
    A, _ = ref.fv_assemble(p)
    H = ref.Hierarchy(A, ref.AmgParams(smoother=ref.ILU0, n_coarse=40))
    S, L, U = _factors(ref, A, H.level_ilu(0))
    D = sp.diags(U.diagonal())
    assert np.allclose((D @ L.T).toarray(), U.toarray(), rtol=1e-12, atol=1e-18)


def test_ilu0_amg_pcg_converges(ref):
    p = gi.heterogeneous_aquifer(20, 16, 8, 4.0, 4, 9)
    A, b = ref.fv_assemble(p)
    exact = sla.spsolve(A.to_scipy().tocsc(), b)
    its = {}
    for sm in (ref.SPAI0, ref.ILU0):
        H = ref.Hierarchy(A, ref.AmgParams(smoother=sm, n_coarse=40))
        x, info = ref.pcg(H, b, rtol=1e-10)
        assert info.status == ref.OK
        assert np.linalg.norm(x - exact) / np.linalg.norm(exact) < 1e-7
        its[sm] = info.iters
    # ILU(0) is the stronger smoother per sweep
    assert its[ref.ILU0] < its[ref.SPAI0]
