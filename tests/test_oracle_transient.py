"""Pins of the oracle's transient flow step (Eq. 2) and reuse criterion (CPU)."""
import numpy as np
import scipy.linalg as la
import scipy.sparse.linalg as sla

import gwinputs as gi


def test_storage_shift_and_ratio_by_hand(ref):
    g = gi.Grid(3, 1, 1, dx=2.0, dy=3.0, dz=0.5)
    s = ref.storage_shift(g, np.array([1e-4, 2e-4, 4e-4]), 10.0)
    assert np.allclose(s, [3e-4 / 10, 6e-4 / 10, 12e-4 / 10], rtol=1e-15)
    A = ref.Csr(np.array([0, 2, 5, 7], np.int32), np.array([0, 1, 0, 1, 2, 1, 2], np.int32),
                np.array([4.0, -1.0, -1.0, 2.0, -1.0, -1.0, 8.0]))
    assert ref.reuse_ratio(A, np.array([0.04, 0.01, 0.08])) == 0.01


def test_steady_state_is_a_fixed_point(ref):
    # h0 = the steady solution: C h0 = b, so (C + S/dt) h0 = b + (S/dt) h0
    p = gi.heterogeneous_aquifer(12, 10, 4, 2.0, 3, 9)
    A, b = ref.fv_assemble(p)
    h_ss = sla.spsolve(A.to_scipy().tocsc(), b)
    Ss = np.full(p.grid.n, 1e-4)
    r = ref.transient_flow(p, Ss, h_ss, [1.0, 100.0, 1e4])
    for h in r.heads:
        assert np.allclose(h, h_ss, rtol=1e-11, atol=1e-11)


def test_long_step_reaches_steady_state(ref):
    p = gi.heterogeneous_aquifer(12, 10, 4, 2.0, 3, 9)
    A, b = ref.fv_assemble(p)
    h_ss = sla.spsolve(A.to_scipy().tocsc(), b)
    r = ref.transient_flow(p, np.full(p.grid.n, 1e-5), np.zeros(p.grid.n), [1e12])
    assert np.allclose(r.heads[0], h_ss, rtol=1e-9, atol=1e-9)
    assert r.reuse == [True]


def test_matches_modal_solution(ref):
    # implicit Euler of S dh/dt = b - C h, solved independently through the
    # eigen-decomposition of the symmetric pencil (C, S): with
    # C V = S V diag(lam) and V^T S V = I, each mode decays by
    # 1 / (1 + lam dt) per step around the steady state
    p = gi.Problem(gi.Grid(7, 3, 2), gi.random_k(gi.Grid(7, 3, 2), 4, 1e-5, 1e-3),
                   wells=[gi.Well(3, 1, 0, 2e-5)])
    g = p.grid
    A, b = ref.fv_assemble(p)
    C = A.dense()
    Ss = np.linspace(1e-4, 3e-4, g.n)
    S = np.diag(Ss * ((g.dx * g.dy) * g.dz))
    lam, V = la.eigh(C, S)
    h_ss = np.linalg.solve(C, b)
    h0 = np.zeros(g.n)
    dts = [0.5, 2.0, 2.0, 30.0]
    r = ref.transient_flow(p, Ss, h0, dts)
    c = V.T @ S @ (h0 - h_ss)
    for dt, h in zip(dts, r.heads):
        c = c / (1.0 + lam * dt)
        assert np.allclose(h, h_ss + V @ c, rtol=1e-9, atol=1e-12)


def test_reuse_decision_follows_the_criterion(ref):
    p = gi.heterogeneous_aquifer(10, 8, 4, 1.0, 3, 2)
    A, _ = ref.fv_assemble(p)
    d = A.to_scipy().diagonal()
    Ss = np.full(p.grid.n, 2e-4)
    # the step at which S V / dt equals delta C_ii for the weakest row
    dt_star = float(np.max(Ss / (0.01 * d)))
    r = ref.transient_flow(p, Ss, np.zeros(p.grid.n), [0.5 * dt_star, 2.0 * dt_star])
    assert r.reuse == [False, True]
    assert np.isclose(r.ratios[0], 0.02, rtol=1e-12) and np.isclose(r.ratios[1], 0.005, rtol=1e-12)
