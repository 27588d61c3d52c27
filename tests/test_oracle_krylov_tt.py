"""Pins of the oracle's Krylov solvers and travel-time system (CPU only)."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import gwinputs as gi


def test_cg_without_preconditioner_matches_scipy_iterates(ref):
    # With the preconditioner off, PCG is textbook CG: after k iterations its
    # iterate equals SciPy's CG after k iterations (same x0 = 0).
    g = gi.Grid(9, 7, 3)
    p = gi.Problem(g, gi.random_k(g, 2, 1e-5, 1e-3))
    A, b = ref.fv_assemble(p)
    H = ref.Hierarchy(A, ref.AmgParams(smoother=ref.NONE))
    S = A.to_scipy()
    for k in (1, 3, 7):
        x, info = ref.pcg(H, b, rtol=1e-30, maxiter=k)
        assert info.status == ref.NOT_CONVERGED and info.iters == k
        xs, _ = sla.cg(S, b, x0=np.zeros(g.n), rtol=1e-30, atol=0.0, maxiter=k)
        assert np.allclose(x, xs, rtol=1e-10, atol=1e-12 * np.abs(xs).max())


def test_flexible_cg_agrees_with_pcg(ref):
    # With an exact-arithmetic-symmetric preconditioner the Polak-Ribiere beta
    # equals the Fletcher-Reeves one: FCG and PCG converge alike.
    p = gi.heterogeneous_aquifer(16, 16, 8, 1.0, 4, 5)
    A, b = ref.fv_assemble(p)
    H = ref.Hierarchy(A, ref.AmgParams(n_coarse=40))
    x1, i1 = ref.pcg(H, b, rtol=1e-10)
    x2, i2 = ref.pcg(H, b, rtol=1e-10, flexible=True)
    assert i1.status == 0 and i2.status == 0
    assert abs(i1.iters - i2.iters) <= 1
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) < 1e-8


def test_status_codes(ref):
    p = gi.heterogeneous_aquifer(12, 12, 6, 1.0, 4, 1)
    A, b = ref.fv_assemble(p)
    H = ref.Hierarchy(A, ref.AmgParams(n_coarse=30))
    x, info = ref.pcg(H, b, rtol=1e-12, maxiter=1)
    assert info.status == ref.NOT_CONVERGED and info.iters == 1 and info.rel_res_true > 1e-12
    x, info = ref.pcg(H, np.zeros_like(b))
    assert info.status == 0 and info.iters == 0 and not x.any()
    bad = b.copy()
    bad[5] = np.nan
    x, info = ref.pcg(H, bad)
    assert info.status == ref.BREAKDOWN
    x, info = ref.bicgstab(H, bad)
    assert info.status == ref.BREAKDOWN
    x, info = ref.bicgstab(H, b, rtol=1e-12, maxiter=1)
    assert info.status == ref.NOT_CONVERGED


def test_bicgstab_on_symmetric_system(ref):
    p = gi.heterogeneous_aquifer(16, 12, 8, 2.0, 4, 8)
    A, b = ref.fv_assemble(p)
    H = ref.Hierarchy(A, ref.AmgParams(n_coarse=40))
    x, info = ref.bicgstab(H, b, rtol=1e-10)
    xd = sla.spsolve(A.to_scipy().tocsc(), b)
    assert info.status == 0 and info.rel_res_true <= 1e-10
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-7


def _uniform_flow(nx=64, ny=8):
    p = gi.homogeneous_slab(nx, ny)
    return p


def test_travel_time_uniform_flow(ref):
    # T1: in uniform flow q = K (h_w - h_e) / L per unit face area, the exact
    # upwind solution is tau_i = phi (i + 1) dx / v, the time to reach the
    # cell's downstream face; it is within half a cell of phi x_centre / v.
    p = _uniform_flow()
    g = p.grid
    A, b = ref.fv_assemble(p)
    h = sla.spsolve(A.to_scipy().tocsc(), b)
    qx, qy, qz = ref.darcy_flux(p, h)
    v = 1e-4 * 10.0 / g.nx
    assert np.allclose(qx, v, rtol=1e-12)
    phi = 0.25
    At, bt, bc, nid = ref.tt_assemble(g, qx, qy, qz, phi)
    assert nid == 0
    i = np.arange(g.n) % g.nx
    tau_exact = phi * (i + 1) * g.dx / v
    tau_sweep = ref.tt_sweep(At, bt, h)
    assert np.allclose(tau_sweep, tau_exact, rtol=1e-10)
    assert np.all(np.abs(tau_sweep - phi * (i + 0.5) * g.dx / v) <= 0.5 * phi * g.dx / v * (1 + 1e-9))
    H = ref.Hierarchy(At, ref.AmgParams(n_coarse=40))
    tau, info = ref.bicgstab(H, bt, rtol=1e-10)
    assert info.status == 0
    assert np.allclose(tau, tau_exact, rtol=1e-8)


def test_travel_time_indicator_and_row_sums(ref):
    p = gi.heterogeneous_aquifer(20, 16, 8, 2.0, 4, 21)
    g = p.grid
    A, b = ref.fv_assemble(p)
    h = sla.spsolve(A.to_scipy().tocsc(), b)
    qx, qy, qz = ref.darcy_flux(p, h)
    At, bt, bc_full, nid = ref.tt_assemble(g, qx, qy, qz, 0.25)
    # T3: row sums = inflow through boundary faces (x = 0 plus x = L)
    qx3 = qx.reshape(g.nz, g.ny, g.nx + 1)
    bnd = np.zeros((g.nz, g.ny, g.nx))
    bnd[:, :, 0] += np.maximum(qx3[:, :, 0], 0)
    bnd[:, :, -1] += np.maximum(-qx3[:, :, -1], 0)
    rs = np.asarray(At.to_scipy().sum(axis=1)).ravel()
    scale = np.abs(At.val).max()
    assert np.allclose(rs, bnd.reshape(-1), atol=1e-12 * scale)
    # T2: the indicator of the whole inflow face; every row is a convex
    # average of 1 (boundary) and upstream values, so 0 <= c <= 1; with all
    # inflow through x = 0 (here no inflow at x = L) c == 1.
    c_full = ref.tt_sweep(At, bc_full, h)
    assert np.all(c_full >= -1e-12) and np.all(c_full <= 1 + 1e-12)
    if not (bnd[:, :, -1] > 0).any():
        assert np.allclose(c_full, 1.0, atol=1e-12)
    # a half-face source zone gives a non-trivial fraction field
    _, _, bc_half, _ = ref.tt_assemble(g, qx, qy, qz, 0.25, zone=(0, g.ny, 0, g.nz // 2))
    c_half = ref.tt_sweep(At, bc_half, h)
    assert np.all(c_half >= -1e-12) and np.all(c_half <= 1 + 1e-12)
    assert 0.05 < c_half.mean() < 0.95
    # T4: the sweep is the exact solution; BiCGSTAB + AMG agrees within rtol * cond
    H = ref.Hierarchy(At, ref.AmgParams(n_coarse=40))
    tau_sweep = ref.tt_sweep(At, bt, h)
    for rhs, exact in ((bt, tau_sweep), (bc_half, c_half)):
        assert np.allclose(At.to_scipy() @ exact, rhs, rtol=1e-12, atol=1e-12 * np.abs(rhs).max())
        x, info = ref.bicgstab(H, rhs, rtol=1e-10)
        assert info.status == 0
        assert np.linalg.norm(x - exact) / np.linalg.norm(exact) < 1e-6
    # the upwind matrix is an M-matrix: off-diagonals <= 0, rows dominated
    D = At.to_scipy().toarray()
    off = D - np.diag(np.diag(D))
    assert np.all(off <= 0) and np.all(np.diag(D) > 0)


def test_travel_time_identity_rows(ref):
    # a cell with no inflow face (all fluxes zero) becomes an identity row
    g = gi.Grid(4, 3, 2)
    qx = np.zeros((g.nx + 1) * g.ny * g.nz)
    qy = np.zeros(g.nx * (g.ny + 1) * g.nz)
    qz = np.zeros(g.nx * g.ny * (g.nz + 1))
    At, bt, bc, nid = ref.tt_assemble(g, qx, qy, qz, 0.25)
    assert nid == g.n
    assert np.array_equal(At.dense(), np.eye(g.n)) and not bt.any() and not bc.any()
