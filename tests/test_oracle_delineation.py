"""Pins of the oracle's dual delineation (CPU only).

Forward and backward travel times have closed forms in uniform flow, and the
indicators are probabilities that must add up: every unit of water entering
a cell came from exactly one source (forward), and every unit leaving it ends
in exactly one sink (backward).  A dropped well term or a misplaced
right-hand side breaks one of these sums.
"""
import numpy as np
import scipy.sparse.linalg as sla

import gwinputs as gi


def _heads(ref, p):
    A, b = ref.fv_assemble(p)
    return sla.spsolve(A.to_scipy().tocsc(), b)


def test_uniform_flow_closed_forms(ref):
    # uniform flow along x: tau_f = phi (i + 1) dx / v (time to the cell's
    # downstream face), tau_b = phi (nx - i) dx / v (time from the upstream
    # face to the outlet), so tau_f + tau_b = phi (nx + 1) dx / v everywhere;
    # two zones splitting the inflow face give indicators 1 on their own
    # streamlines and 0 elsewhere
    p = gi.homogeneous_slab(48, 10)
    g = p.grid
    h = _heads(ref, p)
    qx, qy, qz = ref.darcy_flux(p, h)
    v = qx.reshape(g.nz, g.ny, g.nx + 1)[0, 0, 0]
    phi = 0.3
    d = ref.dual_delineation(g, qx, qy, qz, phi, h, [(0, 4, 0, 1), (4, 10, 0, 1)], [])
    assert d.forward.shape == (3, g.n) and d.backward.shape == (1, g.n)
    i = np.arange(g.n) % g.nx
    j = (np.arange(g.n) // g.nx) % g.ny
    assert np.allclose(d.forward[0], phi * (i + 1) * g.dx / v, rtol=1e-10)
    assert np.allclose(d.backward[0], phi * (g.nx - i) * g.dx / v, rtol=1e-10)
    assert np.allclose(d.forward[0] + d.backward[0], phi * (g.nx + 1) * g.dx / v, rtol=1e-10)
    assert np.allclose(d.forward[1], (j < 4).astype(float), atol=1e-10)
    assert np.allclose(d.forward[2], (j >= 4).astype(float), atol=1e-10)


def _wells_problem():
    g = gi.Grid(24, 18, 6)
    K = gi.lognormal_field((24, 18, 6), 2.0, 4.0, 31)
    wells = [gi.Well(16, 5, 2, 2e-4), gi.Well(8, 12, 3, -1.5e-4), gi.Well(19, 13, 1, 1e-4),
             gi.Well(19, 13, 1, 5e-5)]
    return gi.Problem(g, K, wells=wells)


def test_indicators_add_up(ref):
    p = _wells_problem()
    g = p.grid
    h = _heads(ref, p)
    qx, qy, qz = ref.darcy_flux(p, h)
    phi = 0.25
    zones = [(0, 9, 0, 6), (9, 18, 0, 3), (9, 18, 3, 6)]  # a partition of the x = 0 face
    d = ref.dual_delineation(g, qx, qy, qz, phi, h, zones, p.wells)
    n_inj = sum(w.q < 0 for w in p.wells)
    n_prod = sum(w.q > 0 for w in p.wells)
    assert d.forward.shape == (1 + len(zones) + n_inj, g.n)
    assert d.backward.shape == (1 + n_prod, g.n)
    # exact solutions of their (well-modified) systems
    for A, rhs, X in ((d.A_forward, d.rhs_forward, d.forward), (d.A_backward, d.rhs_backward, d.backward)):
        S = A.to_scipy()
        for b, x in zip(rhs, X):
            assert np.allclose(S @ x, b, rtol=0, atol=1e-12 * max(np.abs(b).max(), 1e-300) + 1e-300)
    qx3 = qx.reshape(g.nz, g.ny, g.nx + 1)
    assert (qx3[:, :, -1] >= 0).all(), "the workload has no inflow through x = L"
    # forward: zones + injection well account for all water
    src = d.forward[1:].sum(axis=0)
    assert np.all(d.forward[1:] >= -1e-12) and np.all(d.forward[1:] <= 1 + 1e-12)
    assert np.allclose(src, 1.0, atol=1e-9)
    # backward: production wells + the x = L outlet account for all water
    east = np.zeros((g.nz, g.ny, g.nx))
    east[:, :, -1] = np.maximum(qx3[:, :, -1], 0.0)
    c_east = ref.tt_sweep(d.A_backward, east.reshape(-1), -h)
    sink = d.backward[1:].sum(axis=0) + c_east
    assert np.all(d.backward[1:] >= -1e-12) and np.all(d.backward[1:] <= 1 + 1e-12)
    assert np.allclose(sink, 1.0, atol=1e-9)
    # the two wells sharing one cell split its capture by rate (2:1)
    cell = 19 + g.nx * (13 + g.ny * 1)
    assert np.isclose(d.backward[2, cell], 2 * d.backward[3, cell], rtol=1e-12)
    # the strong sink keeps most of the water entering its own cell
    c0 = 16 + g.nx * (5 + g.ny * 2)
    assert 0.5 < d.backward[1, c0] <= 1.0
    # travel times are positive where water flows
    assert np.all(d.forward[0] > 0) and np.all(d.backward[0] > 0)


def test_injection_well_only_source(ref):
    # with every zone dropped, the injection well's indicator is the only
    # forward source: 1 in its own cell's plume, 0 upstream of it
    p = _wells_problem()
    g = p.grid
    h = _heads(ref, p)
    qx, qy, qz = ref.darcy_flux(p, h)
    d = ref.dual_delineation(g, qx, qy, qz, 0.25, h, [], p.wells)
    c_inj = d.forward[1]
    cw = 8 + g.nx * (12 + g.ny * 3)
    assert 0.0 < c_inj[cw] <= 1.0
    upstream = h > h[cw] + 1e-9
    assert np.all(c_inj[upstream] == 0.0)
