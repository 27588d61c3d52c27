"""Direct upwind sweep on the GPU against the oracle's sequential sweep.

The GPU solves cells level by level in a topological order of the inflow
graph; the oracle visits them by descending head.  A cell's value depends
only on its inflow neighbours and both sides evaluate its row with the same
operations in the same order, so the results agree bit for bit.  Inputs are
the oracle's own matrices (assembled from oracle heads), so no face can flip
its upwind direction between the two sides.
"""
import sys

import numpy as np
import pytest

import gwinputs as gi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2001_05798_amd as gw
    return gw


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _heads(ref, p):
    import scipy.sparse.linalg as sla
    A, b = ref.fv_assemble(p)
    return sla.spsolve(A.to_scipy().tocsc(), b)


def _gpu_sweep(gw, A, rhs):
    n, k = A.n, len(rhs)
    b = dev(np.concatenate(rhs))
    x = torch.full((n * k,), np.nan, dtype=torch.float64, device="cuda")
    lev = gw.tt_sweep(n, dev(A.rowptr), dev(A.col), dev(A.val), b, x, nrhs=k)
    return host(x).reshape(k, n), lev


SWEEP_CASES = [
    ("3d 32x24x12 lognormal s2=4", lambda: gi.heterogeneous_aquifer(32, 24, 12, 4.0, 6, 4), (0, 24, 0, 6)),
    ("3d 13x7x5 random K, wells", lambda: gi.Problem(gi.Grid(13, 7, 5), gi.random_k(gi.Grid(13, 7, 5), 1),
                                                     wells=[gi.Well(3, 2, 1, 1e-5), gi.Well(9, 5, 3, 2e-5)]),
     None),
    ("nx=1 column 1x9x6", lambda: gi.Problem(gi.Grid(1, 9, 6), gi.random_k(gi.Grid(1, 9, 6), 2)), None),
    ("single cell", lambda: gi.Problem(gi.Grid(1, 1, 1), np.array([3e-4])), None),
    ("2d 64x64 homogeneous", lambda: gi.homogeneous_slab(), (0, 32, 0, 1)),
]


@pytest.mark.parametrize("name,make,zone", SWEEP_CASES, ids=[c[0] for c in SWEEP_CASES])
def test_sweep_bitwise(gw, ref, name, make, zone):
    _say(f"tt_sweep {name}")
    p = make()
    g = p.grid
    h = _heads(ref, p)
    qx, qy, qz = ref.darcy_flux(p, h)
    At, bt, bc, _ = ref.tt_assemble(g, qx, qy, qz, p.phi, zone)
    want = [ref.tt_sweep(At, bt, h), ref.tt_sweep(At, bc, h)]
    got, lev = _gpu_sweep(gw, At, [bt, bc])
    assert 1 <= lev <= g.n
    for k in range(2):
        assert np.array_equal(got[k], want[k]), np.abs(got[k] - want[k]).max()
    # the assembled-and-swept form gives the same two fields
    tau = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    c = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    lev2 = gw.tt_solve_direct(g, dev(qx), dev(qy), dev(qz), p.phi, zone, tau, c)
    assert lev2 == lev
    assert np.array_equal(host(tau), want[0]) and np.array_equal(host(c), want[1])


def test_sweep_many_rhs_and_reversed_flow(gw, ref):
    # five right-hand sides on one matrix (the dual-delineation equations share
    # it), and the reversed-flow matrix of the backward travel time, whose
    # order is ascending head
    _say("tt_sweep 5 rhs + reversed flow, 33x17x9")
    p = gi.heterogeneous_aquifer(33, 17, 9, 4.0, 4, 7)
    g = p.grid
    h = _heads(ref, p)
    qx, qy, qz = ref.darcy_flux(p, h)
    rng = np.random.default_rng(3)
    for sign in (1.0, -1.0):
        At, bt, bc, _ = ref.tt_assemble(g, sign * qx, sign * qy, sign * qz, p.phi)
        rhs = [bt, bc] + [rng.standard_normal(g.n) for _ in range(3)]
        got, _ = _gpu_sweep(gw, At, rhs)
        for k, r in enumerate(rhs):
            want = ref.tt_sweep(At, r, sign * h)
            assert np.array_equal(got[k], want), (sign, k)


def test_sweep_cycle_and_bad_matrix(gw):
    _say("tt_sweep cycle / malformed")
    # cells 0 and 1 feed each other, cell 2 feeds 3: not an upwind matrix
    rowptr = np.array([0, 2, 4, 5, 7], np.int32)
    col = np.array([0, 1, 0, 1, 2, 2, 3], np.int32)
    val = np.array([2.0, -1.0, -1.0, 2.0, 4.0, -1.0, 3.0])
    b = dev(np.array([1.0, 1.0, 2.0, 1.0]))
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(gw.GwError) as e:
        gw.tt_sweep(4, dev(rowptr), dev(col), dev(val), b, x)
    assert e.value.status == gw.BREAKDOWN
    xs = host(x)
    assert xs[2] == 0.5 and xs[3] == (1.0 - (-1.0) * 0.5) / 3.0
    # missing diagonal in row 3
    col_bad = np.array([0, 1, 0, 1, 2, 1, 2], np.int32)
    with pytest.raises(gw.GwError) as e:
        gw.tt_sweep(4, dev(rowptr), dev(col_bad), dev(val), b, x)
    assert e.value.status == gw.EINVAL


def test_sweep_large_synthetic_heads(gw, ref):
    # the 8.4M-cell grid: heads = a west-to-east gradient plus a smooth
    # meander and seeded noise (any head field gives a valid upwind matrix
    # through Darcy's law); checked at every cell against the oracle
    _say("tt_sweep 256x256x128 synthetic heads")
    p = gi.heterogeneous_aquifer(256, 256, 128, 1.0, 8, 13)
    g = p.grid
    x = ((np.arange(g.nx) + 0.5) / g.nx)[None, None, :]
    y = ((np.arange(g.ny) + 0.5) / g.ny)[None, :, None]
    z = ((np.arange(g.nz) + 0.5) / g.nz)[:, None, None]
    h = 10.0 * (1.0 - x) + 0.4 * np.sin(6 * np.pi * y) * np.sin(np.pi * z) * np.sin(3 * np.pi * x)
    rng = np.random.default_rng(17)
    h = np.ascontiguousarray(h.reshape(-1)) + 1e-4 * rng.standard_normal(g.n)
    qx, qy, qz = ref.darcy_flux(p, h)
    At, bt, bc, _ = ref.tt_assemble(g, qx, qy, qz, p.phi, (0, g.ny, 0, g.nz // 2))
    want_t = ref.tt_sweep(At, bt, h)
    want_c = ref.tt_sweep(At, bc, h)
    tau = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    c = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    lev = gw.tt_solve_direct(g, dev(qx), dev(qy), dev(qz), p.phi, (0, g.ny, 0, g.nz // 2), tau, c)
    _say(f"  levels {lev}")
    assert np.array_equal(host(tau), want_t) and np.array_equal(host(c), want_c)
    # the general CSR sweep on the same system: its frontiers (up to 11k cells)
    # overflow the LDS queues into HBM
    got, lev2 = _gpu_sweep(gw, At, [bt, bc])
    assert lev2 == lev
    assert np.array_equal(got[0], want_t) and np.array_equal(got[1], want_c)


def _wells_problem():
    g = gi.Grid(24, 18, 6)
    K = gi.lognormal_field((24, 18, 6), 2.0, 4.0, 31)
    wells = [gi.Well(16, 5, 2, 2e-4), gi.Well(8, 12, 3, -1.5e-4), gi.Well(19, 13, 1, 1e-4),
             gi.Well(19, 13, 1, 5e-5), gi.Well(3, 3, 0, 0.0)]
    return gi.Problem(g, K, wells=wells)


DELINEATION_CASES = [
    ("24x18x6 zones + injection + 2 wells in one cell", _wells_problem,
     [(0, 9, 0, 6), (9, 18, 0, 3), (9, 18, 3, 6)]),
    ("32x24x12 lognormal, four pumping wells, no zones", lambda: gi.heterogeneous_aquifer(32, 24, 12, 4.0, 6, 4),
     []),
    ("2d 64x64 homogeneous, one zone", lambda: gi.homogeneous_slab(), [(0, 64, 0, 1)]),
]


@pytest.mark.parametrize("name,make,zones", DELINEATION_CASES, ids=[c[0] for c in DELINEATION_CASES])
def test_delineation_bitwise(gw, ref, name, make, zones):
    _say(f"tt_delineate {name}")
    p = make()
    g = p.grid
    h = _heads(ref, p)
    qx, qy, qz = ref.darcy_flux(p, h)
    d = ref.dual_delineation(g, qx, qy, qz, p.phi, h, zones, p.wells)
    nf, nb = gw.delineation_fields(zones, p.wells)
    assert (nf, nb) == (d.forward.shape[0], d.backward.shape[0])
    out = torch.full(((nf + nb) * g.n,), np.nan, dtype=torch.float64, device="cuda")
    lf, lb = gw.tt_delineate(g, dev(qx), dev(qy), dev(qz), p.phi, zones, p.wells, out)
    _say(f"  levels forward {lf} backward {lb}")
    got = host(out).reshape(nf + nb, g.n)
    for k in range(nf):
        assert np.array_equal(got[k], d.forward[k]), ("forward", k)
    for k in range(nb):
        assert np.array_equal(got[nf + k], d.backward[k]), ("backward", k)


def test_delineation_rejects_bad_input(gw):
    _say("tt_delineate bad input")
    g = gi.Grid(6, 5, 4)
    q = [torch.zeros(m, dtype=torch.float64, device="cuda") for m in (7 * 5 * 4, 6 * 6 * 4, 6 * 5 * 5)]
    out = torch.zeros(2 * g.n, dtype=torch.float64, device="cuda")
    with pytest.raises(gw.GwError) as e:
        gw.tt_delineate(g, *q, 0.25, [(0, 9, 0, 1)], [], torch.zeros(3 * g.n, dtype=torch.float64, device="cuda"))
    assert e.value.status == gw.EINVAL
    with pytest.raises(gw.GwError) as e:
        gw.tt_delineate(g, *q, 0.25, [], [gi.Well(6, 0, 0, 1.0)], torch.zeros(3 * g.n, dtype=torch.float64,
                                                                                 device="cuda"))
    assert e.value.status == gw.EINVAL
    # no flow at all: every row is an identity row, every field is zero
    gw.tt_delineate(g, *q, 0.25, [], [], out)
    assert not host(out).any()
