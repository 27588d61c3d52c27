"""The ILU(0) smoother (the paper's relaxation) on the GPU against the oracle.

Factors are bit-identical level by level (same IKJ order per entry, rows
scheduled by their dependencies); the V-cycle agrees within 1e-12 and the
PCG heads within 1e-8 at the oracle's iteration count.
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


def _setup(gw, ref, p, n_coarse):
    A, b = ref.fv_assemble(p)
    Hr = ref.Hierarchy(A, ref.AmgParams(smoother=ref.ILU0, n_coarse=n_coarse))
    Hg = gw.amg_setup(p.grid.n, dev(A.rowptr), dev(A.col), dev(A.val),
                      gw.AmgParams(smoother=gw.SMOOTHER_ILU0, n_coarse=n_coarse))
    return A, b, Hr, Hg


def test_ilu0_factors_bitwise(gw, ref):
    _say("ILU(0) factors 24x20x8 and 9x7x5")
    for p, nc in ((gi.heterogeneous_aquifer(24, 20, 8, 4.0, 4, 3), 40),
                  (gi.Problem(gi.Grid(9, 7, 5), gi.random_k(gi.Grid(9, 7, 5), 1), wells=[gi.Well(4, 3, 2, 1e-5)]), 20)):
        A, b, Hr, Hg = _setup(gw, ref, p, nc)
        assert Hg.nlevels == Hr.nlevels >= 2
        for l in range(Hr.nlevels - 1):
            want = Hr.level_ilu(l)
            got = torch.zeros(len(want), dtype=torch.float64, device="cuda")
            gw.amg_ilu_export(Hg, l, got)
            assert np.array_equal(host(got), want), l


def test_ilu0_vcycle_and_pcg(gw, ref):
    _say("ILU(0) V-cycle and PCG 30x22x14")
    p = gi.heterogeneous_aquifer(30, 22, 14, 4.0, 4, 6)
    A, b, Hr, Hg = _setup(gw, ref, p, 60)
    for seed in (1, 2):
        r = gi.random_vector(p.grid.n, seed)
        z_ref = Hr.vcycle(r)
        z = torch.zeros(p.grid.n, dtype=torch.float64, device="cuda")
        gw.amg_vcycle(Hg, dev(r), z)
        err = np.linalg.norm(host(z) - z_ref) / np.linalg.norm(z_ref)
        assert err < 1e-12, err
    h_ref, oinf = ref.pcg(Hr, b, rtol=1e-8)
    x = torch.zeros(p.grid.n, dtype=torch.float64, device="cuda")
    info = gw.amg_solve_pcg(Hg, dev(b), x, gw.SolveParams(rtol=1e-8))
    err = np.linalg.norm(host(x) - h_ref) / np.linalg.norm(h_ref)
    _say(f"  iters gpu {info.iters} oracle {oinf.iters} rel err {err:.2e}")
    assert info.status == gw.OK and abs(info.iters - oinf.iters) <= 1 and err <= 1e-8


def test_ilu0_travel_time_and_errors(gw, ref):
    _say("ILU(0) travel time pair and argument errors")
    import scipy.sparse.linalg as sla
    p = gi.heterogeneous_aquifer(20, 16, 8, 2.0, 4, 8)
    A, b = ref.fv_assemble(p)
    h = sla.spsolve(A.to_scipy().tocsc(), b)
    qx, qy, qz = ref.darcy_flux(p, h)
    zone = (0, 16, 0, 4)
    tr = ref.solve_travel_time(p.grid, qx, qy, qz, p.phi, ref.AmgParams(smoother=ref.ILU0, eps_strong=0.25),
                               rtol=1e-8, zone=zone)
    tau = torch.zeros(p.grid.n, dtype=torch.float64, device="cuda")
    c = torch.zeros(p.grid.n, dtype=torch.float64, device="cuda")
    st, infos = gw.tt_solve(p.grid, dev(qx), dev(qy), dev(qz), p.phi, zone,
                            gw.AmgParams(smoother=gw.SMOOTHER_ILU0, eps_strong=0.25), gw.SolveParams(rtol=1e-8),
                            tau, c)
    assert st == gw.OK
    for got, want in ((host(tau), tr.tau), (host(c), tr.c)):
        assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-8
    with pytest.raises(gw.GwError) as e:
        gw.amg_setup(p.grid.n, dev(A.rowptr), dev(A.col), dev(A.val),
                     gw.AmgParams(smoother=gw.SMOOTHER_ILU0, precision=gw.PRECISION_MIXED))
    assert e.value.status == gw.EINVAL
    Hg = gw.amg_setup(p.grid.n, dev(A.rowptr), dev(A.col), dev(A.val), gw.AmgParams())
    with pytest.raises(gw.GwError) as e:
        gw.amg_ilu_export(Hg, 0, torch.zeros(A.nnz, dtype=torch.float64, device="cuda"))
    assert e.value.status == gw.EINVAL
