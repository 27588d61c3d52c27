"""Ruge-Stueben coarsening on the GPU against the oracle.

Classical strength, the PMIS splitting and direct interpolation are integer
work plus a fixed-order formula per row, so every level (C/F split as coarse
indices, P, the Galerkin operators, the coarse LU) must match the oracle bit
for bit; PCG with that hierarchy then agrees within 1e-8 relative, as the
smoothed-aggregation solves do.
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


def _params(gw, ap):
    return gw.AmgParams(eps_strong=ap.eps_strong, smoother=ap.smoother, omega=ap.omega, npre=ap.npre,
                        npost=ap.npost, n_coarse=ap.n_coarse, max_levels=ap.max_levels, seed=ap.seed,
                        coarsening=gw.COARSEN_RS)


def _setup(gw, A, ap):
    return gw.amg_setup(A.n, dev(A.rowptr), dev(A.col), dev(A.val), _params(gw, ap))


def _compare(gw, ref, Hg, Hr, tag):
    infos, _ = Hg.info()
    assert Hg.nlevels == Hr.nlevels, (tag, Hg.nlevels, Hr.nlevels)
    for l in range(Hr.nlevels):
        R = Hr.level(l)
        li = infos[l]
        assert (li.n, li.nnz) == (R.A.n, R.A.nnz), f"{tag} level {l} size"
        ar = torch.zeros(li.n + 1, dtype=torch.int32, device="cuda")
        ac = torch.zeros(max(li.nnz, 1), dtype=torch.int32, device="cuda")
        av = torch.zeros(max(li.nnz, 1), dtype=torch.float64, device="cuda")
        if l == Hr.nlevels - 1:
            gw.amg_level_export(Hg, l, ar, ac, av)
        else:
            agg = torch.zeros(li.n, dtype=torch.int32, device="cuda")
            M = torch.zeros(li.n, dtype=torch.float64, device="cuda")
            pr = torch.zeros(li.n + 1, dtype=torch.int32, device="cuda")
            pc = torch.zeros(max(li.nnz_p, 1), dtype=torch.int32, device="cuda")
            pv = torch.zeros(max(li.nnz_p, 1), dtype=torch.float64, device="cuda")
            gw.amg_level_export(Hg, l, ar, ac, av, agg, M, pr, pc, pv)
            assert (li.nc, li.mis_rounds, li.nnz_s) == (R.nc, R.mis_rounds, R.nnz_s), f"{tag} level {l}"
            assert li.omega_p == 0.0 and R.omega_p == 0.0
            assert np.array_equal(host(agg), R.agg), f"{tag} C/F split level {l}"
            assert np.array_equal(host(pr), R.P.rowptr) and np.array_equal(host(pc)[:li.nnz_p], R.P.col)
            assert np.array_equal(host(pv)[:li.nnz_p].view(np.uint64), R.P.val.view(np.uint64)), f"{tag} P {l}"
            assert np.array_equal(host(M).view(np.uint64), R.M.view(np.uint64)), f"{tag} M {l}"
        assert np.array_equal(host(ar), R.A.rowptr), f"{tag} A rowptr level {l}"
        assert np.array_equal(host(ac)[:li.nnz], R.A.col), f"{tag} A col level {l}"
        assert np.array_equal(host(av)[:li.nnz].view(np.uint64), R.A.val.view(np.uint64)), f"{tag} A val {l}"
    lu_ref, piv_ref = Hr.coarse_lu()
    nd = lu_ref.shape[0]
    lu = torch.zeros(nd * nd, dtype=torch.float64, device="cuda")
    piv = torch.zeros(nd, dtype=torch.int32, device="cuda")
    gw.amg_coarse_export(Hg, lu, piv)
    assert np.array_equal(host(piv), piv_ref)
    assert np.array_equal(host(lu).view(np.uint64), lu_ref.reshape(-1).view(np.uint64)), f"{tag} coarse LU"


CASES = [
    ("2d 64x64 homogeneous", lambda: gi.homogeneous_slab(), dict()),
    ("3d 24x20x12 s2=4", lambda: gi.heterogeneous_aquifer(24, 20, 12, 4.0, 4, 5), dict()),
    ("3d 37x23x11 s2=1 ragged", lambda: gi.heterogeneous_aquifer(37, 23, 11, 1.0, 3, 8), dict(n_coarse=40)),
    ("3d 20x16x8 theta 0.5 jacobi", lambda: gi.heterogeneous_aquifer(20, 16, 8, 2.0, 4, 3),
     dict(eps_strong=0.5, smoother=0)),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_rs_hierarchy_bitwise(gw, ref, name, make, kw):
    _say(f"rs hierarchy {name}")
    kw = dict(dict(eps_strong=0.25), **kw)
    p = make()
    A, b = ref.fv_assemble(p)
    ap = ref.AmgParams(coarsening=ref.RS, **kw)
    Hr = ref.Hierarchy(A, ap)
    assert Hr.nlevels >= 2
    _compare(gw, ref, _setup(gw, A, ap), Hr, name)


def test_rs_travel_time_hierarchy_bitwise(gw, ref):
    # the upwind operator is not symmetric: S and S^T differ
    _say("rs hierarchy travel time 24x20x12")
    import scipy.sparse.linalg as sla
    p = gi.heterogeneous_aquifer(24, 20, 12, 4.0, 4, 5)
    A, b = ref.fv_assemble(p)
    h = sla.spsolve(A.to_scipy().tocsc(), b)
    qx, qy, qz = ref.darcy_flux(p, h)
    At, bt, bc, nid = ref.tt_assemble(p.grid, qx, qy, qz, 0.25, zone=(0, 20, 0, 6))
    ap = ref.AmgParams(coarsening=ref.RS, eps_strong=0.25, n_coarse=40)
    Hr = ref.Hierarchy(At, ap)
    _compare(gw, ref, _setup(gw, At, ap), Hr, "travel time")


def test_rs_pcg_parity(gw, ref):
    _say("rs pcg 40x32x16 s2=4 wells")
    p = gi.heterogeneous_aquifer(40, 32, 16, 4.0, 8, 11)
    A, b = ref.fv_assemble(p)
    ap = ref.AmgParams(coarsening=ref.RS, eps_strong=0.25)
    Hr = ref.Hierarchy(A, ap)
    want, oinf = ref.pcg(Hr, b, rtol=1e-8)
    Hg = _setup(gw, A, ap)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    info = gw.amg_solve_pcg(Hg, dev(b), x, gw.SolveParams(rtol=1e-8, check_every=3))
    err = np.linalg.norm(host(x) - want) / np.linalg.norm(want)
    _say(f"  iters gpu {info.iters} oracle {oinf.iters} err {err:.2e}")
    assert info.status == gw.OK and info.rel_res_true <= 1e-8
    assert abs(info.iters - oinf.iters) <= 1 and err <= 1e-8


def test_rs_full_size(gw, ref):
    # the 1M-cell aquifer: the C/F split and P of every level bit for bit,
    # heads within 1e-8 of the oracle's PCG with its own RS hierarchy
    _say("rs full-size 128x128x64")
    p = gi.heterogeneous_aquifer(128, 128, 64, 4.0, 8, 11)
    A, b = ref.fv_assemble(p)
    ap = ref.AmgParams(coarsening=ref.RS, eps_strong=0.25)
    Hr = ref.Hierarchy(A, ap)
    want, oinf = ref.pcg(Hr, b, rtol=1e-8)
    Hg = _setup(gw, A, ap)
    infos, _ = Hg.info()
    assert Hg.nlevels == Hr.nlevels
    for l in range(Hr.nlevels - 1):
        li = infos[l]
        agg = torch.zeros(li.n, dtype=torch.int32, device="cuda")
        pv = torch.zeros(max(li.nnz_p, 1), dtype=torch.float64, device="cuda")
        gw.amg_level_export(Hg, l, agg=agg, p_val=pv)
        assert np.array_equal(host(agg), Hr.level(l).agg), f"level {l}"
        assert np.array_equal(host(pv)[:li.nnz_p].view(np.uint64), Hr.level(l).P.val.view(np.uint64)), f"P {l}"
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    info = gw.amg_solve_pcg(Hg, dev(b), x, gw.SolveParams(rtol=1e-8))
    err = np.linalg.norm(host(x) - want) / np.linalg.norm(want)
    _say(f"  levels {Hg.nlevels} iters gpu {info.iters} oracle {oinf.iters} err {err:.2e}")
    assert info.status == gw.OK and info.rel_res_true <= 1e-8 and err <= 1e-8


def test_rs_with_ilu0(gw, ref):
    # the paper's relaxation on the RS hierarchy
    _say("rs + ilu0 24x20x12")
    p = gi.heterogeneous_aquifer(24, 20, 12, 4.0, 4, 5)
    A, b = ref.fv_assemble(p)
    ap = ref.AmgParams(coarsening=ref.RS, eps_strong=0.25, smoother=ref.ILU0, npre=1, npost=1)
    Hr = ref.Hierarchy(A, ap)
    want, oinf = ref.pcg(Hr, b, rtol=1e-10)
    Hg = _setup(gw, A, ap)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    info = gw.amg_solve_pcg(Hg, dev(b), x, gw.SolveParams(rtol=1e-10))
    err = np.linalg.norm(host(x) - want) / np.linalg.norm(want)
    _say(f"  iters gpu {info.iters} oracle {oinf.iters} err {err:.2e}")
    assert info.status == gw.OK and abs(info.iters - oinf.iters) <= 1 and err <= 1e-8


def test_rs_rejects_unknown_coarsening(gw, ref):
    p = gi.homogeneous_slab(16, 16)
    A, b = ref.fv_assemble(p)
    with pytest.raises(gw.GwError):
        gw.amg_setup(A.n, dev(A.rowptr), dev(A.col), dev(A.val), gw.AmgParams(coarsening=2))
