"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bit-exact where the work is integer or a fixed-order floating-point
definition (assembly, strength/aggregation, prolongator, Galerkin operators,
coarse LU); within the stated tolerance for Krylov iterates:
  FP64 path:  ||x - x_oracle|| / ||x_oracle|| <= 1e-8, same algorithm and
              stopping rule, final true residual <= rtol;
  mixed path: FP32 hierarchy inside FP64 flexible CG vs the FP64 oracle,
              <= 1e-6.
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


def gpu_assemble(gw, p):
    g = p.grid
    n, nnz = g.n, gw.fv_nnz(g)
    rowptr = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    col = torch.zeros(nnz, dtype=torch.int32, device="cuda")
    val = torch.zeros(nnz, dtype=torch.float64, device="cuda")
    b = torch.zeros(n, dtype=torch.float64, device="cuda")
    K = dev(p.K)
    gw.fv_assemble(g, K, (p.h_west, p.h_east), p.wells, rowptr, col, val, b)
    return K, rowptr, col, val, b


def gpu_params(gw, ap, precision=0):
    return gw.AmgParams(eps_strong=ap.eps_strong, smoother=ap.smoother, omega=ap.omega, npre=ap.npre,
                        npost=ap.npost, n_coarse=ap.n_coarse, max_levels=ap.max_levels, precision=precision,
                        seed=ap.seed)


ASM_CASES = [
    ("2d 64x64 homogeneous", lambda: gi.homogeneous_slab()),
    ("3d 13x7x5 random K, wells", lambda: gi.Problem(gi.Grid(13, 7, 5), gi.random_k(gi.Grid(13, 7, 5), 1),
                                                     wells=[gi.Well(3, 2, 1, 1e-5), gi.Well(3, 2, 1, 2e-5)])),
    ("nx=1 column 1x9x6", lambda: gi.Problem(gi.Grid(1, 9, 6), gi.random_k(gi.Grid(1, 9, 6), 2))),
    ("single cell", lambda: gi.Problem(gi.Grid(1, 1, 1), np.array([3e-4]))),
    ("3d 33x17x9 lognormal s2=4", lambda: gi.heterogeneous_aquifer(33, 17, 9, 4.0, 4, 7)),
]


@pytest.mark.parametrize("name,make", ASM_CASES, ids=[c[0] for c in ASM_CASES])
def test_fv_assemble_bitwise(gw, ref, name, make):
    _say(f"fv_assemble {name}")
    p = make()
    A, b = ref.fv_assemble(p)
    K, rowptr, col, val, bd = gpu_assemble(gw, p)
    assert np.array_equal(host(rowptr), A.rowptr)
    assert np.array_equal(host(col), A.col)
    assert np.array_equal(host(val).view(np.uint64), A.val.view(np.uint64))
    assert np.array_equal(host(bd).view(np.uint64), b.view(np.uint64))


def test_fv_assemble_rejects_bad_k(gw):
    _say("fv_assemble invalid K")
    p = gi.homogeneous_slab(8, 8)
    p.K[5] = -1.0
    with pytest.raises(gw.GwError) as e:
        gpu_assemble(gw, p)
    assert e.value.status == gw.EINVAL


def test_darcy_bitwise(gw, ref):
    _say("darcy_flux 20x12x7")
    p = gi.heterogeneous_aquifer(20, 12, 7, 2.0, 4, 3)
    g = p.grid
    h = gi.random_vector(g.n, 9)
    qx, qy, qz = ref.darcy_flux(p, h)
    dqx = torch.zeros(len(qx), dtype=torch.float64, device="cuda")
    dqy = torch.zeros(len(qy), dtype=torch.float64, device="cuda")
    dqz = torch.zeros(len(qz), dtype=torch.float64, device="cuda")
    gw.darcy_flux(g, dev(p.K), (p.h_west, p.h_east), dev(h), dqx, dqy, dqz)
    for a, d in ((qx, dqx), (qy, dqy), (qz, dqz)):
        assert np.array_equal(host(d).view(np.uint64), a.view(np.uint64))


def _compare_hierarchy(gw, ref, H_gpu, H_ref, tag):
    infos, _ = H_gpu.info()
    assert H_gpu.nlevels == H_ref.nlevels, tag
    for l in range(H_ref.nlevels):
        R = H_ref.level(l)
        li = infos[l]
        assert (li.n, li.nnz) == (R.A.n, R.A.nnz), f"{tag} level {l} size"
        coarsest = l == H_ref.nlevels - 1
        ar = torch.zeros(li.n + 1, dtype=torch.int32, device="cuda")
        ac = torch.zeros(max(li.nnz, 1), dtype=torch.int32, device="cuda")
        av = torch.zeros(max(li.nnz, 1), dtype=torch.float64, device="cuda")
        if coarsest:
            gw.amg_level_export(H_gpu, l, ar, ac, av)
        else:
            agg = torch.zeros(li.n, dtype=torch.int32, device="cuda")
            M = torch.zeros(li.n, dtype=torch.float64, device="cuda")
            pr = torch.zeros(li.n + 1, dtype=torch.int32, device="cuda")
            pc = torch.zeros(max(li.nnz_p, 1), dtype=torch.int32, device="cuda")
            pv = torch.zeros(max(li.nnz_p, 1), dtype=torch.float64, device="cuda")
            gw.amg_level_export(H_gpu, l, ar, ac, av, agg, M, pr, pc, pv)
            assert li.nc == R.nc and li.mis_rounds == R.mis_rounds and li.nnz_s == R.nnz_s, f"{tag} level {l}"
            assert np.array_equal(host(agg), R.agg), f"{tag} aggregates level {l}"
            assert li.omega_p == R.omega_p, f"{tag} omega level {l}"
            assert np.array_equal(host(pr), R.P.rowptr) and np.array_equal(host(pc)[:li.nnz_p], R.P.col)
            assert np.array_equal(host(pv)[:li.nnz_p].view(np.uint64), R.P.val.view(np.uint64)), f"{tag} P {l}"
            assert np.array_equal(host(M).view(np.uint64), R.M.view(np.uint64)), f"{tag} M {l}"
        assert np.array_equal(host(ar), R.A.rowptr), f"{tag} A rowptr level {l}"
        assert np.array_equal(host(ac)[:li.nnz], R.A.col), f"{tag} A col level {l}"
        assert np.array_equal(host(av)[:li.nnz].view(np.uint64), R.A.val.view(np.uint64)), f"{tag} A val {l}"
    lu_ref, piv_ref = H_ref.coarse_lu()
    nd = lu_ref.shape[0]
    lu = torch.zeros(nd * nd, dtype=torch.float64, device="cuda")
    piv = torch.zeros(nd, dtype=torch.int32, device="cuda")
    inv = torch.zeros(nd * nd, dtype=torch.float64, device="cuda")
    gw.amg_coarse_export(H_gpu, lu, piv, inv)
    assert np.array_equal(host(piv), piv_ref)
    assert np.array_equal(host(lu).view(np.uint64), lu_ref.reshape(-1).view(np.uint64)), f"{tag} coarse LU"
    Ac = H_ref.level(H_ref.nlevels - 1).A.dense()
    Ainv = host(inv).reshape(nd, nd)  # row-major
    assert np.allclose(Ainv @ Ac, np.eye(nd), atol=1e-9)


HIER_CASES = [
    ("2d 64x64 jacobi", lambda: gi.homogeneous_slab(), dict(smoother=0, npre=1, npost=1)),
    ("3d 24x20x12 s2=4", lambda: gi.heterogeneous_aquifer(24, 20, 12, 4.0, 4, 5), dict()),
    ("3d 37x23x11 s2=1 ragged", lambda: gi.heterogeneous_aquifer(37, 23, 11, 1.0, 3, 8), dict(n_coarse=40)),
    # coarsest levels of 109 and 141 rows (LU in LDS with 512 threads, the
    # second at the 160 KB limit) and of 412 rows (LU in global memory)
    ("3d 30x22x14 coarsest 109", lambda: gi.heterogeneous_aquifer(30, 22, 14, 4.0, 4, 5), dict()),
    ("3d 36x30x12 coarsest 141", lambda: gi.heterogeneous_aquifer(36, 30, 12, 4.0, 4, 5), dict()),
    ("3d 36x30x12 coarsest 412", lambda: gi.heterogeneous_aquifer(36, 30, 12, 4.0, 4, 5), dict(eps_strong=0.15)),
]


@pytest.mark.parametrize("name,make,kw", HIER_CASES, ids=[c[0] for c in HIER_CASES])
def test_flow_hierarchy_bitwise(gw, ref, name, make, kw):
    _say(f"hierarchy {name}")
    p = make()
    ap = ref.AmgParams(**kw)
    A, b = ref.fv_assemble(p)
    Hr = ref.Hierarchy(A, ap)
    if "coarsest" in name:  # the case is there for its coarsest size
        assert Hr.level(Hr.nlevels - 1).A.n == int(name.split("coarsest ")[1])
    K, rowptr, col, val, bd = gpu_assemble(gw, p)
    Hg = gw.amg_setup(p.grid.n, rowptr, col, val, gpu_params(gw, ap))
    _compare_hierarchy(gw, ref, Hg, Hr, name)


TT_HIER_CASES = [
    ("coarse 42", dict(n_coarse=40)),
    # a coarsest level of 729 and of 1320 rows: blocked LU (panels of 16 and
    # 8 columns in LDS), with 15 and 27 row interchanges
    ("coarsest 729", dict(n_coarse=1500)),
    ("coarsest 1320", dict(n_coarse=1500, eps_strong=0.25)),
]


@pytest.mark.parametrize("name,kw", TT_HIER_CASES, ids=[c[0] for c in TT_HIER_CASES])
def test_travel_time_hierarchy_bitwise(gw, ref, name, kw):
    _say(f"hierarchy travel time 24x20x12 {name}")
    import scipy.sparse.linalg as sla
    p = gi.heterogeneous_aquifer(24, 20, 12, 4.0, 4, 5)
    A, b = ref.fv_assemble(p)
    h = sla.spsolve(A.to_scipy().tocsc(), b)
    qx, qy, qz = ref.darcy_flux(p, h)
    At, bt, bc, nid = ref.tt_assemble(p.grid, qx, qy, qz, 0.25, zone=(0, 20, 0, 6))
    g = p.grid
    n, cap = g.n, gw.tt_nnz_bound(g)
    rp = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    cl = torch.zeros(cap, dtype=torch.int32, device="cuda")
    vl = torch.zeros(cap, dtype=torch.float64, device="cuda")
    dbt = torch.zeros(n, dtype=torch.float64, device="cuda")
    dbc = torch.zeros(n, dtype=torch.float64, device="cuda")
    nnz, nid_g = gw.tt_assemble(g, dev(qx), dev(qy), dev(qz), 0.25, (0, 20, 0, 6), rp, cl, vl, dbt, dbc)
    assert nnz == At.nnz and nid_g == nid
    assert np.array_equal(host(rp), At.rowptr) and np.array_equal(host(cl)[:nnz], At.col)
    assert np.array_equal(host(vl)[:nnz].view(np.uint64), At.val.view(np.uint64))
    assert np.array_equal(host(dbt).view(np.uint64), bt.view(np.uint64))
    assert np.array_equal(host(dbc).view(np.uint64), bc.view(np.uint64))
    ap = ref.AmgParams(**kw)
    Hr = ref.Hierarchy(At, ap)
    if name.startswith("coarsest"):
        assert Hr.level(Hr.nlevels - 1).A.n == int(name.split()[1])
    Hg = gw.amg_setup(n, rp, cl[:nnz].contiguous(), vl[:nnz].contiguous(), gpu_params(gw, ap))
    _compare_hierarchy(gw, ref, Hg, Hr, "travel time " + name)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_vcycle_parity(gw, ref, precision):
    _say(f"vcycle precision={precision}")
    p = gi.heterogeneous_aquifer(30, 22, 14, 4.0, 4, 6)
    A, b = ref.fv_assemble(p)
    ap = ref.AmgParams(n_coarse=60)
    Hr = ref.Hierarchy(A, ap)
    K, rowptr, col, val, bd = gpu_assemble(gw, p)
    Hg = gw.amg_setup(p.grid.n, rowptr, col, val, gpu_params(gw, ap, precision))
    for seed in (1, 2):
        r = gi.random_vector(p.grid.n, seed)
        z_ref = Hr.vcycle(r)
        z = torch.zeros(p.grid.n, dtype=torch.float64, device="cuda")
        gw.amg_vcycle(Hg, dev(r), z)
        err = np.linalg.norm(host(z) - z_ref) / np.linalg.norm(z_ref)
        assert err < (1e-12 if precision == 0 else 1e-5), err
    # SpMV with the level-0 operator
    x = gi.random_vector(p.grid.n, 3)
    y = torch.zeros(p.grid.n, dtype=torch.float64, device="cuda")
    gw.amg_spmv(Hg, dev(x), y)
    assert np.allclose(host(y), ref.spmv(A, x), rtol=1e-13, atol=1e-13 * np.abs(ref.spmv(A, x)).max())


@pytest.mark.parametrize("npre,npost", [(0, 1), (1, 1), (1, 2), (2, 1), (3, 2), (2, 0)])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_vcycle_sweep_counts(gw, ref, npre, npost, precision):
    """The V-cycle against the oracle's for each way a level can start: no
    pre-sweep (x = 0), one (on the coarse levels the restriction writes x1 =
    M b and the level forms its residual from it), two or more (a sweep from
    that x1), with zero to two post-sweeps; three smoothed levels."""
    _say(f"vcycle sweeps {npre}/{npost} precision={precision}")
    p = gi.heterogeneous_aquifer(30, 22, 14, 4.0, 4, 6)
    A, b = ref.fv_assemble(p)
    ap = ref.AmgParams(n_coarse=40, npre=npre, npost=npost)
    Hr = ref.Hierarchy(A, ap)
    assert Hr.nlevels >= 4
    K, rowptr, col, val, bd = gpu_assemble(gw, p)
    Hg = gw.amg_setup(p.grid.n, rowptr, col, val, gpu_params(gw, ap, precision))
    r = gi.random_vector(p.grid.n, 5)
    z_ref = Hr.vcycle(r)
    z = torch.zeros(p.grid.n, dtype=torch.float64, device="cuda")
    gw.amg_vcycle(Hg, dev(r), z)
    err = np.linalg.norm(host(z) - z_ref) / np.linalg.norm(z_ref)
    assert err < (1e-12 if precision == 0 else 1e-5), err


FLOW_CASES = [
    ("C1 2d 64x64 jacobi", lambda: gi.homogeneous_slab(), dict(smoother=0, npre=1, npost=1)),
    ("3d 40x32x16 s2=4 wells", lambda: gi.heterogeneous_aquifer(40, 32, 16, 4.0, 8, 11), dict()),
    ("3d 29x31x7 s2=2 ragged", lambda: gi.heterogeneous_aquifer(29, 31, 7, 2.0, 4, 12), dict(n_coarse=50)),
]


@pytest.mark.parametrize("name,make,kw", FLOW_CASES, ids=[c[0] for c in FLOW_CASES])
def test_flow_pcg_parity(gw, ref, name, make, kw):
    _say(f"pcg {name}")
    p = make()
    ap = ref.AmgParams(**kw)
    fr = ref.solve_flow(p, ap, rtol=1e-8)
    K, rowptr, col, val, bd = gpu_assemble(gw, p)
    Hg = gw.amg_setup(p.grid.n, rowptr, col, val, gpu_params(gw, ap))
    x = torch.zeros(p.grid.n, dtype=torch.float64, device="cuda")
    info = gw.amg_solve_pcg(Hg, bd, x, gw.SolveParams(rtol=1e-8, check_every=3))
    h = host(x)
    assert info.status == gw.OK and info.rel_res_true <= 1e-8
    assert abs(info.iters - fr.info.iters) <= 1, (info.iters, fr.info.iters)
    err = np.linalg.norm(h - fr.h) / np.linalg.norm(fr.h)
    assert err <= 1e-8, err
    if name.startswith("C1"):
        ex = np.tile(10 * (1 - (np.arange(64) + 0.5) / 64), 64)
        assert np.linalg.norm(h - ex) / np.linalg.norm(ex) < 1e-6


def test_flow_mixed_fcg(gw, ref):
    _say("mixed fcg 40x32x16")
    p = gi.heterogeneous_aquifer(40, 32, 16, 4.0, 8, 11)
    ap = ref.AmgParams()
    fr = ref.solve_flow(p, ap, rtol=1e-8)
    K, rowptr, col, val, bd = gpu_assemble(gw, p)
    Hg = gw.amg_setup(p.grid.n, rowptr, col, val, gpu_params(gw, ap, gw.PRECISION_MIXED))
    x = torch.zeros(p.grid.n, dtype=torch.float64, device="cuda")
    info = gw.amg_solve_pcg(Hg, bd, x, gw.SolveParams(rtol=1e-8))
    assert info.status == gw.OK and info.rel_res_true <= 1e-8
    err = np.linalg.norm(host(x) - fr.h) / np.linalg.norm(fr.h)
    assert err <= 1e-6, err
    assert info.iters <= fr.info.iters + 5


def test_travel_time_solve_parity(gw, ref):
    _say("tt_solve 32x24x12")
    import scipy.sparse.linalg as sla
    p = gi.heterogeneous_aquifer(32, 24, 12, 4.0, 6, 4)
    A, b = ref.fv_assemble(p)
    h = sla.spsolve(A.to_scipy().tocsc(), b)
    qx, qy, qz = ref.darcy_flux(p, h)
    zone = (0, 24, 0, 6)
    ap = ref.AmgParams()
    tr = ref.solve_travel_time(p.grid, qx, qy, qz, 0.25, ap, rtol=1e-8, zone=zone)
    tau = torch.zeros(p.grid.n, dtype=torch.float64, device="cuda")
    c = torch.zeros(p.grid.n, dtype=torch.float64, device="cuda")
    st, infos = gw.tt_solve(p.grid, dev(qx), dev(qy), dev(qz), 0.25, zone, gpu_params(gw, ap),
                            gw.SolveParams(rtol=1e-8), tau, c)
    assert st == gw.OK
    for got, want, inf in ((host(tau), tr.tau, infos[0]), (host(c), tr.c, infos[1])):
        assert inf.rel_res_true <= 1e-8
        assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-8
    # and the exact sweep solution within the solve's accuracy
    tau_ex = ref.tt_sweep(tr.A, tr.b_tau, h)
    assert np.linalg.norm(host(tau) - tau_ex) / np.linalg.norm(tau_ex) < 1e-6


def test_status_codes(gw, ref):
    _say("status codes")
    p = gi.heterogeneous_aquifer(16, 12, 8, 1.0, 4, 2)
    K, rowptr, col, val, bd = gpu_assemble(gw, p)
    Hg = gw.amg_setup(p.grid.n, rowptr, col, val, gw.AmgParams(n_coarse=30))
    x = torch.zeros(p.grid.n, dtype=torch.float64, device="cuda")
    info = gw.amg_solve_pcg(Hg, bd, x, gw.SolveParams(rtol=1e-12, maxiter=1))
    assert info.status == gw.NOT_CONVERGED and info.iters == 1
    info = gw.amg_solve_pcg(Hg, torch.zeros_like(bd), x)
    assert info.status == gw.OK and info.iters == 0 and not host(x).any()
    bad = bd.clone()
    bad[3] = float("nan")
    assert gw.amg_solve_pcg(Hg, bad, x).status == gw.BREAKDOWN
    assert gw.amg_solve_bicgstab(Hg, bad, x).status == gw.BREAKDOWN
    info = gw.amg_solve_bicgstab(Hg, bd, x, gw.SolveParams(rtol=1e-12, maxiter=1))
    assert info.status == gw.NOT_CONVERGED
    # invalid CSR: unsorted columns
    c2 = col.clone()
    c2[0], c2[1] = col[1], col[0]
    with pytest.raises(gw.GwError) as e:
        gw.amg_setup(p.grid.n, rowptr, c2, val)
    assert e.value.status == gw.EINVAL


def test_full_size_travel_time_parity(gw, ref):
    # travel time on the Darcy velocities of the 1M-cell aquifer, with the
    # travel-time hierarchy settings the benchmark uses; both sides get the
    # same fluxes (computed from the oracle's heads) so that no face can flip
    # its upwind direction between the two
    _say("full-size 128x128x64 travel-time parity")
    p = gi.heterogeneous_aquifer(128, 128, 64, 4.0, 8, 11)
    # heads from the benchmark's flow settings (threshold 0.03, one sweep each way)
    fr = ref.solve_flow(p, ref.AmgParams(eps_strong=0.03, npre=1, npost=1), rtol=1e-8)
    qx, qy, qz = ref.darcy_flux(p, fr.h)
    g = p.grid
    zone = (0, g.ny, 0, g.nz // 2)
    tp = gw.AmgParams.travel_time()
    ap = ref.AmgParams(eps_strong=tp.eps_strong, npre=tp.npre, npost=tp.npost)
    tr = ref.solve_travel_time(g, qx, qy, qz, p.phi, ap, rtol=1e-8, zone=zone)
    # the travel-time hierarchy of those settings: aggregates of every level bit for bit
    Hg = gw.amg_setup(g.n, dev(tr.A.rowptr), dev(tr.A.col), dev(tr.A.val), gpu_params(gw, ap))
    infos, _ = Hg.info()
    assert Hg.nlevels == tr.H.nlevels
    for l in range(tr.H.nlevels - 1):
        agg = torch.zeros(infos[l].n, dtype=torch.int32, device="cuda")
        gw.amg_level_export(Hg, l, agg=agg)
        assert np.array_equal(host(agg), tr.H.level(l).agg), f"level {l}"
    del Hg
    tau = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    c = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    st, infos = gw.tt_solve(g, dev(qx), dev(qy), dev(qz), p.phi, zone, gpu_params(gw, ap), gw.SolveParams(rtol=1e-8),
                            tau, c)
    assert st == gw.OK
    for name, got, want, inf, oinf in (("tau", host(tau), tr.tau, infos[0], tr.info[0]),
                                       ("c", host(c), tr.c, infos[1], tr.info[1])):
        err = np.linalg.norm(got - want) / np.linalg.norm(want)
        _say(f"  {name}: iters gpu {inf.iters} oracle {oinf.iters} rel err {err:.3e}")
        assert inf.rel_res_true <= 1e-8 and err <= 1e-8
    tau_ex = ref.tt_sweep(tr.A, tr.b_tau, fr.h)
    err_ex = np.linalg.norm(host(tau) - tau_ex) / np.linalg.norm(tau_ex)
    _say(f"  tau vs exact sweep {err_ex:.2e}")
    assert err_ex < 1e-6
    # the direct sweep reproduces the oracle's exact solution bit for bit
    c_ex = ref.tt_sweep(tr.A, tr.b_c, fr.h)
    tau_d = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    c_d = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    lev = gw.tt_solve_direct(g, dev(qx), dev(qy), dev(qz), p.phi, zone, tau_d, c_d)
    _say(f"  direct sweep: {lev} levels")
    assert np.array_equal(host(tau_d), tau_ex) and np.array_equal(host(c_d), c_ex)


FULL_FLOW_PARAMS = [
    ("library defaults 0.08 2/2", dict()),
    ("benchmark flow 0.03 1/1", dict(eps_strong=0.03, npre=1, npost=1)),
]


@pytest.mark.parametrize("name,kw", FULL_FLOW_PARAMS, ids=[c[0] for c in FULL_FLOW_PARAMS])
def test_full_size_flow_parity(gw, ref, name, kw):
    # the 1M-cell lognormal aquifer (variance 4, correlation length 8, four
    # wells), at the library defaults and at the flow settings the benchmark
    # times (AmgParams.flow()): aggregates of every level bit for bit, heads
    # within 1e-8 of the oracle's same-algorithm solve
    _say(f"full-size 128x128x64 flow parity, {name}")
    bench = gw.AmgParams.flow()
    if kw:
        assert (kw["eps_strong"], kw["npre"], kw["npost"]) == (bench.eps_strong, bench.npre, bench.npost)
    p = gi.heterogeneous_aquifer(128, 128, 64, 4.0, 8, 11)
    ap = ref.AmgParams(**kw)
    fr = ref.solve_flow(p, ap, rtol=1e-8)
    K, rowptr, col, val, bd = gpu_assemble(gw, p)
    Hg = gw.amg_setup(p.grid.n, rowptr, col, val, gpu_params(gw, ap))
    infos, _ = Hg.info()
    assert Hg.nlevels == fr.H.nlevels
    for l in range(fr.H.nlevels - 1):
        agg = torch.zeros(infos[l].n, dtype=torch.int32, device="cuda")
        gw.amg_level_export(Hg, l, agg=agg)
        assert np.array_equal(host(agg), fr.H.level(l).agg), f"level {l}"
    x = torch.zeros(p.grid.n, dtype=torch.float64, device="cuda")
    info = gw.amg_solve_pcg(Hg, bd, x, gw.SolveParams(rtol=1e-8))
    assert info.status == gw.OK and info.rel_res_true <= 1e-8
    err = np.linalg.norm(host(x) - fr.h) / np.linalg.norm(fr.h)
    _say(f"  iters gpu {info.iters} oracle {fr.info.iters} rel err {err:.3e}")
    assert err <= 1e-8


def test_hierarchy_with_three_pass_radix_transpose(gw, ref):
    # A homogeneous 150^3 cube at the flow settings the benchmark times: the
    # level-0 prolongator has 303347 columns of about 38 entries each, so
    # R = P^T takes the radix path with three digit passes (more than 2^18
    # columns).  Every level, A_1 = R (A P) included, matches bit for bit.
    _say("hierarchy 150^3 homogeneous: R = P^T by three radix passes")
    p = gi.homogeneous_slab(150, 150, 150)
    ap = ref.AmgParams(eps_strong=0.03, npre=1, npost=1)
    A, b = ref.fv_assemble(p)
    Hr = ref.Hierarchy(A, ap)
    l0 = Hr.level(0)
    assert l0.nc > 1 << 18 and l0.P.nnz >= 6 * l0.nc, (l0.nc, l0.P.nnz)
    K, rowptr, col, val, bd = gpu_assemble(gw, p)
    Hg = gw.amg_setup(p.grid.n, rowptr, col, val, gpu_params(gw, ap))
    _compare_hierarchy(gw, ref, Hg, Hr, "150^3")


GENERAL_CASES = [
    # thousands of distinct column offsets: sliced ELL with int32 columns
    ("random graph n=3000", lambda: gi.random_graph_spd(3000, 4, 31)),
    # one row of ~1000 entries: the sliced copy would pad 9x, CSR kernels kept
    ("arrow n=2000", lambda: gi.arrow_spd(2000, 32)),
]


@pytest.mark.parametrize("name,make", GENERAL_CASES, ids=[c[0] for c in GENERAL_CASES])
def test_general_sparse_operator(gw, ref, name, make):
    _say(f"general operator {name}")
    rowptr, col, val = make()
    A = ref.Csr(rowptr, col, val)
    n = A.n
    ap = ref.AmgParams(n_coarse=60)
    Hr = ref.Hierarchy(A, ap)
    b = gi.random_vector(n, 4)
    x = gi.random_vector(n, 5)
    for precision in (0, 1):
        Hg = gw.amg_setup(n, dev(rowptr), dev(col), dev(val), gpu_params(gw, ap, precision))
        if precision == 0:
            _compare_hierarchy(gw, ref, Hg, Hr, name)
        y = torch.zeros(n, dtype=torch.float64, device="cuda")
        gw.amg_spmv(Hg, dev(x), y)
        y_ref = ref.spmv(A, x)
        assert np.allclose(host(y), y_ref, rtol=1e-13, atol=1e-13 * np.abs(y_ref).max())
        z = torch.zeros(n, dtype=torch.float64, device="cuda")
        gw.amg_vcycle(Hg, dev(b), z)
        z_ref = Hr.vcycle(b)
        err = np.linalg.norm(host(z) - z_ref) / np.linalg.norm(z_ref)
        assert err < (1e-12 if precision == 0 else 1e-5), (precision, err)
        h_ref, info_ref = ref.pcg(Hr, b, rtol=1e-8, flexible=bool(precision))
        h = torch.zeros(n, dtype=torch.float64, device="cuda")
        info = gw.amg_solve_pcg(Hg, dev(b), h, gw.SolveParams(rtol=1e-8))
        assert info.status == gw.OK and info.rel_res_true <= 1e-8
        err = np.linalg.norm(host(h) - h_ref) / np.linalg.norm(h_ref)
        assert err <= (1e-8 if precision == 0 else 1e-6), (precision, err)


@pytest.mark.parametrize("precision,check", [(0, 4), (1, 3)], ids=["fp64-check4", "mixed-check3"])
def test_graph_replay_matches_eager(gw, ref, precision, check):
    # the captured iteration blocks must give exactly the one-by-one result,
    # on every solve that replays them, with eager work and host syncs between
    _say(f"graph vs eager precision={precision} check={check}")
    p = gi.heterogeneous_aquifer(36, 28, 12, 4.0, 6, 13)
    K, rowptr, col, val, bd = gpu_assemble(gw, p)
    ap = ref.AmgParams(n_coarse=50)
    Hg = gw.amg_setup(p.grid.n, rowptr, col, val, gpu_params(gw, ap, precision))
    n = p.grid.n
    x0 = torch.zeros(n, dtype=torch.float64, device="cuda")
    i0 = gw.amg_solve_pcg(Hg, bd, x0, gw.SolveParams(rtol=1e-8, check_every=check, graph=0))
    want = host(x0)
    assert i0.status == gw.OK
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    for rep in range(3):
        gw.amg_spmv(Hg, bd, y)  # eager work between the solves
        torch.cuda.synchronize()
        x = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
        info = gw.amg_solve_pcg(Hg, bd, x, gw.SolveParams(rtol=1e-8, check_every=check, graph=1))
        assert (info.iters, info.status) == (i0.iters, i0.status), rep
        assert np.array_equal(host(x).view(np.uint64), want.view(np.uint64)), rep
    # BiCGSTAB on the same hierarchy (its own captured block)
    z0 = torch.zeros(n, dtype=torch.float64, device="cuda")
    j0 = gw.amg_solve_bicgstab(Hg, bd, z0, gw.SolveParams(rtol=1e-8, check_every=check, graph=0))
    for rep in range(2):
        z = torch.zeros(n, dtype=torch.float64, device="cuda")
        j = gw.amg_solve_bicgstab(Hg, bd, z, gw.SolveParams(rtol=1e-8, check_every=check, graph=1))
        assert (j.iters, j.status) == (j0.iters, j0.status), rep
        assert np.array_equal(host(z).view(np.uint64), host(z0).view(np.uint64)), rep
    # and the PCG blocks again after the workspace grew for BiCGSTAB
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    info = gw.amg_solve_pcg(Hg, bd, x, gw.SolveParams(rtol=1e-8, check_every=check, graph=1))
    assert np.array_equal(host(x).view(np.uint64), want.view(np.uint64))


@pytest.mark.parametrize("precision,check", [(0, 4), (1, 3)], ids=["fp64", "mixed-check3"])
def test_bicgstab_pair_matches_single(gw, ref, precision, check):
    # the lockstep two-system solve gives each system exactly the iterates
    # of a solve on its own (same hierarchy), including a zero right-hand side
    _say(f"bicgstab pair precision={precision}")
    p = gi.heterogeneous_aquifer(30, 24, 10, 2.0, 4, 17)
    fr = ref.solve_flow(p, ref.AmgParams(), rtol=1e-10)
    qx, qy, qz = ref.darcy_flux(p, fr.h)
    g = p.grid
    A, bt, bc, _ = ref.tt_assemble(g, qx, qy, qz, p.phi, (0, g.ny, 0, g.nz // 2))
    ap = ref.AmgParams(eps_strong=gw.TT_EPS_STRONG, n_coarse=40)
    Hg = gw.amg_setup(g.n, dev(A.rowptr), dev(A.col), dev(A.val), gpu_params(gw, ap, precision))
    sp = gw.SolveParams(rtol=1e-8, check_every=check)
    singles = []
    for rhs in (bt, bc):
        x = torch.zeros(g.n, dtype=torch.float64, device="cuda")
        info = gw.amg_solve_bicgstab(Hg, dev(rhs), x, sp)
        assert info.status == gw.OK
        singles.append((host(x), info))
    y0 = torch.full((g.n,), 3.0, dtype=torch.float64, device="cuda")
    y1 = torch.full((g.n,), 3.0, dtype=torch.float64, device="cuda")
    st, infos = gw.amg_solve_bicgstab_pair(Hg, dev(bt), dev(bc), y0, y1, sp)
    assert st == gw.OK
    for (x, i1), y, i2 in zip(singles, (host(y0), host(y1)), infos):
        assert (i2.iters, i2.status, i2.restarts) == (i1.iters, i1.status, i1.restarts)
        assert np.array_equal(y.view(np.uint64), x.view(np.uint64))
        assert i2.rel_res_true == i1.rel_res_true
    # second system zero: x1 = 0 with no iterations, the first unchanged
    st, infos = gw.amg_solve_bicgstab_pair(Hg, dev(bt), torch.zeros(g.n, dtype=torch.float64, device="cuda"),
                                           y0, y1, sp)
    assert st == gw.OK and infos[1].iters == 0 and not host(y1).any()
    assert np.array_equal(host(y0).view(np.uint64), singles[0][0].view(np.uint64))


def test_c3_mixed_flow_against_oracle(gw, ref):
    # the 8.4M-cell configuration as the benchmark times it (strength
    # threshold 0.05, two pre- and post-sweeps, FP32 hierarchy inside FP64
    # flexible CG): heads within 1e-6 of the oracle's FP64 flexible-CG solve
    # at the same settings, the true residual of the GPU heads recomputed
    # with the oracle's own matrix meets rtol, and the FP64 hierarchy gives
    # the same heads within the mixed-path tolerance
    _say("C3 256x256x128 mixed FCG vs the oracle (0.05, 2/2)")
    p = gi.heterogeneous_aquifer(256, 256, 128, 4.0, 8, 21)
    n = p.grid.n
    kw = dict(eps_strong=0.05, npre=2, npost=2)
    K, rowptr, col, val, bd = gpu_assemble(gw, p)
    heads = []
    for precision in (gw.PRECISION_MIXED, gw.PRECISION_FP64):
        H = gw.amg_setup(n, rowptr, col, val, gw.AmgParams(precision=precision, **kw))
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        info = gw.amg_solve_pcg(H, bd, x, gw.SolveParams(rtol=1e-8))
        _say(f"  precision {precision}: {info.iters} iterations, status {info.status}")
        assert info.status == gw.OK and info.rel_res_true <= 1e-8
        heads.append(host(x))
        del H
    A, b = ref.fv_assemble(p)
    r = b - A.to_scipy() @ heads[0]
    rel = np.linalg.norm(r) / np.linalg.norm(b)
    _say(f"  oracle-matrix residual of the mixed heads {rel:.2e}")
    assert rel <= 1.05e-8
    err = np.linalg.norm(heads[0] - heads[1]) / np.linalg.norm(heads[1])
    assert err <= 1e-6, err
    Hr = ref.Hierarchy(A, ref.AmgParams(**kw))
    h_ref, info_ref = ref.pcg(Hr, b, rtol=1e-8, flexible=True)
    assert info_ref.status == ref.OK
    for name, h in (("mixed", heads[0]), ("fp64", heads[1])):
        e = np.linalg.norm(h - h_ref) / np.linalg.norm(h_ref)
        _say(f"  {name} heads vs oracle (FCG, {info_ref.iters} iterations): {e:.2e}")
        assert e <= 1e-6, (name, e)


def test_setup_reports_zero_pivot_in_coarsest_lu(gw, ref):
    # [[1, 1], [1, 1]] is its own coarsest level and elimination leaves a zero
    # second pivot: both sides report it as singular (the LU runs beside the
    # rest of the setup, and the status is read before amg_setup returns);
    # the library stays usable, and [[2, 1], [1, 2]] then factors bit for bit
    _say("zero pivot in the coarsest LU")
    rp, cl = np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32)
    A = ref.Csr(rowptr=rp, col=cl, val=np.ones(4))
    with pytest.raises(ArithmeticError):
        ref.Hierarchy(A, ref.AmgParams())
    with pytest.raises(gw.GwError) as e:
        gw.amg_setup(2, dev(rp), dev(cl), dev(A.val))
    assert e.value.status == gw.SINGULAR
    B = ref.Csr(rowptr=rp, col=cl, val=np.array([2.0, 1.0, 1.0, 2.0]))
    lu_ref, piv_ref = ref.Hierarchy(B, ref.AmgParams()).coarse_lu()
    Hg = gw.amg_setup(2, dev(rp), dev(cl), dev(B.val))
    lu = torch.zeros(4, dtype=torch.float64, device="cuda")
    piv = torch.zeros(2, dtype=torch.int32, device="cuda")
    gw.amg_coarse_export(Hg, lu, piv)
    assert np.array_equal(host(piv), piv_ref)
    assert np.array_equal(host(lu).view(np.uint64), lu_ref.reshape(-1).view(np.uint64))


@pytest.mark.parametrize("n", [60, 120, 128, 130])
def test_coarsest_lu_with_row_interchanges(gw, ref, n):
    # A dense nonsymmetric matrix that is its own coarsest level, with
    # off-diagonal entries up to eight times the diagonal, so partial
    # pivoting interchanges rows at most steps (the flow hierarchies'
    # coarsest matrices rarely need one).  n = 60 and 120 take the two LDS
    # forms of the factorization (256 and 512 threads), 128 the largest
    # inverse by column-oriented substitutions and 130 the row-oriented one;
    # factors and pivots bit for bit.
    _say(f"coarsest LU with row interchanges, n={n}")
    rng = np.random.default_rng(1000 + n)
    M = rng.uniform(-4.0, 4.0, (n, n))
    np.fill_diagonal(M, rng.uniform(0.5, 1.0, n))
    rp = np.arange(0, n * n + 1, n, dtype=np.int32)
    cl = np.tile(np.arange(n, dtype=np.int32), n)
    A = ref.Csr(rowptr=rp, col=cl, val=M.reshape(-1).copy())
    Hr = ref.Hierarchy(A, ref.AmgParams())
    assert Hr.nlevels == 1
    lu_ref, piv_ref = Hr.coarse_lu()
    assert np.count_nonzero(piv_ref != np.arange(n)) > n // 2
    Hg = gw.amg_setup(n, dev(rp), dev(cl), dev(A.val))
    lu = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    piv = torch.zeros(n, dtype=torch.int32, device="cuda")
    inv = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    gw.amg_coarse_export(Hg, lu, piv, inv)
    assert np.array_equal(host(piv), piv_ref)
    assert np.array_equal(host(lu).view(np.uint64), lu_ref.reshape(-1).view(np.uint64))
    # the inverse undoes the interchanges (each column starts from the
    # permuted unit vector): A^-1 A = I
    Ainv = host(inv).reshape(n, n)
    assert np.abs(Ainv @ M - np.eye(n)).max() < 1e-10 * np.linalg.cond(M)


def test_breakdown_when_rhat_v_vanishes(gw, ref):
    # identity preconditioner on A = [[1, -3], [1, 1]], b = (1, 1): r_hat = r
    # = p = b and v = A b = (-2, 2), so r_hat.v = 0 exactly at the first
    # BiCGSTAB step and p.A p = 0 at the first CG step: both sides report
    # BREAKDOWN with no iteration taken.  (The skew matrix [[0, 1], [-1, 0]]
    # has the same zero but no positive diagonal: EINVAL on both sides.)
    _say("breakdown r_hat.v = 0")
    rp, cl = np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32)
    val = np.array([1.0, -3.0, 1.0, 1.0])
    b = np.array([1.0, 1.0])
    Hr = ref.Hierarchy(ref.Csr(rp, cl, val), ref.AmgParams(smoother=ref.NONE))
    assert ref.bicgstab(Hr, b)[1].status == ref.BREAKDOWN
    assert ref.pcg(Hr, b)[1].status == ref.BREAKDOWN
    Hg = gw.amg_setup(2, dev(rp), dev(cl), dev(val), gw.AmgParams(smoother=gw.SMOOTHER_NONE))
    for solve in (gw.amg_solve_bicgstab, gw.amg_solve_pcg):
        x = torch.full((2,), 5.0, dtype=torch.float64, device="cuda")
        info = solve(Hg, dev(b), x, gw.SolveParams(rtol=1e-8))
        assert info.status == gw.BREAKDOWN and info.iters == 0, (solve.__name__, info)
    with pytest.raises(gw.GwError) as e:
        gw.amg_setup(2, dev(rp), dev(cl), dev(np.array([0.0, 1.0, -1.0, 0.0])),
                     gw.AmgParams(smoother=gw.SMOOTHER_NONE))
    assert e.value.status == gw.EINVAL
