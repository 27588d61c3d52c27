"""Transient flow (Eq. 2) on the GPU against the oracle.

The oracle solves every implicit step directly; the GPU solves it with PCG
to a relative residual of 1e-10, either preconditioned by the kept hierarchy
of the conductance matrix (shifted operator) or by a hierarchy of the step's
own matrix.  Heads agree within 1e-8 relative (FP64) or 1e-6 (FP32
hierarchy); the reuse ratio and decision are bit-identical.
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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _problem():
    g = gi.Grid(24, 18, 8)
    K = gi.lognormal_field((24, 18, 8), 2.0, 4.0, 41)
    return gi.Problem(g, K, wells=[gi.Well(15, 9, 3, 3e-4), gi.Well(6, 4, 5, 1e-4)])


def _storage(g, seed=5):
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(-5, -4, g.n)


def test_shifted_pcg_matches_direct(gw, ref):
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    _say("amg_solve_pcg_shifted 24x18x8")
    p = _problem()
    g = p.grid
    A, b = ref.fv_assemble(p)
    rowptr, col, val = dev(A.rowptr), dev(A.col), dev(A.val)
    H = gw.amg_setup(g.n, rowptr, col, val, gw.AmgParams())
    Ss = _storage(g)
    for dt in (1e4, 1e-3):   # reuse ratio below 0.01, then far above 1
        s = ref.storage_shift(g, Ss, dt)
        rhs = b + s * np.linspace(0.0, 1.0, g.n)
        want = sla.spsolve((A.to_scipy() + sp.diags(s)).tocsc(), rhs)
        x = torch.zeros(g.n, dtype=torch.float64, device="cuda")
        info = gw.amg_solve_pcg_shifted(H, dev(s), dev(rhs), x, gw.SolveParams(rtol=1e-10))
        _say(f"  dt {dt:g} ratio {ref.reuse_ratio(A, s):.2e}: iters {info.iters}")
        assert info.status == gw.OK and info.rel_res_true <= 1e-10
        assert _rel(host(x), want) <= 1e-8


@pytest.mark.parametrize("precision,tol", [(0, 1e-8), (1, 1e-6)], ids=["fp64", "mixed"])
def test_transient_steps_match_oracle(gw, ref, precision, tol):
    _say(f"flow_transient 24x18x8 precision {precision}")
    p = _problem()
    g = p.grid
    Ss = _storage(g)
    A, b = ref.fv_assemble(p)
    d = A.to_scipy().diagonal()
    dt_star = float(np.max(Ss / (0.01 * d)))   # V = 1: the step where the ratio is delta
    dts = [0.05 * dt_star, 0.05 * dt_star, 3.0 * dt_star, 40.0 * dt_star, 0.05 * dt_star]
    h0 = np.full(g.n, 5.0)
    r = ref.transient_flow(p, Ss, h0, dts)
    h = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    hs = torch.zeros(g.n * len(dts), dtype=torch.float64, device="cuda")
    st, info = gw.flow_transient(g, dev(p.K), (p.h_west, p.h_east), p.wells, dev(Ss), dev(h0), dts, h,
                                 params=gw.AmgParams(precision=precision), sp=gw.SolveParams(rtol=1e-10),
                                 h_steps=hs)
    assert st == gw.OK
    steps = host(hs).reshape(len(dts), g.n)
    for k, (inf, want) in enumerate(zip(info, r.heads)):
        err = _rel(steps[k], want)
        _say(f"  step {k}: reused {inf.reused} ratio {inf.ratio:.3e} iters {inf.iters} err {err:.2e}")
        assert inf.ratio == r.ratios[k]
        assert (inf.reused == 1) == r.reuse[k]
        assert inf.rel_res_true <= 1e-10 and err <= tol
    # the first short step builds, the second reuses it, the long ones keep
    # the setup of C, and the last short step finds its setup still cached
    assert [i.reused for i in info] == [0, 2, 1, 1, 2]
    assert np.array_equal(host(h), steps[-1])


def test_transient_full_size_step(gw, ref):
    # one long step on the 1M-cell aquifer with the kept hierarchy of C,
    # against the oracle's own AMG-PCG on C + S/dt (different preconditioner,
    # same system; both to relative residual 1e-10)
    import scipy.sparse as sp
    _say("flow_transient 128x128x64, one step with the setup of C kept")
    p = gi.heterogeneous_aquifer(128, 128, 64, 4.0, 8, 11)
    g = p.grid
    Ss = np.full(g.n, 1e-5)
    dt = 36000.0
    A, b = ref.fv_assemble(p)
    s = ref.storage_shift(g, Ss, dt)
    h0 = np.zeros(g.n)
    At = ref.Csr(A.rowptr, A.col, (A.to_scipy() + sp.diags(s)).tocsr().data.copy())
    assert np.array_equal(At.to_scipy().indices, A.col)
    H = ref.Hierarchy(At, ref.AmgParams())
    want, oinf = ref.pcg(H, b + s * h0, rtol=1e-10)
    h = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    st, info = gw.flow_transient(g, dev(p.K), (p.h_west, p.h_east), p.wells, dev(Ss), dev(h0), [dt], h,
                                 sp=gw.SolveParams(rtol=1e-10))
    err = _rel(host(h), want)
    _say(f"  ratio {info[0].ratio:.3e} reused {info[0].reused} iters gpu {info[0].iters} oracle {oinf.iters} "
         f"err {err:.2e}")
    assert st == gw.OK and info[0].reused == 1 and info[0].rel_res_true <= 1e-10
    assert err <= 1e-8
