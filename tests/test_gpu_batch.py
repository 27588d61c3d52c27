"""Shared launches for many solves: amg_solve_pcg_batch and
amg_solve_bicgstab_pair_batch against the one-system solves on the same
hierarchies -- iterates, iteration counts, statuses and residuals bit for
bit -- on systems of uneven size and depth (a coarsest-only hierarchy among
them), with a zero right-hand side, a system stopped by maxiter, FP64 and
mixed hierarchies, launched one by one and as captured graphs; and one
system of a batch against the oracle.
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


def bits(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def _flow(gw, p):
    g = p.grid
    n, nnz = g.n, gw.fv_nnz(g)
    rowptr = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    col = torch.zeros(nnz, dtype=torch.int32, device="cuda")
    val = torch.zeros(nnz, dtype=torch.float64, device="cuda")
    b = torch.zeros(n, dtype=torch.float64, device="cuda")
    gw.fv_assemble(g, dev(p.K), (p.h_west, p.h_east), p.wells, rowptr, col, val, b)
    return rowptr, col, val, b


FLOW = [  # uneven sizes and depths; the 6x5x4 grid is its own coarsest level
    (48, 40, 20, 4.0, 6, 41),
    (6, 5, 4, 1.0, 2, 42),
    (30, 24, 12, 2.0, 4, 43),
    (64, 48, 32, 4.0, 8, 44),
    (17, 13, 7, 1.0, 3, 45),
]


@pytest.mark.parametrize("precision,graph", [(0, 0), (1, 0), (0, 1), (1, 1)],
                         ids=["fp64", "mixed", "fp64-graph", "mixed-graph"])
def test_pcg_batch_equals_single(gw, precision, graph):
    _say(f"pcg batch precision {precision} graph {graph}")
    Hs, bs = [], []
    for nx, ny, nz, s2, lam, seed in FLOW:
        p = gi.heterogeneous_aquifer(nx, ny, nz, s2, lam, seed)
        rowptr, col, val, b = _flow(gw, p)
        Hs.append(gw.amg_setup(p.grid.n, rowptr, col, val, gw.AmgParams(precision=precision)))
        bs.append(b)
    bs[2] = torch.zeros_like(bs[2])  # b = 0: x = 0 with no iteration
    depths = [H.nlevels for H in Hs]
    assert min(depths) == 1 and max(depths) >= 3, depths
    sp = gw.SolveParams(rtol=1e-8, check_every=3, graph=graph)
    want = []
    for H, b in zip(Hs, bs):
        x = torch.zeros(b.numel(), dtype=torch.float64, device="cuda")
        want.append((gw.amg_solve_pcg(H, b, x, sp), bits(x)))
    xs = [torch.full((b.numel(),), 5.0, dtype=torch.float64, device="cuda") for b in bs]
    infos = gw.amg_solve_pcg_batch(Hs, bs, xs, sp)
    for k, (info, x) in enumerate(zip(infos, xs)):
        w, wx = want[k]
        _say(f"  system {k}: levels {depths[k]} iters {info.iters}/{w.iters} status {info.status}")
        assert (info.iters, info.status, info.restarts) == (w.iters, w.status, w.restarts), k
        assert info.rel_res_true == w.rel_res_true and info.rel_res == w.rel_res, k
        assert np.array_equal(bits(x), wx), k
    assert infos[2].iters == 0 and not bits(xs[2]).any()
    # a second batch on the same hierarchies (workspace reused) with one
    # system stopped by maxiter
    sp2 = gw.SolveParams(rtol=1e-10, maxiter=4, check_every=3, graph=graph)
    want2 = []
    for H, b in zip(Hs[:2], bs[:2]):
        x = torch.zeros(b.numel(), dtype=torch.float64, device="cuda")
        want2.append((gw.amg_solve_pcg(H, b, x, sp2), bits(x)))
    xs2 = [torch.zeros(b.numel(), dtype=torch.float64, device="cuda") for b in bs[:2]]
    infos2 = gw.amg_solve_pcg_batch(Hs[:2], bs[:2], xs2, sp2)
    assert infos2[0].status == gw.NOT_CONVERGED
    for (w, wx), info, x in zip(want2, infos2, xs2):
        assert (info.iters, info.status, info.restarts) == (w.iters, w.status, w.restarts)
        assert np.array_equal(bits(x), wx)


def _tt_system(gw, ref, nx, ny, nz, s2, lam, seed, precision):
    p = gi.heterogeneous_aquifer(nx, ny, nz, s2, lam, seed)
    fr = ref.solve_flow(p, ref.AmgParams(), rtol=1e-10)
    qx, qy, qz = ref.darcy_flux(p, fr.h)
    g = p.grid
    A, bt, bc, _ = ref.tt_assemble(g, qx, qy, qz, p.phi, (0, g.ny, 0, max(1, g.nz // 2)))
    H = gw.amg_setup(g.n, dev(A.rowptr), dev(A.col), dev(A.val), gw.AmgParams.travel_time(precision=precision))
    return A, bt, bc, H


TT = [(36, 30, 12, 2.0, 4, 51), (20, 16, 8, 4.0, 3, 52), (44, 36, 16, 1.0, 6, 53)]


@pytest.mark.parametrize("precision,graph", [(0, 0), (1, 0), (1, 1)], ids=["fp64", "mixed", "mixed-graph"])
def test_bicgstab_pair_batch_equals_single(gw, ref, precision, graph):
    _say(f"bicgstab pair batch precision {precision} graph {graph}")
    sysl = [_tt_system(gw, ref, *c, precision) for c in TT]
    Hs = [s[3] for s in sysl]
    b0 = [dev(s[1]) for s in sysl]
    b1 = [dev(s[2]) for s in sysl]
    b1[1] = torch.zeros_like(b1[1])  # a zero second right-hand side
    sp = gw.SolveParams(rtol=1e-8, check_every=4, graph=graph)
    want = []
    for H, u, v in zip(Hs, b0, b1):
        x0 = torch.zeros(u.numel(), dtype=torch.float64, device="cuda")
        x1 = torch.zeros(u.numel(), dtype=torch.float64, device="cuda")
        st, infos = gw.amg_solve_bicgstab_pair(H, u, v, x0, x1, sp)
        want.append((infos, bits(x0), bits(x1)))
    x0s = [torch.full((u.numel(),), 2.0, dtype=torch.float64, device="cuda") for u in b0]
    x1s = [torch.full((u.numel(),), 3.0, dtype=torch.float64, device="cuda") for u in b0]
    st, infos = gw.amg_solve_bicgstab_pair_batch(Hs, b0, b1, x0s, x1s, sp)
    assert st == gw.OK
    for k, ((i0, i1), x0, x1) in enumerate(zip(infos, x0s, x1s)):
        (w0, w1), wx0, wx1 = want[k]
        _say(f"  system {k}: iters {i0.iters}/{w0.iters}, {i1.iters}/{w1.iters}")
        for got, w in ((i0, w0), (i1, w1)):
            assert (got.iters, got.status, got.restarts) == (w.iters, w.status, w.restarts), k
            assert got.rel_res_true == w.rel_res_true, k
        assert np.array_equal(bits(x0), wx0) and np.array_equal(bits(x1), wx1), k
    assert infos[1][1].iters == 0 and not bits(x1s[1]).any()


def test_batch_system_against_oracle(gw, ref):
    # one FP64 system of a batch against the oracle's same-algorithm solve
    _say("pcg batch vs oracle")
    probs = [gi.heterogeneous_aquifer(*c[:3], c[3], c[4], c[5]) for c in FLOW[:3]]
    Hs, bs = [], []
    for p in probs:
        rowptr, col, val, b = _flow(gw, p)
        Hs.append(gw.amg_setup(p.grid.n, rowptr, col, val, gw.AmgParams()))
        bs.append(b)
    xs = [torch.zeros(b.numel(), dtype=torch.float64, device="cuda") for b in bs]
    infos = gw.amg_solve_pcg_batch(Hs, bs, xs, gw.SolveParams(rtol=1e-8))
    fr = ref.solve_flow(probs[0], ref.AmgParams(), rtol=1e-8)
    err = np.linalg.norm(xs[0].cpu().numpy() - fr.h) / np.linalg.norm(fr.h)
    _say(f"  iters {infos[0].iters} oracle {fr.info.iters} rel err {err:.2e}")
    assert infos[0].status == gw.OK and err <= 1e-8


def test_batch_rejects_mismatched_hierarchies(gw):
    _say("batch refusals")
    p = gi.heterogeneous_aquifer(12, 10, 6, 1.0, 3, 46)
    rowptr, col, val, b = _flow(gw, p)
    H64 = gw.amg_setup(p.grid.n, rowptr, col, val, gw.AmgParams(n_coarse=40))
    H32 = gw.amg_setup(p.grid.n, rowptr, col, val, gw.AmgParams(n_coarse=40, precision=gw.PRECISION_MIXED))
    x = [torch.zeros(p.grid.n, dtype=torch.float64, device="cuda") for _ in range(2)]
    with pytest.raises(gw.GwError) as e:
        gw.amg_solve_pcg_batch([H64, H32], [b, b], x)
    assert e.value.status == gw.EINVAL
    with pytest.raises(gw.GwError) as e:
        gw.amg_solve_pcg_batch([H64, H64], [b, b], x)
    assert e.value.status == gw.EINVAL
