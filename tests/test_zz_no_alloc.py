"""The allocation-free PCG entry point (amg_solve_pcg_noalloc) against
amg_solve_pcg: the same heads, iteration counts and residuals bit for bit,
on two calls in a row where the second solves a smaller system, with the
FP64 and the mixed hierarchy; the workspace limit and the graph switch are
refused before any kernel runs.
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


def _assemble(gw, p):
    g = p.grid
    n, nnz = g.n, gw.fv_nnz(g)
    rowptr = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    col = torch.zeros(nnz, dtype=torch.int32, device="cuda")
    val = torch.zeros(nnz, dtype=torch.float64, device="cuda")
    b = torch.zeros(n, dtype=torch.float64, device="cuda")
    K = torch.from_numpy(np.ascontiguousarray(p.K)).cuda()
    gw.fv_assemble(g, K, (p.h_west, p.h_east), p.wells, rowptr, col, val, b)
    return rowptr, col, val, b


def _bits(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


CASES = [
    # (grid, variance, correlation length, seed, precision): the second call
    # of each pair solves a smaller system in the same workspace
    ((96, 80, 40), 4.0, 8, 31, 0),
    ((30, 24, 12), 2.0, 4, 32, 0),
    ((64, 48, 32), 4.0, 6, 33, 1),
    ((17, 13, 7), 1.0, 3, 34, 1),
]


def test_noalloc_pcg_equals_pcg_two_calls(gw):
    # the first call in the process has the runtime place the workspace
    # array on the device (with its code object); after that no call takes
    # device memory
    p = gi.heterogeneous_aquifer(8, 6, 4, 1.0, 3, 30)
    rowptr, col, val, b = _assemble(gw, p)
    H = gw.amg_setup(p.grid.n, rowptr, col, val, gw.AmgParams(n_coarse=20))
    x = torch.zeros(p.grid.n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    assert gw.amg_solve_pcg_noalloc(H, b, x).status == gw.OK
    torch.cuda.synchronize()
    _say(f"first call: device free memory change {(free0 - torch.cuda.mem_get_info()[0]) / 2**20:.2f} MiB")
    del H
    for (nx, ny, nz), s2, lam, seed, precision in CASES:
        _say(f"noalloc pcg {nx}x{ny}x{nz} precision {precision}")
        p = gi.heterogeneous_aquifer(nx, ny, nz, s2, lam, seed)
        n = p.grid.n
        rowptr, col, val, b = _assemble(gw, p)
        H = gw.amg_setup(n, rowptr, col, val, gw.AmgParams(precision=precision, n_coarse=100))
        sp = gw.SolveParams(rtol=1e-8, check_every=3)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        x = torch.full((n,), 9.0, dtype=torch.float64, device="cuda")
        info = gw.amg_solve_pcg_noalloc(H, b, x, sp)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        want = torch.zeros(n, dtype=torch.float64, device="cuda")
        info_ref = gw.amg_solve_pcg(H, b, want, sp)
        _say(f"  iters {info.iters}/{info_ref.iters} rel_res_true {info.rel_res_true:.2e}; "
             f"device free memory change {(free0 - free1) / 2**20:.2f} MiB")
        assert info.status == gw.OK and info_ref.status == gw.OK
        assert (info.iters, info.restarts) == (info_ref.iters, info_ref.restarts)
        assert info.rel_res_true == info_ref.rel_res_true and info.rel_res == info_ref.rel_res
        assert np.array_equal(_bits(x), _bits(want))
        # the workspace of this solve (6 n-vectors: 14 MiB for the first
        # system) was not taken from the device
        assert free0 - free1 < (2 << 20)
        del H


def test_noalloc_refusals(gw):
    _say("noalloc refusals")
    p = gi.heterogeneous_aquifer(12, 10, 6, 1.0, 3, 35)
    n = p.grid.n
    rowptr, col, val, b = _assemble(gw, p)
    H = gw.amg_setup(n, rowptr, col, val, gw.AmgParams(n_coarse=40))
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(gw.GwError) as e:
        gw.amg_solve_pcg_noalloc(H, b, x, gw.SolveParams(graph=1))
    assert e.value.status == gw.EINVAL
    # one row past the limit: a diagonal operator without a preconditioner
    m = gw.NOALLOC_MAX_ROWS + 1
    ar = torch.arange(m + 1, dtype=torch.int32, device="cuda")
    ac = torch.arange(m, dtype=torch.int32, device="cuda")
    av = torch.ones(m, dtype=torch.float64, device="cuda")
    Hd = gw.amg_setup(m, ar, ac, av, gw.AmgParams(smoother=gw.SMOOTHER_NONE))
    bd = torch.ones(m, dtype=torch.float64, device="cuda")
    xd = torch.zeros(m, dtype=torch.float64, device="cuda")
    with pytest.raises(gw.GwError) as e:
        gw.amg_solve_pcg_noalloc(Hd, bd, xd, gw.SolveParams())
    assert e.value.status == gw.EINVAL
    # at the limit itself the diagonal system solves (in one iteration)
    Hm = gw.amg_setup(m - 1, ar[:m], ac[:m - 1], av[:m - 1], gw.AmgParams(smoother=gw.SMOOTHER_NONE))
    info = gw.amg_solve_pcg_noalloc(Hm, bd, xd, gw.SolveParams())
    assert info.status == gw.OK and info.iters == 1
    assert torch.all(xd[:m - 1] == 1.0).item()
    # the library still works after the refusals
    info = gw.amg_solve_pcg_noalloc(H, b, x, gw.SolveParams())
    assert info.status == gw.OK
