"""The convergence poll only decides how many iterations are launched before
the host looks at the device flag; iterations after convergence are early
exits.  So the iterates, the iteration counts and the final residuals must
not depend on the poll interval (check_every), nor on whether the blocks are
launched one by one or replayed from a graph: checked bit for bit for CG on
the flow system, the mixed-precision flexible CG, BiCGSTAB and the
BiCGSTAB pair on the travel-time system.
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


POLLS = [(1, 0), (3, 0), (4, 0), (9, 0), (4, 1)]  # (check_every, graph)


def _bits(a):
    return a.view(np.uint64)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_pcg_independent_of_poll_interval(gw, ref, precision):
    _say(f"pcg poll intervals precision {precision}")
    p = gi.heterogeneous_aquifer(40, 32, 16, 4.0, 8, 11)
    A, b = ref.fv_assemble(p)
    H = gw.amg_setup(A.n, dev(A.rowptr), dev(A.col), dev(A.val), gw.AmgParams.flow(precision=precision))
    runs = []
    for ce, graph in POLLS:
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        info = gw.amg_solve_pcg(H, dev(b), x, gw.SolveParams(rtol=1e-8, check_every=ce, graph=graph))
        assert info.status == gw.OK
        runs.append((host(x), info))
    x0, i0 = runs[0]
    for (ce, graph), (x, info) in zip(POLLS[1:], runs[1:]):
        assert info.iters == i0.iters and info.rel_res_true == i0.rel_res_true, (ce, graph)
        assert np.array_equal(_bits(x), _bits(x0)), (ce, graph)


def test_bicgstab_single_and_pair_independent_of_poll_interval(gw, ref):
    _say("bicgstab poll intervals")
    import scipy.sparse.linalg as sla
    p = gi.heterogeneous_aquifer(32, 24, 12, 4.0, 6, 4)
    A, b = ref.fv_assemble(p)
    h = sla.spsolve(A.to_scipy().tocsc(), b)
    qx, qy, qz = ref.darcy_flux(p, h)
    At, bt, bc, nid = ref.tt_assemble(p.grid, qx, qy, qz, 0.25, zone=(0, 24, 0, 6))
    H = gw.amg_setup(At.n, dev(At.rowptr), dev(At.col), dev(At.val), gw.AmgParams.travel_time())
    single, pair = [], []
    for ce, graph in POLLS:
        sp = gw.SolveParams(rtol=1e-8, check_every=ce, graph=graph)
        x = torch.zeros(At.n, dtype=torch.float64, device="cuda")
        info = gw.amg_solve_bicgstab(H, dev(bt), x, sp)
        assert info.status == gw.OK
        single.append((host(x), info))
        x0 = torch.zeros(At.n, dtype=torch.float64, device="cuda")
        x1 = torch.zeros(At.n, dtype=torch.float64, device="cuda")
        st, infos = gw.amg_solve_bicgstab_pair(H, dev(bt), dev(bc), x0, x1, sp)
        assert st == gw.OK
        pair.append((host(x0), host(x1), infos))
    xs0, is0 = single[0]
    a0, b0, ip0 = pair[0]
    # the pair's first system is the single solve, bit for bit
    assert np.array_equal(_bits(a0), _bits(xs0)) and ip0[0].iters == is0.iters
    for (ce, graph), (x, info), (a, bb, ip) in zip(POLLS[1:], single[1:], pair[1:]):
        assert info.iters == is0.iters and np.array_equal(_bits(x), _bits(xs0)), (ce, graph)
        assert [q.iters for q in ip] == [q.iters for q in ip0], (ce, graph)
        assert np.array_equal(_bits(a), _bits(a0)) and np.array_equal(_bits(bb), _bits(b0)), (ce, graph)
