"""The paper-size workload: 550 x 500 x 10 blocks of 20 m with four doublets.

Its homogeneous case is the problem of the paper's hierarchy table (Results,
Table 1: 2,750,000 unknowns, 18,679,000 nonzeros at level 0).  The GPU
hierarchy matches the oracle's level by level (sizes and aggregate maps bit
for bit), the heads match the oracle's same-algorithm solve within 1e-8, and
the report prints our levels beside the paper's (context: the paper's AMG
differs in its coarsening constants, which it does not give).
"""
import os
import sys

import numpy as np
import pytest

import gwinputs as gi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_hierarchy.txt")


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2001_05798_amd as gw
    return gw


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _table1():
    rows = [tuple(int(v) for v in line.split()) for line in open(GOLDEN) if line.strip() and line[0] != "#"]
    return rows


def test_paper_size_homogeneous_hierarchy(gw, ref):
    _say("paper-size 550x500x10 homogeneous, four doublets")
    p = gi.paper_like_aquifer(sigma2=0.0)
    g = p.grid
    n, nnz = g.n, gw.fv_nnz(g)
    t1 = _table1()
    assert (n, nnz) == (t1[0][1], t1[0][2])
    d = dict(device="cuda")
    rowptr = torch.zeros(n + 1, dtype=torch.int32, **d)
    col = torch.zeros(nnz, dtype=torch.int32, **d)
    val = torch.zeros(nnz, dtype=torch.float64, **d)
    b = torch.zeros(n, dtype=torch.float64, **d)
    gw.fv_assemble(g, torch.from_numpy(p.K).cuda(), (p.h_west, p.h_east), p.wells, rowptr, col, val, b)
    ap = ref.AmgParams()
    fr = ref.solve_flow(p, ap, rtol=1e-8)
    Hg = gw.amg_setup(n, rowptr, col, val, gw.AmgParams())
    infos, _ = Hg.info()
    assert Hg.nlevels == fr.H.nlevels
    oc = sum(i.nnz for i in infos) / infos[0].nnz
    gc = sum(i.n for i in infos) / infos[0].n
    oc1 = sum(r[2] for r in t1) / t1[0][2]
    gc1 = sum(r[1] for r in t1) / t1[0][1]
    _say(f"  level  unknowns (ours / paper)   nonzeros (ours / paper)")
    for l in range(max(len(infos), len(t1))):
        ours = (infos[l].n, infos[l].nnz) if l < len(infos) else ("-", "-")
        theirs = t1[l][1:] if l < len(t1) else ("-", "-")
        _say(f"  {l:5d}  {ours[0]:>9} / {theirs[0]:<9}  {ours[1]:>10} / {theirs[1]}")
    _say(f"  operator complexity {oc:.2f} (paper {oc1:.2f}), grid complexity {gc:.2f} (paper {gc1:.2f})")
    for l in range(fr.H.nlevels - 1):
        lv = fr.H.level(l)
        assert (infos[l].n, infos[l].nnz) == (lv.A.n, lv.A.nnz), f"level {l}"
        agg = torch.zeros(infos[l].n, dtype=torch.int32, device="cuda")
        gw.amg_level_export(Hg, l, agg=agg)
        assert np.array_equal(host(agg), lv.agg), f"level {l}"
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    info = gw.amg_solve_pcg(Hg, b, x, gw.SolveParams(rtol=1e-8))
    err = np.linalg.norm(host(x) - fr.h) / np.linalg.norm(fr.h)
    _say(f"  iters gpu {info.iters} oracle {fr.info.iters} rel err {err:.3e}")
    assert info.status == gw.OK and info.rel_res_true <= 1e-8 and err <= 1e-8
