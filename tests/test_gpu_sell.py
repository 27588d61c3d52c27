"""The level-0 copies the solve kernels read.  The sliced copy: its slice
height and stored entry count against a count made on the host from the
operator's row lengths (each slice of C rows as wide as its longest row; C
the largest of 64, 32, 16, 8 whose count is within 2 % of the count at 8),
for the 7-point flow operator (stencil copy switched off) and the upwind
travel-time operator (rows of 1 to 7 entries, short slices); the travel-time
pair solved on short slices against the oracle's exact sweep.  The symmetric
stencil copy: taken by the 7- and 5-point flow operators, the same PCG
iterates bit for bit as on the sliced copy, and not taken when one value
breaks the symmetry.  The one-sided stencil copy: taken by the upwind
travel-time operator, the same pair iterates bit for bit as on the sliced
copy and the oracle's exact sweep, and not taken when a face is stored by
both of its rows or an off-diagonal is not negative.
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


def _padded(rowptr, c):
    lens = np.diff(np.asarray(rowptr, dtype=np.int64))
    return int(np.pad(lens, (0, (-lens.size) % c)).reshape(-1, c).max(axis=1).sum()) * c


def _expected(rowptr):
    pad = {c: _padded(rowptr, c) for c in (8, 16, 32, 64)}
    for c in (64, 32, 16):
        if pad[c] <= 1.02 * pad[8]:
            return c, pad[c]
    return 8, pad[8]


def _tt_operator(ref, nx, ny, nz, s2, lam, seed):
    p = gi.heterogeneous_aquifer(nx, ny, nz, s2, lam, seed)
    fr = ref.solve_flow(p, ref.AmgParams(), rtol=1e-10)
    qx, qy, qz = ref.darcy_flux(p, fr.h)
    g = p.grid
    A, bt, bc, _ = ref.tt_assemble(g, qx, qy, qz, p.phi, (0, g.ny, 0, max(1, g.nz // 2)))
    return p, fr.h, A, bt, bc


@pytest.mark.parametrize("case", [(48, 40, 20, 4.0, 6, 61), (37, 29, 11, 1.0, 3, 62)], ids=["48x40x20", "37x29x11"])
def test_slice_height_and_padding(gw, ref, case, monkeypatch):
    _say(f"sliced copy {case}")
    monkeypatch.setenv("GWAMG_STENCIL", "0")
    p, _, A, bt, bc = _tt_operator(ref, *case)
    n = p.grid.n
    for name, (rowptr, col, val), prm in (
            ("flow", _flow_csr(ref, p), gw.AmgParams.flow()),
            ("travel time", (A.rowptr, A.col, A.val), gw.AmgParams.travel_time())):
        H = gw.amg_setup(n, dev(rowptr), dev(col), dev(val), prm)
        lv = H.info()[0][0]
        c, padded = _expected(rowptr)
        _say(f"  {name}: slice rows {lv.slice_rows} (host {c}), entries {lv.nnz_sliced} (host {padded}), "
             f"nnz {int(rowptr[-1])}")
        assert (lv.slice_rows, lv.nnz_sliced) == (c, padded)
        if name == "travel time":  # short slices pad less than whole-wave ones
            assert c < 64 and padded < 0.95 * _padded(rowptr, 64)


def _flow_csr(ref, p):
    A, _ = ref.fv_assemble(p)
    return A.rowptr, A.col, A.val


def test_pair_on_short_slices_against_oracle(gw, ref, monkeypatch):
    # the upwind system is acyclic: the oracle's sweep in head order gives
    # its exact solution
    _say("travel-time pair on short slices vs the oracle's exact sweep")
    monkeypatch.setenv("GWAMG_STENCIL", "0")
    p, h, A, bt, bc = _tt_operator(ref, 48, 40, 20, 4.0, 6, 61)
    n = p.grid.n
    H = gw.amg_setup(n, dev(A.rowptr), dev(A.col), dev(A.val), gw.AmgParams.travel_time())
    assert H.info()[0][0].slice_rows < 64
    x0 = torch.zeros(n, dtype=torch.float64, device="cuda")
    x1 = torch.zeros(n, dtype=torch.float64, device="cuda")
    st, (i0, i1) = gw.amg_solve_bicgstab_pair(H, dev(bt), dev(bc), x0, x1, gw.SolveParams(rtol=1e-10))
    assert st == gw.OK
    for got, b in ((x0, bt), (x1, bc)):
        want = ref.tt_sweep(A, b, h)
        err = np.linalg.norm(got.cpu().numpy() - want) / np.linalg.norm(want)
        _say(f"  iters {i0.iters}/{i1.iters}, rel err {err:.2e}")
        assert err <= 1e-8


def _pcg(gw, n, rowptr, col, val, b):
    H = gw.amg_setup(n, dev(rowptr), dev(col), dev(val), gw.AmgParams.flow())
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    info = gw.amg_solve_pcg(H, dev(b), x, gw.SolveParams(rtol=1e-10))
    assert info.status == gw.OK
    return H.info()[0][0], x.cpu().numpy(), info.iters


@pytest.mark.parametrize("make,k", [(lambda: gi.heterogeneous_aquifer(37, 29, 11, 1.0, 3, 62), 3),
                                    (lambda: gi.homogeneous_slab(), 2)], ids=["7-point", "5-point"])
def test_flow_operator_takes_the_stencil_copy(gw, ref, make, k, monkeypatch):
    p = make()
    _say(f"stencil copy {p.grid.nx}x{p.grid.ny}x{p.grid.nz}")
    A, b = ref.fv_assemble(p)
    n = p.grid.n
    lv, x, it = _pcg(gw, n, A.rowptr, A.col, A.val, b)
    assert (lv.stencil_offsets, lv.slice_rows, lv.nnz_sliced) == (k, 0, 0)
    monkeypatch.setenv("GWAMG_STENCIL", "0")
    lv2, x2, it2 = _pcg(gw, n, A.rowptr, A.col, A.val, b)
    assert lv2.stencil_offsets == 0 and lv2.slice_rows > 0
    _say(f"  iterations {it} (stencil) / {it2} (sliced)")
    assert it == it2
    assert np.array_equal(x.view(np.uint64), x2.view(np.uint64))
    want = ref.pcg(ref.Hierarchy(A, ref.AmgParams(eps_strong=0.03, npre=1, npost=1)), b, rtol=1e-10)[0]
    assert np.linalg.norm(x - want) <= 1e-8 * np.linalg.norm(want)


def test_asymmetric_values_keep_the_sliced_copy(gw, ref):
    # found by the setup's pattern probe (AMG preconditioner), or by the
    # copy's own check of every mirror pair (no preconditioner: no probe)
    p = gi.heterogeneous_aquifer(37, 29, 11, 1.0, 3, 62)
    _say("one value off its mirror: sliced copy")
    A, b = ref.fv_assemble(p)
    n = p.grid.n
    val = A.val.copy()
    # an off-diagonal entry right of the diagonal in the middle row
    i = n // 2
    q = next(q for q in range(A.rowptr[i], A.rowptr[i + 1]) if A.col[q] > i)
    val[q] = np.nextafter(val[q], 0.0)
    lv, x, it = _pcg(gw, n, A.rowptr, A.col, val, b)
    assert lv.stencil_offsets == 0 and lv.slice_rows > 0
    for v, k in ((A.val, 3), (val, 0)):
        H = gw.amg_setup(n, dev(A.rowptr), dev(A.col), dev(v), gw.AmgParams(smoother=gw.SMOOTHER_NONE))
        lv = H.info()[0][0]
        assert lv.stencil_offsets == k and (lv.slice_rows > 0) == (k == 0)


def _pair(gw, n, A, bt, bc):
    H = gw.amg_setup(n, dev(A.rowptr), dev(A.col), dev(A.val), gw.AmgParams.travel_time())
    x0 = torch.zeros(n, dtype=torch.float64, device="cuda")
    x1 = torch.zeros(n, dtype=torch.float64, device="cuda")
    st, (i0, i1) = gw.amg_solve_bicgstab_pair(H, dev(bt), dev(bc), x0, x1, gw.SolveParams(rtol=1e-10))
    assert st == gw.OK
    return H.info()[0][0], x0.cpu().numpy(), x1.cpu().numpy(), (i0.iters, i1.iters)


def test_upwind_operator_takes_the_one_sided_copy(gw, ref, monkeypatch):
    _say("travel-time pair on the one-sided stencil copy")
    p, h, A, bt, bc = _tt_operator(ref, 48, 40, 20, 4.0, 6, 61)
    n = p.grid.n
    lv, x0, x1, it = _pair(gw, n, A, bt, bc)
    assert (lv.stencil_offsets, lv.slice_rows, lv.nnz_sliced) == (3, 0, 0)
    monkeypatch.setenv("GWAMG_STENCIL", "0")
    lv2, y0, y1, it2 = _pair(gw, n, A, bt, bc)
    assert lv2.stencil_offsets == 0 and lv2.slice_rows > 0
    _say(f"  iterations {it} (stencil) / {it2} (sliced)")
    assert it == it2
    assert np.array_equal(x0.view(np.uint64), y0.view(np.uint64))
    assert np.array_equal(x1.view(np.uint64), y1.view(np.uint64))
    for got, b in ((x0, bt), (x1, bc)):
        want = ref.tt_sweep(A, b, h)
        assert np.linalg.norm(got - want) <= 1e-8 * np.linalg.norm(want)


@pytest.mark.parametrize("how", ["both rows", "positive"])
def test_two_sided_face_keeps_the_sliced_copy(gw, ref, how):
    _say(f"upwind operator with a face {how}: sliced copy")
    p, h, A, bt, bc = _tt_operator(ref, 30, 22, 14, 4.0, 6, 63)
    n = p.grid.n
    rowptr, col, val = A.rowptr.copy(), A.col.copy(), A.val.copy()
    # a row with an off-diagonal entry
    i = next(r for r in range(n // 2, n) if rowptr[r + 1] - rowptr[r] > 1)
    q = next(q for q in range(rowptr[i], rowptr[i + 1]) if col[q] != i)
    if how == "positive":
        val[q] = -val[q]
    else:
        # store the face's mirror too: insert a_{j,i} into row j
        j = int(col[q])
        cols_j = list(col[rowptr[j]:rowptr[j + 1]])
        assert i not in cols_j
        pos = rowptr[j] + int(np.searchsorted(cols_j, i))
        col = np.insert(col, pos, i)
        val = np.insert(val, pos, val[q] * 0.5)
        rowptr = rowptr.copy()
        rowptr[j + 1:] += 1
    # the setup's pattern probe finds the pattern nonsymmetric, so the
    # one-sided form is tried and its check refuses it
    H = gw.amg_setup(n, dev(rowptr), dev(col), dev(val), gw.AmgParams.travel_time())
    lv = H.info()[0][0]
    assert lv.stencil_offsets == 0 and lv.slice_rows > 0
