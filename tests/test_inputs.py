"""Checks of the seeded input generator (CPU only)."""
import numpy as np

import gwinputs as gi


def test_field_is_seeded():
    a = gi.lognormal_field((16, 12, 8), 4.0, 4, 11)
    b = gi.lognormal_field((16, 12, 8), 4.0, 4, 11)
    c = gi.lognormal_field((16, 12, 8), 4.0, 4, 12)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.dtype == np.float64 and a.shape == (16 * 12 * 8,) and np.all(a > 0)


def test_field_statistics():
    # Y = ln K - ln(1e-4): zero mean, variance sigma2 and exponential
    # covariance sigma2 exp(-r / lambda); on a domain much larger than lambda
    # the single-realisation estimates are within a few sampling errors.
    s2, lam = 2.0, 4.0
    K, clip = gi.lognormal_field((512, 512, 1), s2, lam, 5, return_clip=True)
    y = (np.log(K) - np.log(1e-4)).reshape(512, 512)
    assert clip < 0.05
    assert abs(y.mean()) < 0.15
    assert abs(y.var() - s2) < 0.25 * s2
    lag = int(lam)
    cov = np.mean((y[:, :-lag] - y.mean()) * (y[:, lag:] - y.mean()))
    assert abs(cov - s2 * np.exp(-1.0)) < 0.25 * s2


def test_well_layout_rule():
    g = gi.Grid(128, 128, 64)
    w = gi.four_well_layout(g)
    assert [(x.ix, x.iy, x.iz) for x in w] == [(32, 32, 32), (96, 32, 32), (32, 96, 32), (96, 96, 32)]
    regional = 1e-4 * (10.0 / 128) * (128 * 64)
    assert np.isclose(sum(x.q for x in w), 0.4 * regional)


def test_serve_stream():
    s = gi.serve_stream(200, 10.0, seed=5)
    assert len(s) == 200 and s[0].t == 0.0
    assert all(32 <= a.side <= 192 for a in s)
    assert {a.sigma2 for a in s} <= {1.0, 2.0, 4.0}
    assert all(4 <= a.corr_len <= 16 for a in s)
    assert np.all(np.diff([a.t for a in s]) >= 0)


def test_general_matrix_generators():
    import scipy.sparse as sp
    for rowptr, col, val in (gi.random_graph_spd(500, 4, 1), gi.arrow_spd(300, 2)):
        n = len(rowptr) - 1
        A = sp.csr_matrix((val, col, rowptr), shape=(n, n))
        assert (A - A.T).nnz == 0
        for i in range(n):
            c = col[rowptr[i]:rowptr[i + 1]]
            assert np.all(np.diff(c) > 0) and i in c
        d = A.diagonal()
        off = np.asarray(abs(A).sum(axis=1)).ravel() - d
        assert np.all(d > off)


def test_paper_like_layout():
    # the paper's 3D model size (Benchmarking Examples; Results, Table 1):
    # 550 x 500 x 10 blocks of 20 m, four doublets whose injectors are
    # screened over the five lower layers and producers over the five top ones
    g = gi.Grid(550, 500, 10, 20.0, 20.0, 20.0)
    w = gi.doublet_layout(g, 0.02)
    assert len(w) == 40 and abs(sum(x.q for x in w)) < 1e-15
    inj = [x for x in w if x.q < 0]
    prod = [x for x in w if x.q > 0]
    assert sorted({x.iz for x in inj}) == [0, 1, 2, 3, 4] and sorted({x.iz for x in prod}) == [5, 6, 7, 8, 9]
    assert len({(x.ix, x.iy) for x in inj}) == 4 and len({(x.ix, x.iy) for x in prod}) == 4
    p = gi.paper_like_aquifer(sigma2=0.0)
    assert p.grid == g and np.all(p.K == gi.K_PAPER)
    w2 = gi.doublet_layout(gi.Grid(550, 500, 1, 20.0, 20.0, 20.0), 0.02)
    assert len(w2) == 8 and all(x.iz == 0 for x in w2)
