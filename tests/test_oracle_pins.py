"""Hand-worked pins of oracle steps whose output no closed form fixes.

Each case is small enough to work out on paper from the readings the oracle
implements (aggregation passes, prolongator smoothing, the flexible-CG
direction update, the PMIS splitting), so that a plausible slip in any of
them -- the first or the weakest neighbour instead of the heaviest, the raw
diagonal instead of the lumped one, a dropped 4/3 factor, a Fletcher-Reeves
beta, a C test against any instead of every neighbour -- changes a value
written out below.

Paper: Results, Groundwater Flow Problems (smoothed aggregation with nodal
aggregates, CG with the AMG preconditioner); Introduction (the setup phase
builds the grids and transfer operators); Results, figures' RS variant.
"""
import numpy as np
import pytest
import scipy.sparse as sp

ROOT_STATE = 2


def _csr(ref, M):
    M = sp.csr_matrix(M)
    M.sort_indices()
    return ref.Csr(M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64).copy())


def _weighted_chain(n, weights, shift=0.0, extra=()):
    """Graph Laplacian of a chain 0-1-...-(n-1) with edge (i, i+1) of weight
    weights[i], extra edges (i, j, w), plus shift on the diagonal."""
    A = np.zeros((n, n))
    edges = [(i, i + 1, weights[i]) for i in range(n - 1)] + list(extra)
    for i, j, w in edges:
        A[i, j] -= w
        A[j, i] -= w
        A[i, i] += w
        A[j, j] += w
    A += shift * np.eye(n)
    return A


def _hier_with_roots(ref, A, roots, eps=0.08, **kw):
    """Setup whose level-0 MIS-2 roots are `roots` (the hash seed decides
    which of the valid MIS-2 sets the rounds pick, so scan seeds)."""
    Ac = _csr(ref, A)
    for seed in range(1, 20000):
        H = ref.Hierarchy(Ac, ref.AmgParams(eps_strong=eps, n_coarse=2, seed=seed, **kw))
        lv = H.level(0)
        if set(np.flatnonzero(lv.state == ROOT_STATE).tolist()) == set(roots):
            return H, lv
    pytest.fail(f"no seed gives the roots {roots}")


def test_aggregation_pass2_by_hand(ref):
    # chain 0..8 with roots 0, 4, 8 (aggregates 0, 1, 2).  Pass 1: 1 -> 0,
    # 3 and 5 -> 1, 7 -> 2.  Node 2 touches aggregate 0 through weight 1 and
    # aggregate 1 through weight 3: the heavier wins -> 1.  Node 6 touches
    # aggregates 1 and 2 through equal weights 2: the tie goes to the smaller
    # id -> 1.  (Joining the first, the lightest or the last neighbour, or
    # ties to the larger id, each change one of the two.)
    w = [1.0, 1.0, 3.0, 1.0, 1.0, 2.0, 2.0, 1.0]
    A = _weighted_chain(9, w, shift=0.5)
    H, lv = _hier_with_roots(ref, A, {0, 4, 8})
    assert lv.nc == 3
    assert lv.agg.tolist() == [0, 0, 1, 1, 1, 1, 1, 2, 2]


def test_aggregation_pass2_weight_from_either_side(ref):
    # nonsymmetric operator: pass 2 weighs an edge by max(|a_ij|, |a_ji|).
    # Node 2's own row holds -1 toward 1 and -2 toward 3, but a_12 is -4: the
    # edge to aggregate 0 weighs 4 against 2 -> 0 (its own row alone would
    # pick aggregate 1).
    A = _weighted_chain(9, [1.0] * 8, shift=0.5)
    A[1, 2] = -4.0
    A[1, 1] += 3.0
    A[2, 3] = -2.0
    A[2, 2] += 1.0
    H, lv = _hier_with_roots(ref, A, {0, 4, 8})
    assert lv.agg[2] == 0
    assert lv.agg[6] == 1  # equal weights 1 and 1: the smaller id


def test_prolongator_chain_by_hand(ref):
    # 1D Laplacian tridiag(-1, 2, -1) on 9 nodes, roots 1, 4, 7 (aggregates
    # {0,1,2}, {3,4,5}, {6,7,8}), plus a weak link 3-8 of weight 0.05
    # (0.05^2 < 0.08^2 * 2.05 * 2.05): a_33 = a_88 = 2.05, and lumping it
    # gives dF_3 = dF_8 = 2.  Gershgorin: interior rows sum |a_ij| / a_ii = 2,
    # so omega_P = (4/3)/2 = 2/3 and omega_P/dF = 1/3 on every row.
    #   P_iI = [agg(i) = I] - (1/3) * sum_{j in I} aF_ij
    # e.g. row 3: I = 0: -(1/3)(-1) = 1/3;  I = 1: 1 - (1/3)(dF_3 - 1) = 2/3.
    # With a_33 in place of dF_3 row 3 would read 0.325 / 0.675 (or 0.65 with
    # a_33 only in the sum); without the 4/3 factor the 2/3 entries read 3/4.
    A = _weighted_chain(9, [1.0] * 8, extra=[(3, 8, 0.05)])
    A[0, 0] += 1.0
    A[8, 8] += 1.0   # Dirichlet ends: tridiag(-1, 2, -1) plus the weak link
    H, lv = _hier_with_roots(ref, A, {1, 4, 7})
    assert lv.agg.tolist() == [0, 0, 0, 1, 1, 1, 2, 2, 2]
    assert lv.omega_p == pytest.approx(2.0 / 3.0, rel=1e-15)
    t, h = 1.0 / 3.0, 2.0 / 3.0
    want = np.array([
        [h, 0, 0],
        [1, 0, 0],
        [h, t, 0],
        [t, h, 0],
        [0, 1, 0],
        [0, h, t],
        [0, t, h],
        [0, 0, 1],
        [0, 0, h],
    ])
    got = lv.P.dense()
    assert np.allclose(got, want, rtol=0, atol=1e-15)
    # the stored pattern is exactly the nonzeros above, columns ascending
    assert [list(lv.P.col[lv.P.rowptr[i]:lv.P.rowptr[i + 1]]) for i in range(9)] == \
        [list(np.flatnonzero(want[i])) for i in range(9)]


def _nonsym_vcycle_problem(ref, gi):
    p = gi.heterogeneous_aquifer(14, 12, 6, 2.0, 3, 5)
    A, b = ref.fv_assemble(p)
    # two pre-sweeps and no post-sweep: the V-cycle is not a symmetric operator
    H = ref.Hierarchy(A, ref.AmgParams(n_coarse=20, npre=2, npost=0))
    return A, b, H


def test_vcycle_without_post_sweeps_is_nonsymmetric(ref):
    import gwinputs as gi
    A, b, H = _nonsym_vcycle_problem(ref, gi)
    rng = np.random.default_rng(1)
    u, v = rng.standard_normal(A.n), rng.standard_normal(A.n)
    a, c = u @ H.vcycle(v), v @ H.vcycle(u)
    assert abs(a - c) > 1e-6 * abs(a)


def test_flexible_cg_directions_locally_a_orthogonal(ref):
    # Flexible CG's Polak-Ribiere beta = z_{k+1}.(r_{k+1} - r_k) / (z_k.r_k)
    # equals -z_{k+1}.A p_k / (p_k.A p_k) (since r_{k+1} - r_k = -alpha A p_k
    # and alpha = r_k.z_k / p_k.A p_k), so p_{k+1}.A p_k = 0 whatever the
    # preconditioner does (Notay's FCG(1) property).  The Fletcher-Reeves beta
    # r_{k+1}.z_{k+1} / r_k.z_k keeps it only for a symmetric preconditioner:
    # the plain-PCG run under the same nonsymmetric V-cycle shows the test can
    # tell the two apart.
    import gwinputs as gi
    A, b, H = _nonsym_vcycle_problem(ref, gi)
    As = A.to_scipy()

    def worst(dirs):
        w = 0.0
        for k in range(len(dirs) - 1):
            p0, p1 = dirs[k], dirs[k + 1]
            a01 = p1 @ (As @ p0)
            scale = np.sqrt((p0 @ (As @ p0)) * (p1 @ (As @ p1)))
            w = max(w, abs(a01) / scale)
        return w

    x, info, dirs = ref.pcg_directions(H, b, rtol=1e-10, flexible=True)
    assert info.status == ref.OK and len(dirs) >= 5
    assert worst(dirs) < 1e-10
    x2, info2, dirs2 = ref.pcg_directions(H, b, rtol=1e-10, flexible=False)
    assert len(dirs2) >= 5
    assert worst(dirs2) > 1e-4
    # the directions are those of the solve itself
    x3, info3 = ref.pcg(H, b, rtol=1e-10, flexible=True)
    assert np.array_equal(x, x3) and info3.iters == info.iters


def test_pmis_splitting_by_hand(ref):
    # Symmetric graph Laplacian + I, every off-diagonal -1, so every
    # connection is strong for theta <= 1 and a point's weight is its degree
    # plus a hash fraction < 1:
    #   X (0) with leaves 1-4 and neighbour Y: degree 5
    #   Z (5) with leaves 6-8 and neighbour Y: degree 4
    #   Y (9) neighbours X, Z, W: degree 3
    #   W (10) neighbours Y, V: degree 2;  V (11) neighbour W: degree 1
    # Round 1: X and Z beat every undecided neighbour -> C; Y and the leaves
    # depend on a C point -> F; W and V stay undecided (W loses to Y, V to W).
    # Round 2: W beats its only undecided neighbour V -> C; V -> F.
    # So C = {X, Z, W} for every hash seed.  (A C test against any neighbour
    # would also take Y; one against decided neighbours too would never take
    # W.)
    edges = [(0, j) for j in (1, 2, 3, 4)] + [(5, j) for j in (6, 7, 8)] + \
            [(0, 9), (5, 9), (9, 10), (10, 11)]
    n = 12
    A = np.eye(n)
    for i, j in edges:
        A[i, j] = A[j, i] = -1.0
        A[i, i] += 1.0
        A[j, j] += 1.0
    for seed in (1, 2, 3, 77, 12345):
        H = ref.Hierarchy(_csr(ref, A), ref.AmgParams(coarsening=ref.RS, eps_strong=0.25,
                                                      n_coarse=2, seed=seed))
        lv = H.level(0)
        c_points = set(np.flatnonzero(lv.state == ref.CF_C).tolist())
        assert c_points == {0, 5, 10}, seed
        assert lv.mis_rounds == 2


def test_breakdown_when_rhat_v_vanishes(ref):
    # Right-preconditioned BiCGSTAB with the identity preconditioner on
    # A = [[1, -3], [1, 1]], b = (1, 1): r_hat = r = p = b, v = A b = (-2, 2)
    # and r_hat.v = 0 exactly -> BREAKDOWN at the first alpha.  CG meets the
    # same zero in p.A p.  (The skew matrix [[0, 1], [-1, 0]] has the same
    # zero but no positive diagonal, which both setups reject.)
    A = _csr(ref, np.array([[1.0, -3.0], [1.0, 1.0]]))
    b = np.array([1.0, 1.0])
    H = ref.Hierarchy(A, ref.AmgParams(smoother=ref.NONE))
    x, info = ref.bicgstab(H, b)
    assert info.status == ref.BREAKDOWN and info.iters == 0
    x, info = ref.pcg(H, b)
    assert info.status == ref.BREAKDOWN and info.iters == 0
    with pytest.raises(ValueError):
        ref.Hierarchy(_csr(ref, np.array([[0.0, 1.0], [-1.0, 0.0]])), ref.AmgParams(smoother=ref.NONE))


def test_pmis_direction_of_dependence_by_hand(ref):
    # Nonsymmetric strength (theta 0.25): row 0 holds -1 toward 1, 2, 3 and
    # -10 toward 4, so S_0 = {4}; rows 1-4 hold -1 toward 0 (row 1 also -0.1
    # toward 5, too weak), so S_1 = ... = S_4 = {0}; row 5 holds -1 toward 1,
    # S_5 = {1}.  Dependents (points whose S holds the point): 0 has four
    # (1, 2, 3, 4), 1 and 4 one each, 2, 3, 5 none -> F at once.
    # Round 1: 0 (weight 4 + f) beats its undecided neighbours 1 and 4 -> C;
    # 1 and 4 depend on it -> F.  C = {0} after one round, for every seed.
    # (Making F the points a C point depends on would leave 1 undecided and
    # make it C in round 2; weighting by a point's own strong count would
    # give every point weight 1 + f and let the hash pick.)
    A = np.array([
        [14.0, -1.0, -1.0, -1.0, -10.0, 0.0],
        [-1.0, 2.0, 0.0, 0.0, 0.0, -0.1],
        [-1.0, 0.0, 2.0, 0.0, 0.0, 0.0],
        [-1.0, 0.0, 0.0, 2.0, 0.0, 0.0],
        [-1.0, 0.0, 0.0, 0.0, 2.0, 0.0],
        [0.0, -1.0, 0.0, 0.0, 0.0, 2.0],
    ])
    for seed in (1, 2, 3, 77, 12345):
        H = ref.Hierarchy(_csr(ref, A), ref.AmgParams(coarsening=ref.RS, eps_strong=0.25,
                                                      n_coarse=2, seed=seed))
        lv = H.level(0)
        assert np.flatnonzero(lv.state == ref.CF_C).tolist() == [0], seed
        assert lv.mis_rounds == 1
        # direct interpolation: F points 2-4 take their one strong C
        # neighbour with weight -(alpha a_i0)/d = 1/2 (alpha = -1/-1, d = 2);
        # row 1's alpha also counts its weak -0.1: (-1.1)/(-1), weight 0.55;
        # 5 has no strong C neighbour -> empty row
        P = lv.P.dense()
        assert np.allclose(P[:, 0], [1.0, 0.55, 0.5, 0.5, 0.5, 0.0], rtol=0, atol=1e-15)
