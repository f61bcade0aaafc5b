"""Pins for the oracle's tensor-train algebra (Section 3, Algorithm 1) and the TT step."""
import itertools
import math

import numpy as np
import pytest

from oracle import fv_grid, tt, tt_fv


def rand_tt(rng, n1, n2, r, decay=0.6):
    return tt.TT(rng.standard_normal((n1, r)) * decay ** np.arange(r), rng.standard_normal((n2, r)))


def test_round_equals_truncated_svd_of_full_matrix():
    """For two cores, rounding is the truncated SVD of the full matrix (Eckart-Young)."""
    rng = np.random.default_rng(0)
    for n1, n2, r in ((30, 20, 12), (15, 40, 25), (8, 8, 20)):
        X = rand_tt(rng, n1, n2, r)
        F = X.full()
        u, s, vt = np.linalg.svd(F)
        for eps, rmax in ((1e-3, 100), (1e-8, 5), (0.0, 100)):
            Y = tt.tt_round(X, eps, rmax)
            # brute-force rank choice
            k = 1
            while k < len(s) and math.sqrt(np.sum(s[k:] ** 2)) > eps * np.linalg.norm(s):
                k += 1
            k = min(k, rmax, r)            # at eps = 0 only the r nonzero values count
            assert Y.rank == k
            ref = (u[:, :k] * s[:k]) @ vt[:k]
            assert np.linalg.norm(Y.full() - ref) <= 1e-12 * np.linalg.norm(F)
            if k < rmax:
                assert np.linalg.norm(Y.full() - F) <= eps * np.linalg.norm(F) * (1 + 1e-9) + 1e-13


def test_round_idempotent_and_zero():
    rng = np.random.default_rng(1)
    X = tt.tt_round(rand_tt(rng, 20, 30, 6), 0.0, 100)
    Y = tt.tt_round(X, 1e-12, 100)
    assert Y.rank == X.rank
    assert np.allclose(Y.full(), X.full(), atol=1e-13)
    Z = tt.tt_round(tt.zero_tt(5, 7), 1e-10, 4)
    assert Z.rank == 1 and not np.any(Z.full())


def test_sum_hadamard_norm_against_elementwise():
    rng = np.random.default_rng(2)
    X, Y = rand_tt(rng, 11, 13, 4), rand_tt(rng, 11, 13, 3)
    assert np.allclose(tt.hadamard(X, Y).full(), X.full() * Y.full(), atol=1e-13)
    assert tt.hadamard(X, Y).rank == 12
    S = tt.add([(2.0, X), (-0.5, Y)])
    assert np.allclose(S.full(), 2 * X.full() - 0.5 * Y.full(), atol=1e-13)
    assert S.rank == 7
    shared = tt.TT(X.A * 3, X.B)
    S2 = tt.add([(1.0, X), (1.0, shared)])
    assert S2.rank == X.rank
    assert np.allclose(S2.full(), 4 * X.full(), atol=1e-13)
    assert abs(tt.tt_sum(X) - X.full().sum()) < 1e-12
    assert abs(tt.norm(X) - np.linalg.norm(X.full())) < 1e-12


def test_reciprocal_special_cases_and_bound():
    n1, n2 = 12, 9
    # constant input: x~ = 0, exact after the first term
    c = tt.TT(np.full((n1, 1), 2.5), np.ones((n2, 1)))
    y, err, terms = tt.reciprocal(c, 1e-12, 8, 10)
    assert np.allclose(y.full(), 0.4, atol=1e-15)
    # eps = 0, no cap: y is exactly the truncated geometric series sum_{k<K} x~^k / xbar
    rng = np.random.default_rng(4)
    x = tt.TT(np.concatenate([np.ones((n1, 1)), 0.1 * rng.standard_normal((n1, 2))], 1),
              np.concatenate([np.ones((n2, 1)), 0.3 * rng.standard_normal((n2, 2))], 1))
    F = x.full()
    xbar = F.mean()
    xt = 1 - F / xbar
    for K in (2, 4, 6):
        y, err, terms = tt.reciprocal(x, 0.0, K, 1000)
        series = sum(xt ** k for k in range(K)) / xbar
        assert terms == K
        assert np.allclose(y.full(), series, atol=1e-13)
        bound = np.abs(xt) ** K / ((1 - np.abs(xt)) * xbar)
        assert np.all(np.abs(y.full() - 1 / F) <= bound + 1e-13)
    # with a tolerance the loop stops once ||dy||/sqrt(N) <= eps
    y, err, terms = tt.reciprocal(x, 1e-6, 50, 1000)
    assert err <= 1e-6 and terms < 50


def test_reciprocal_detects_divergent_series():
    """x = 1/2 on half the rows and 9/2 on the other half has mean 5/2, so z = 1 - x/mean is
    4/5 and -4/5: the series converges (terms shrink by 4/5).  x = 8 on one row and 1 on the
    other nine has mean 17/10, so z = -63/17 on that row: its terms grow like (63/17)^k and
    the reciprocal must report divergence (reading R8), not a slow wrong answer."""
    n1, n2 = 10, 4
    col = np.full((n1, 1), 0.5)
    col[5:] = 4.5
    ok = tt.TT(col, np.ones((n2, 1)))
    y, err, terms = tt.reciprocal(ok, 1e-12, 200, 10)
    assert err <= 1e-12
    assert np.allclose(y.full(), 1.0 / ok.full(), rtol=1e-10)
    bad_col = np.ones((n1, 1))
    bad_col[0] = 8.0
    bad = tt.TT(bad_col, np.ones((n2, 1)))
    mean = bad.full().mean()
    assert np.max(np.abs(1.0 - bad.full() / mean)) > 1.0
    with pytest.raises(tt.SeriesDiverges):
        tt.reciprocal(bad, 1e-12, 200, 10)


def _vol(Q, rows):
    return abs(np.linalg.det(Q[list(rows)]))


def test_maxvol_against_brute_force():
    rng = np.random.default_rng(7)
    for trial in range(30):
        n = int(rng.integers(4, 13))
        r = int(rng.integers(1, 4))
        Q = np.linalg.qr(rng.standard_normal((n, r)))[0]
        I = tt.maxvol(Q, tau=1.0 + 1e-12, maxit=500)
        B = Q @ np.linalg.inv(Q[I])
        assert np.max(np.abs(B)) <= 1.0 + 1e-9            # dominance
        assert np.allclose(B[I], np.eye(r), atol=1e-10)
        best = max(_vol(Q, c) for c in itertools.combinations(range(n), r))
        if r == 1:
            assert _vol(Q, I) == pytest.approx(best)        # r = 1: exact argmax
        # a dominant set is a local maximum: no single swap increases the volume
        v = _vol(Q, I)
        for j in range(r):
            for i in range(n):
                J = list(I)
                J[j] = i
                assert _vol(Q, J) <= v * (1 + 1e-9)
        assert v >= best / (r ** (r / 2.0)) - 1e-12      # Goreinov et al. bound


def test_maxvol_returns_identity_block():
    rng = np.random.default_rng(8)
    r = 3
    A = 0.5 * (2 * rng.random((10, r)) - 1)
    A[[2, 5, 7]] = np.eye(r)
    I = tt.maxvol(A, tau=1.0 + 1e-12)
    assert sorted(I.tolist()) == [2, 5, 7]


class _Full:
    def __init__(self, F):
        self.F = F

    def cols(self, J):
        return self.F[:, J]

    def rows(self, I):
        return self.F[I, :]


def test_cross_reproduces_low_rank_and_full_rank():
    rng = np.random.default_rng(9)
    X = rand_tt(rng, 40, 35, 5, decay=0.8)
    F = X.full()
    Y, J = tt.cross(_Full(F), 40, 35, np.arange(3), 1e-14, 20, sweeps=3, kick=4, key=11)
    assert np.linalg.norm(Y.full() - F) < 1e-11 * np.linalg.norm(F)
    G = np.exp(-rng.random((9, 8)))
    Y, J = tt.cross(_Full(G), 9, 8, np.arange(8), 0.0, 100, sweeps=1, kick=0)
    assert np.allclose(Y.full(), G, atol=1e-12)


def test_splitmix64_reference_outputs():
    s, a = tt.splitmix64(0)
    s, b = tt.splitmix64(s)
    assert a == 0xE220A8397B1DCDAF
    assert b == 0x6E789E6AA1B965F4
    k = tt.kick_indices([0, 1, 2], 10, 4, key=123)
    assert len(set(k)) == 4 and not set(k) & {0, 1, 2}
    assert k == tt.kick_indices([0, 1, 2], 10, 4, key=123)


def _svd_tt(U):
    u, s, vt = np.linalg.svd(U)
    return tt.TT(u * s, vt.T)


@pytest.mark.parametrize("scheme,nonlinear,periodic", [
    ("upwind3", False, True), ("upwind5", False, True), ("upwind3", True, False),
    ("upwind5", True, True), ("upwind5", True, False), ("weno5", True, True), ("weno5", True, False)])
def test_tt_step_equals_grid_step_at_full_rank(scheme, nonlinear, periodic):
    """With eps = 0, no rank cap, Taylor run to round-off and full-rank crosses, the TT step
    is the full-grid step (the whole fixed sequence of TT operations against the definition)."""
    n = 10
    x = (np.arange(n) + 0.5) / n
    if nonlinear:
        h = 1 + 0.02 * np.outer(np.cos(2 * np.pi * x), np.sin(2 * np.pi * x + 0.3)) \
            + 0.01 * np.outer(np.sin(4 * np.pi * x), np.ones(n))
        hu = 0.03 * np.outer(np.sin(2 * np.pi * x + 0.1), np.cos(2 * np.pi * x))
        hv = 0.02 * np.outer(np.cos(2 * np.pi * x), np.cos(4 * np.pi * x + 0.2))
        U = [h, hu, hv]
    else:
        U = [0.01 * np.outer(np.cos(2 * np.pi * x), np.sin(2 * np.pi * x)),
             0.01 * np.outer(np.sin(2 * np.pi * x), np.ones(n)),
             0.001 * np.outer(np.ones(n), np.cos(2 * np.pi * x))]
    gs = fv_grid.GridSolver(n, scheme, nonlinear, periodic)
    ts = tt_fv.TTSolver(n, scheme, nonlinear, periodic, eps=0.0, rmax=10 ** 6, taylor_terms=30,
                        cross_full=True)
    Ug = gs.step(U, 1e-3)
    Qt = ts.step([_svd_tt(u) for u in U], 1e-3)
    for q, u in zip(Qt, Ug):
        assert np.linalg.norm(q.full() - u) <= 1e-12 * np.linalg.norm(u)


def test_linear_gaussian_tt_run_tracks_grid_run():
    """The 64^2 linear Gaussian at rank cap 8, tol 1e-12: TT compression error stays small."""
    import synth
    st = synth.linear_gaussian(seed=0)
    gs = fv_grid.GridSolver(st.n, "upwind3", False, True, g=st.g, H=st.H0)
    ts = tt_fv.TTSolver(st.n, "upwind3", False, True, g=st.g, H=st.H0, eps=1e-12, rmax=8)
    Q = [tt.TT(f.A, f.B) for f in st.tt]
    U = st.fields
    for _ in range(10):
        U = gs.step(U, st.dt)
        Q = ts.step(Q, st.dt)
    rel = np.linalg.norm(Q[0].full() - U[0]) / np.linalg.norm(U[0])
    assert rel < 1e-3
    assert all(r <= 8 for r in ts.stats["ranks"][-1])


@pytest.mark.parametrize("scheme", ["upwind5", "weno5"])
def test_tt_step_with_cross_reciprocal_equals_grid_step(scheme):
    """1/h by a full-rank cross of 1/x (Section 4.2's alternative to Algorithm 1) reproduces the
    grid step on a dam break with walls, where the Taylor series would diverge."""
    import synth
    st = synth.dam_break(seed=1, n=12, rmax=12, eps=0.0, width=0.1)
    U = st.fields
    xt = 1 - U[0] / U[0].mean()
    assert np.max(np.abs(xt)) > 0.3
    gs = fv_grid.GridSolver(12, scheme, True, False)
    ts = tt_fv.TTSolver(12, scheme, True, False, eps=0.0, rmax=10 ** 6, cross_full=True,
                        recip="cross")
    Ug = gs.step(U, 1e-3)
    Qt = ts.step([_svd_tt(u) for u in U], 1e-3)
    for q, u in zip(Qt, Ug):
        if np.linalg.norm(u) > 0:
            assert np.linalg.norm(q.full() - u) <= 1e-11 * np.linalg.norm(Ug[0])


def test_tt_lambda_entries_hand_values():
    """The lambda cross function of the TT step (Section 4.2, LLF flux) on constant rank-1 TTs,
    g = 4: minus state (h, hu, hv) = (1, 1/2, -3), plus state (1/4, -1/2, 1/4).  In x the
    momentum is hu: max(1/2 + 2, 2 + 1) = 3; in y (the step passes hv as the momentum)
    max(3 + 2, 1 + 1) = 5.  A missing |.|, a one-sided speed or g h in place of sqrt(g h)
    changes one of them."""
    n1, n2 = 5, 7

    def const(c):
        return tt.TT(np.full((n1, 1), c), np.ones((n2, 1)))

    hm, hp = const(1.0), const(0.25)
    lx = tt_fv._Lambda(hm, const(0.5), hp, const(-0.5), 4.0)
    ly = tt_fv._Lambda(hm, const(-3.0), hp, const(0.25), 4.0)
    assert np.all(lx.cols(np.array([0, 3])) == 3.0) and np.all(lx.rows(np.array([1])) == 3.0)
    assert np.all(ly.cols(np.array([2])) == 5.0) and np.all(ly.rows(np.array([0, 4])) == 5.0)


def test_lf_cross_equals_full_grid_and_product_flux():
    """LF-cross (the whole LLF flux vector of a direction by one cross, Section 4.2's
    alternative): with full-rank crosses it equals the full-grid scheme, and at a working
    tolerance it agrees with the product flux to that tolerance."""
    import math
    import synth
    from oracle import fv_grid
    from oracle.tt import TT
    from oracle.tt_fv import TTSolver
    st = synth.nonlinear_bumps(seed=3, n=12, rmax=12, eps=1e-14, kmax=2)
    Q0 = [TT(x.A, x.B) for x in st.tt]
    grid = fv_grid.GridSolver(12, "upwind5", True, periodic=True, g=st.g)
    U = grid.run([x.copy() for x in st.fields], st.dt, 2)
    s = TTSolver(12, "upwind5", True, True, g=st.g, eps=0.0, rmax=64, cross_full=True,
                 flux="lf_cross")
    Q = s.run(Q0, st.dt, 2)
    rel = math.sqrt(sum(float(np.sum((q.A @ q.B.T - u) ** 2)) for q, u in zip(Q, U)) /
                    sum(float(np.sum(u * u)) for u in U))
    assert rel < 1e-12, rel
    st = synth.nonlinear_bumps(seed=4, n=48, rmax=16, eps=1e-10, kmax=3)
    Q0 = [TT(x.A, x.B) for x in st.tt]
    a = TTSolver(48, "upwind5", True, True, g=st.g, eps=1e-9, rmax=32, flux="lf_cross")
    b = TTSolver(48, "upwind5", True, True, g=st.g, eps=1e-9, rmax=32)
    Qa, Qb = a.run(Q0, st.dt, 2), b.run(Q0, st.dt, 2)
    for qa, qb in zip(Qa, Qb):
        Fa, Fb = qa.A @ qa.B.T, qb.A @ qb.B.T
        assert np.linalg.norm(Fa - Fb) <= 1e-7 * np.linalg.norm(Fb)


def test_from_full_closed_form():
    """from_full on F = U diag(s) V^T with a known spectrum: the kept rank is the smallest whose
    discarded tail is within eps (from s alone), and the error equals that tail exactly
    (Eckart-Young); a zero matrix gives rank 1 and zero."""
    from oracle.tt import from_full
    rng = np.random.default_rng(11)
    n1, n2, r = 60, 45, 30
    U, _ = np.linalg.qr(rng.standard_normal((n1, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n2, r)))
    s = 0.7 ** np.arange(r)
    F = (U * s) @ V.T
    for eps in (1e-1, 1e-3, 1e-6):
        tail = np.sqrt(np.cumsum((s * s)[::-1])[::-1])
        k = int(np.argmax(np.append(tail[1:], 0.0) <= eps * np.linalg.norm(s))) + 1
        X = from_full(F, eps, 64)
        assert X.rank == k
        assert np.linalg.norm(F - X.A @ X.B.T) == pytest.approx(
            np.sqrt(np.sum(s[k:] ** 2)), rel=1e-9, abs=1e-14)
    assert from_full(F, 0.0, 5).rank == 5
    Z = from_full(np.zeros((7, 9)), 1e-8, 4)
    assert Z.rank == 1 and not np.any(Z.A @ Z.B.T)


def test_rook_max_speed():
    """The CFL speed estimate by rook pivoting on the TTs: never above the true maximum of
    |m/h| + sqrt(g h) over the cells, equal to it on smooth fields, and exact on a rank-1
    field whose maximum sits where the starting columns do not look."""
    import synth
    from oracle.tt import TT
    from oracle.tt_fv import TTSolver, _Lambda, rook_max
    for seed in range(4):
        st = synth.nonlinear_bumps(seed=seed, n=64, rmax=24, eps=1e-12, kmax=4)
        Q = [TT(x.A, x.B) for x in st.tt]
        s = TTSolver(64, "upwind5", True, True, g=st.g)
        h, hu, hv = [q.A @ q.B.T for q in Q]
        for d, m in ((0, hu), (1, hv)):
            true = float(np.max(np.abs(m / h) + np.sqrt(st.g * h)))
            est = s.max_speed(Q, d)
            assert est <= true * (1 + 1e-14)
            assert est == pytest.approx(true, rel=1e-12)
        assert s.cfl_dt(Q, 0.4) == pytest.approx(st.dt, rel=1e-12)
    # rank-1 h with a single peak away from column 0; m = 0
    n = 40
    x = np.exp(-((np.arange(n) - 29.0) / 3.0) ** 2)
    h = TT((1.0 + x)[:, None], (1.0 + 0.5 * x[::-1])[:, None])
    z = TT(np.zeros((n, 1)), np.zeros((n, 1)))
    val, i, j = rook_max(_Lambda(h, z, h, z, 9.81), n, n, np.array([0]))
    full = np.sqrt(9.81 * (h.A @ h.B.T))
    assert val == pytest.approx(float(full.max()), rel=1e-15)


def test_residual_enrichment_finds_a_localised_feature():
    """Residual-based enrichment keeps the candidate columns the current skeleton fits worst:
    on a smooth rank-3 matrix plus a narrow bump in 6 of 400 columns, crosses started from the
    smooth part recover the bump more often with it than with seeded kicks (same key, sweeps
    and number of added columns), and each added column is the worst-fitted candidate."""
    from oracle.tt import cross, kick_indices, orth, maxvol, residual_columns

    class Mat:
        def __init__(self, F):
            self.F = F

        def cols(self, J):
            return self.F[:, np.asarray(J)]

        def rows(self, I):
            return self.F[np.asarray(I), :]

    n1, n2 = 300, 400
    x = np.linspace(0, 1, n1)[:, None]
    y = np.linspace(0, 1, n2)[None, :]
    smooth = np.sin(3 * x + 2 * y) + 0.5 * np.cos(5 * x) * np.sin(4 * y) + x * y
    bump = np.exp(-((x - 0.7) / 0.02) ** 2) * (np.abs(y - 0.33) < 0.007)
    F = smooth + 1e-3 * bump
    fun = Mat(F)
    J0 = np.array([0, 133, 266, 399])
    wins = {"random": 0, "residual": 0}
    for key in range(12):
        for mode in wins:
            X, _ = cross(fun, n1, n2, J0, 1e-12, 20, sweeps=3, kick=4, key=key, enrich=mode)
            err = np.linalg.norm(F - X.A @ X.B.T) / np.linalg.norm(F)
            wins[mode] += err < 1e-9
    assert wins["residual"] > wins["random"], wins
    # the chosen columns are the worst-fitted candidates
    C = fun.cols(J0)
    Qc = orth(C)
    I = maxvol(Qc)
    R = fun.rows(I)
    got = residual_columns(fun, Qc, I, R, list(J0), n2, 3, 77)
    cand = kick_indices(list(J0), n2, 12, 77)
    res = np.linalg.norm(F[:, cand] - Qc @ np.linalg.solve(Qc[I], R[:, cand]), axis=0)
    assert got == [cand[t] for t in np.argsort(-res, kind="stable")[:3]]


def test_gauss_sketch_generator_and_sketched_rounding():
    """The seeded sketch: entries come from SplitMix64's output function (pinned by its
    published first output through tt.splitmix64) and Box-Muller, so their moments are those of
    a standard normal; and the sketched rounding of a rank-300 TT whose spectrum decays agrees
    with the exact rounding to the leak bound."""
    from oracle.tt import TT, gauss_sketch, splitmix64, tt_round, tt_round_sketched
    # entry (0, 0) with seed s: h1 = mix64(s ^ golden); SplitMix64 from state 0 outputs
    # mix64(golden) first, so with s = 0 the h1 of entry 0 is that published output
    golden, mask = 0x9E3779B97F4A7C15, (1 << 64) - 1
    s0, first = splitmix64(0)                         # published: 0xE220A8397B1DCDAF
    _, h2 = splitmix64((first + 0x632BE59BD9B4E019 - golden) & mask)
    u1 = ((first >> 11) + 1.0) / 9007199254740993.0
    u2 = (h2 >> 11) / 9007199254740992.0
    G = gauss_sketch(4, 3, 0)
    assert np.isfinite(G).all()
    assert G[0, 0] == pytest.approx(math.sqrt(-2.0 * math.log(u1)) * math.cos(2 * math.pi * u2),
                                    rel=1e-15)
    big = gauss_sketch(20000, 5, 1234)
    assert abs(big.mean()) < 0.02 and abs(big.std() - 1.0) < 0.02
    assert abs(np.mean(big ** 4) - 3.0) < 0.1
    rng = np.random.default_rng(8)
    A = rng.standard_normal((400, 300)) * (0.9 ** np.arange(300))[None, :]
    B = rng.standard_normal((500, 300))
    X = TT(A, B)
    Ys, Ye = tt_round_sketched(X, 1e-6, 32), tt_round(X, 1e-6, 32)
    F = A @ B.T
    assert Ys.rank == Ye.rank
    assert np.linalg.norm(Ys.A @ Ys.B.T - Ye.A @ Ye.B.T) <= 1e-10 * np.linalg.norm(F)
