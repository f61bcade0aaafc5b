"""GPU parity of each TT primitive against the CPU oracle (called through the C ABI)."""
import math
import sys

import numpy as np
import pytest

from oracle import tt as ott
from oracle import tt_fv as otf

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_03483_amd import ttfv
    ttfv.load_library()
    return ttfv


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.tt_ctx_create(1 << 30)
    yield c
    c.close()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def decaying_tt(rng, n1, n2, r, decay=0.7):
    A = rng.standard_normal((n1, r)) * decay ** np.arange(r)
    B = rng.standard_normal((n2, r))
    return A, B


@pytest.mark.parametrize("scheme", [3, 5])
@pytest.mark.parametrize("periodic", [True, False])
def test_recon_core_parity(lib, ctx, scheme, periodic):
    import torch
    _say(f"recon scheme={scheme} periodic={periodic}")
    rng = np.random.default_rng(0)
    n, r = 333, 7
    core = rng.standard_normal((n, r))
    sign = -1.0
    fm, fp, q = lib.tt_recon_core(ctx, torch.from_numpy(core.T.copy()).cuda(), scheme, periodic,
                                  sign)
    name = {3: "upwind3", 5: "upwind5"}[scheme]
    s = otf.TTSolver(n, name, True, periodic)
    m_ref, p_ref = s.face_cores(core, sign)
    q_ref = s.quad_core(core, sign)
    assert np.max(np.abs(fm.T.cpu().numpy() - m_ref)) < 1e-14
    assert np.max(np.abs(fp.T.cpu().numpy() - p_ref)) < 1e-14
    assert np.max(np.abs(q.T.cpu().numpy() - q_ref)) < 1e-14


@pytest.mark.parametrize("n1,n2,r,eps,rmax", [
    (300, 200, 20, 1e-10, 32),      # exact path, rank from tolerance
    (1000, 3000, 40, 1e-10, 8),     # exact path, cap binds
    (1000, 3000, 300, 1e-10, 32),   # randomized path (R > sketch width)
    (777, 1531, 1024, 1e-12, 16),   # randomized path, ragged sizes
    (50, 40, 200, 0.0, 64),         # tiny modes: materialised
    (3001, 2503, 400, 1e-12, 64),   # widest sketch (96 columns: two columns per lane group)
    (2049, 6144, 90, 1e-12, 64),    # exact path at 90 columns (192-row blocks)
])
def test_round_parity(lib, ctx, n1, n2, r, eps, rmax):
    _say(f"round {n1}x{n2} r={r} eps={eps} rmax={rmax}")
    rng = np.random.default_rng(1)
    A, B = decaying_tt(rng, n1, n2, r, decay=0.8)
    x = lib.DeviceTT.from_factors(A, B)
    y = lib.DeviceTT(n1, n2, rmax)
    w, sig = lib.tt_round(ctx, x, eps, rmax, y)
    ref = ott.tt_round(ott.TT(A, B), eps, rmax)
    assert y.rank == ref.rank
    F = A @ B.T
    assert rel(y.full(), ref.full()) < 1e-10
    # singular values of the kept part agree with the exact ones
    s_ref = np.linalg.svd(ref.A, compute_uv=False) * 0 + np.linalg.norm(ref.A, axis=0)
    assert np.allclose(sig, s_ref, rtol=1e-9, atol=1e-12 * np.linalg.norm(F))


@pytest.mark.parametrize("n1,n2,r,eps,rmax", [
    (300, 200, 20, 1e-6, 32),       # exact path
    (1000, 3000, 300, 1e-6, 32),    # randomized path
    (777, 1531, 1024, 1e-5, 16),    # randomized path, ragged sizes
    (3001, 2503, 400, 1e-6, 64),    # widest sketch (96 columns)
])
def test_round_fp32_contractions(lib, n1, n2, r, eps, rmax):
    """FP32 contractions (GEMMs and QR panels on the matrix cores, SVD in FP64): the result
    is within the FP32 noise (1e-5 relative) of the FP64 oracle's rounding."""
    _say(f"round fp32 {n1}x{n2} r={r} eps={eps} rmax={rmax}")
    c = lib.tt_ctx_create(1 << 30)
    lib.tt_ctx_set_precision(c, "f32")
    rng = np.random.default_rng(1)
    A, B = decaying_tt(rng, n1, n2, r, decay=0.8)
    x = lib.DeviceTT.from_factors(A, B)
    y = lib.DeviceTT(n1, n2, rmax)
    lib.tt_round(c, x, eps, rmax, y)
    c.close()
    ref = ott.tt_round(ott.TT(A, B), eps, rmax)
    F = A @ B.T
    assert y.rank <= rmax
    e = np.linalg.norm(y.full() - ref.full()) / np.linalg.norm(F)
    _say(f"  ranks gpu {y.rank} oracle {ref.rank}, rel diff {e:.2e}")
    assert e < 1e-5


@pytest.mark.parametrize("eps", [0.0, 1e-20, 1e-17])
@pytest.mark.parametrize("r", [4, 12, 30])
def test_round_below_round_off_of_a_rank_deficient_sum(lib, ctx, eps, r):
    """A tolerance below round-off on a sum whose concatenated cores are rank deficient (the
    state of a linear step at a fine grid under Section 4.4's rule, where the formula asks for
    1e-18 or less): the rounding keeps every direction the SVD resolved and none of the
    unresolved noise, so the result is X to round-off, not a garbled projection."""
    _say(f"round below round-off r={r} eps={eps}")
    rng = np.random.default_rng(7 + r)
    n1, n2 = 700, 900
    A = rng.standard_normal((n1, r)) * (0.7 ** np.arange(r))[None, :]
    B = rng.standard_normal((n2, r))
    # x = A B^T + 0.5 A (2B)^T - 1.5 A B^T + A B^T = 1.5 A B^T: exact rank r from 4 r columns
    Ac = np.concatenate([A, 0.5 * A, -1.5 * A, A], axis=1)
    Bc = np.concatenate([B, 2.0 * B, B, B], axis=1)
    x = lib.DeviceTT.from_factors(Ac, Bc)
    rmax = min(4 * r, 64)
    y = lib.DeviceTT(n1, n2, rmax)
    lib.tt_round(ctx, x, eps, rmax, y)
    F = 1.5 * (A @ B.T)
    e = rel(y.full(), F)
    _say(f"  rank {y.rank}, rel error {e:.2e}")
    assert e < 1e-13


@pytest.mark.parametrize("m", [1, 7, 17, 33, 63, 65, 81, 96])
def test_round_full_rank_orthonormal_factor(lib, ctx, m):
    """Full-rank rounding (eps = 0, r_max = m) takes the exact path: two TSQRs (leaves of 250
    or 171 rows, node levels, the compact-WY top-down pass) and the SVD of Ra Rb^T.  The TT is
    reproduced to round-off, the first output core is orthonormal, and the singular values
    match LAPACK's."""
    _say(f"full-rank round m={m}")
    rng = np.random.default_rng(100 + m)
    n1, n2 = 1000, 4097
    Ua, _ = np.linalg.qr(rng.standard_normal((n1, m)))
    Ub, _ = np.linalg.qr(rng.standard_normal((n2, m)))
    s = np.logspace(0, -3, m)
    A, B = Ua * s, Ub
    x = lib.DeviceTT.from_factors(A, B)
    y = lib.DeviceTT(n1, n2, m)
    _, sig = lib.tt_round(ctx, x, 0.0, m, y)
    assert y.rank == m
    Ay, By = y.factors()
    assert np.max(np.abs(Ay.T @ Ay - np.eye(m))) < 1e-12
    assert rel(Ay @ By.T, A @ B.T) < 1e-12
    assert np.allclose(sig, s, rtol=1e-12, atol=0)


def test_round_with_gemm_autotune(lib, ctx):
    """With the tile-shape autotuner on, every candidate shape gives the same rounding (to the
    oracle's tolerance), and a second call of a tuned class reuses the stored choice."""
    _say("round with GEMM autotune")
    rng = np.random.default_rng(3)
    try:
        n0 = lib.tt_gemm_autotune(True)
        for n1, n2, r, eps, rmax in ((1000, 3000, 300, 1e-10, 32), (2049, 6144, 90, 1e-12, 64)):
            A, B = decaying_tt(rng, n1, n2, r, decay=0.8)
            x = lib.DeviceTT.from_factors(A, B)
            ref = ott.tt_round(ott.TT(A, B), eps, rmax)
            outs = []
            for _ in range(2):
                y = lib.DeviceTT(n1, n2, rmax)
                lib.tt_round(ctx, x, eps, rmax, y)
                assert y.rank == ref.rank
                assert rel(y.full(), ref.full()) < 1e-10
                outs.append(y.full())
            n1c = lib.tt_gemm_autotune(True)
            assert n1c > n0
            n0 = n1c
            assert rel(outs[0], outs[1]) < 1e-13      # the same tiles on the second call
    finally:
        lib.tt_gemm_autotune(False)


def test_hadamard_round_parity(lib, ctx):
    _say("hadamard")
    rng = np.random.default_rng(2)
    n1, n2 = 1024, 3072
    x = np.linspace(0, 1, n1)[:, None]
    y = np.linspace(0, 1, n2)[:, None]
    k1 = np.arange(1, 25)[None, :]
    A1 = np.cos(np.pi * k1 * x) * (0.6 ** k1)
    B1 = np.sin(np.pi * k1 * y + 0.3)
    A2 = np.cos(np.pi * k1 * x + 0.1) * (0.5 ** k1)
    B2 = np.cos(np.pi * k1 * y)
    X = lib.DeviceTT.from_factors(A1, B1)
    Z = lib.DeviceTT.from_factors(A2, B2)
    Y = lib.DeviceTT(n1, n2, 32)
    lib.tt_hadamard_round(ctx, X, Z, 1e-10, 32, Y)
    ref = ott.tt_round(ott.hadamard(ott.TT(A1, B1), ott.TT(A2, B2)), 1e-10, 32)
    assert Y.rank == ref.rank
    assert rel(Y.full(), ref.full()) < 1e-10


def test_reciprocal_parity(lib, ctx):
    _say("reciprocal")
    import synth
    rng = np.random.default_rng(3)
    f = synth.smooth_factored(rng, 900, 2700, 6, base=1.0)
    X = lib.DeviceTT.from_factors(f.A, f.B)
    Y = lib.DeviceTT(900, 2700, 32)
    w, err, terms = lib.tt_reciprocal(ctx, X, 1e-10, 8, 32, Y)
    ref, err_r, terms_r = ott.reciprocal(ott.TT(f.A, f.B), 1e-10, 8, 32)
    assert terms == terms_r
    assert abs(err - err_r) <= 1e-6 * err_r + 1e-15
    assert rel(Y.full(), ref.full()) < 1e-10


def test_maxvol_parity(lib, ctx):
    import torch
    _say("maxvol")
    rng = np.random.default_rng(4)
    for n, r in ((1000, 16), (3001, 40), (64, 64), (200, 1)):
        Q = np.linalg.qr(rng.standard_normal((n, r)))[0]
        I = lib.tt_maxvol(ctx, torch.from_numpy(Q.T.copy()).cuda(), 1.05, 100)
        I_ref = ott.maxvol(Q, 1.05, 100)
        assert sorted(I.tolist()) == sorted(I_ref.tolist())
        B = Q @ np.linalg.inv(Q[I])
        assert np.max(np.abs(B)) <= 1.05 + 1e-12


@pytest.mark.parametrize("r,rmax,ncols", [(6, 16, 3), (50, 64, 52), (40, 64, 64)])
def test_cross_identity_reproduces_low_rank(lib, ctx, r, rmax, ncols):
    """With 52 and 64 start columns the orthogonalisations of the cross take the pivoted-QR
    SVD path (m >= 48); the graded spectrum (0.8^i) is what that path is for."""
    _say(f"cross identity r={r}")
    rng = np.random.default_rng(5)
    A, B = decaying_tt(rng, 700, 900, r, decay=0.9 if r < 10 else 0.8)
    X = lib.DeviceTT.from_factors(A, B)
    Y = lib.DeviceTT(700, 900, rmax)
    J0 = list(range(0, 900, 900 // ncols))[:ncols]
    w, J = lib.tt_cross(ctx, lib.TT_FN_IDENTITY, [X], [], 700, 900, J0, 1e-13, rmax, 3, 4,
                        7, Y)
    assert rel(Y.full(), A @ B.T) < 1e-11


def test_cross_lambda_parity(lib, ctx):
    _say("cross lambda")
    import synth
    rng = np.random.default_rng(6)
    n1, n2 = 256, 768
    fh = synth.smooth_factored(rng, n1, n2, 5, base=1.0)
    fm = synth.smooth_factored(rng, n1, n2, 7, base=0.0)
    fh2 = synth.smooth_factored(rng, n1, n2, 5, base=1.0)
    fm2 = synth.smooth_factored(rng, n1, n2, 7, base=0.0)
    T = [ott.TT(f.A, f.B) for f in (fh, fm, fh2, fm2)]
    D = [lib.DeviceTT.from_factors(f.A, f.B) for f in (fh, fm, fh2, fm2)]
    g = 9.81
    fun = otf._Lambda(T[0], T[1], T[2], T[3], g)
    J0 = ott.initial_columns(T[1])
    ref, J_ref = ott.cross(fun, n1, n2, J0, 1e-10, 32, 3, 4, key=99)
    Y = lib.DeviceTT(n1, n2, 32)
    w, J = lib.tt_cross(ctx, lib.TT_FN_LLF_LAMBDA, D, [g], n1, n2, J0.tolist(), 1e-10, 32, 3, 4,
                        99, Y)
    assert sorted(J.tolist()) == sorted(J_ref.tolist())
    assert Y.rank == ref.rank
    assert rel(Y.full(), ref.full()) < 1e-9


def test_cross_lambda_hand_values(lib, ctx):
    """The device lambda function (Section 4.2, LLF) on constant rank-1 TTs, g = 4: minus state
    (h, m) = (1, 1/2), plus (1/4, -1/2) gives max(1/2 + 2, 2 + 1) = 3; with the momenta
    -3 and 1/4 it gives max(3 + 2, 1 + 1) = 5 (the values derived by hand for the oracle)."""
    _say("cross lambda hand values")
    n1, n2 = 40, 30

    def const(c):
        return lib.DeviceTT.from_factors(np.full((n1, 1), c), np.ones((n2, 1)))

    hm, hp = const(1.0), const(0.25)
    for mm, mp, want in ((0.5, -0.5, 3.0), (-3.0, 0.25, 5.0)):
        Y = lib.DeviceTT(n1, n2, 4)
        lib.tt_cross(ctx, lib.TT_FN_LLF_LAMBDA, [hm, const(mm), hp, const(mp)], [4.0], n1, n2,
                     [0], 1e-12, 4, 1, 0, 1, Y)
        assert Y.rank == 1
        assert np.max(np.abs(Y.full() - want)) <= 1e-13 * want


def test_cross_skeleton_replays_oracle_pivots(lib, ctx):
    """Given the oracle's final column and row sets of a capped lambda cross (Section 3.3), the
    device skeleton equals the oracle's: the skeleton is fixed by its pivots."""
    _say("cross skeleton from oracle pivots")
    import synth
    rng = np.random.default_rng(16)
    n1, n2 = 300, 900
    fs = [synth.smooth_factored(rng, n1, n2, 9, base=b) for b in (1.0, 0.0, 1.0, 0.0)]
    T = [ott.TT(f.A, f.B) for f in fs]
    D = [lib.DeviceTT.from_factors(f.A, f.B) for f in fs]
    fun = otf._Lambda(T[0], T[1], T[2], T[3], 9.81)
    rows = []
    ref, J = ott.cross(fun, n1, n2, ott.initial_columns(T[1]), 1e-10, 12, 3, 4, key=3,
                       rows_out=rows)
    I = rows[0]
    assert len(I) >= 8                       # the cap binds: many valid pivot sets exist
    Y = lib.DeviceTT(n1, n2, 12)
    lib.tt_cross_skeleton(ctx, lib.TT_FN_LLF_LAMBDA, D, [9.81], n1, n2, J.tolist(), I.tolist(),
                          1e-10, 12, Y)
    assert Y.rank == ref.rank
    e = rel(Y.full(), ref.full())
    _say(f"  rank {Y.rank}, rel {e:.2e}")
    assert e < 1e-10


@pytest.mark.parametrize("periodic", [True, False])
def test_cross_weno_parity(lib, ctx, periodic):
    _say(f"cross weno periodic={periodic}")
    from oracle import stencils
    rng = np.random.default_rng(7)
    n = 96
    x = (np.arange(n) + 0.5) / n
    h = 1 + 0.5 * np.tanh((0.3 - np.sqrt((x[:, None] - 0.45) ** 2 + (x[None, :] - 0.55) ** 2))
                         / 0.05)
    u, s, vt = np.linalg.svd(h)
    k = int(np.sum(s > 1e-10 * s[0]))
    q = ott.TT(u[:, :k] * s[:k], vt[:k].T)
    tab = stencils.tables("weno5")
    nf = n if periodic else n + 1
    eps_w = (1.0 / n) ** 2
    sign = -1.0
    for side, fn in ((-1, lib.TT_FN_WENO_FACE_M), (1, lib.TT_FN_WENO_FACE_P)):
        fun = otf._WenoFace(q, periodic, sign, side, nf, tab, eps_w)
        J0 = ott.initial_columns(q)
        ref, J_ref = ott.cross(fun, nf, n, J0, 1e-10, 64, 3, 4, key=5)
        Y = lib.DeviceTT(nf, n, 64)
        X = lib.DeviceTT.from_factors(q.A, q.B)
        w, J = lib.tt_cross(ctx, fn, [X], [1.0 if periodic else 0.0, sign, eps_w], nf, n,
                            J0.tolist(), 1e-10, 64, 3, 4, 5, Y)
        assert rel(Y.full(), ref.full()) < 1e-8
    # step 2 on a face TT
    v = ott.TT(rng.standard_normal((nf, 4)) * 0.1 + 1.0, np.cos(np.outer(x, np.arange(4))))
    fun = otf._WenoQuad(v, periodic, sign, n, tab, eps_w)
    y0 = ott.TT(v.A, np.repeat(v.B, 3, axis=0))
    J0 = ott.initial_columns(y0)
    ref, _ = ott.cross(fun, nf, 3 * n, J0, 1e-10, 64, 3, 4, key=9)
    Y = lib.DeviceTT(nf, 3 * n, 64)
    X = lib.DeviceTT.from_factors(v.A, v.B)
    w, J = lib.tt_cross(ctx, lib.TT_FN_WENO_QUAD, [X], [1.0 if periodic else 0.0, sign, eps_w],
                        nf, 3 * n, J0.tolist(), 1e-10, 64, 3, 4, 9, Y)
    assert rel(Y.full(), ref.full()) < 1e-8


def test_error_paths(lib, ctx):
    _say("errors")
    X = lib.DeviceTT(10, 10, 2)
    X.rank = 3                      # rank above capacity
    Y = lib.DeviceTT(10, 10, 4)
    with pytest.raises(RuntimeError, match="rank"):
        lib.tt_round(ctx, X, 1e-10, 4, Y)
    X.rank = 1
    with pytest.raises(RuntimeError, match="cap"):
        lib.tt_round(ctx, X, 1e-10, 8, Y)


# ---- failure detection, each condition forced from the host ---------------------------

def _spectrum_tt(rng, n1, n2, R, decay):
    """A TT of rank R with singular values decay^i (orthonormal factors)."""
    qa, _ = np.linalg.qr(rng.standard_normal((n1, R)))
    qb, _ = np.linalg.qr(rng.standard_normal((n2, R)))
    return qa * decay ** np.arange(R), qb


def test_round_sketch_limit_redone_exactly(lib):
    """A slowly decaying spectrum (0.97^i, rank 80 > the 32-column sketch of r_max 16) keeps
    the discarded directions leaking past the subspace-iteration limit; at rank <= 96 the
    rounding is then redone exactly, so it must equal the oracle's truncated SVD."""
    _say("round: unconverged sketch redone exactly")
    rng = np.random.default_rng(21)
    A, B = _spectrum_tt(rng, 700, 500, 80, 0.97)
    c = lib.tt_ctx_create(1 << 28)
    for limit in (8, 0):
        lib.tt_ctx_set_limits(c, 40, limit)
        X = lib.DeviceTT.from_factors(A, B)
        Y = lib.DeviceTT(700, 500, 16)
        w, _ = lib.tt_round(c, X, 1e-10, 16, Y)
        ref = ott.tt_round(ott.TT(A, B), 1e-10, 16)
        assert w & lib.TT_WRANKCAP and not (w & lib.TT_WSKETCH)
        assert rel(Y.full(), ref.full()) < 1e-10
    c.close()


def test_round_sketch_unconverged_warns(lib):
    """The same spectrum at rank 200 (beyond the exact path's 96 columns): the rounding keeps
    the sketch's answer and returns TT_WSKETCH; its error stays within a few times the optimal
    truncation error."""
    _say("round: unconverged sketch warning")
    rng = np.random.default_rng(22)
    A, B = _spectrum_tt(rng, 700, 500, 200, 0.97)
    c = lib.tt_ctx_create(1 << 28)
    X = lib.DeviceTT.from_factors(A, B)
    Y = lib.DeviceTT(700, 500, 16)
    w, _ = lib.tt_round(c, X, 1e-10, 16, Y)
    F = A @ B.T
    best = np.linalg.norm(F - ott.tt_round(ott.TT(A, B), 1e-10, 16).full())
    got = np.linalg.norm(F - Y.full())
    _say(f"  warnings {w}, error {got:.4e} vs optimal {best:.4e}")
    assert w & lib.TT_WSKETCH
    assert got <= 1.5 * best
    c.close()


def test_jacobi_sweep_cap_warns(lib):
    """With the sweep cap forced to 1, the Jacobi SVD of a rounding stops while still
    rotating and the rounding returns TT_WJACOBI; with the default cap it does not."""
    _say("jacobi sweep cap warning")
    rng = np.random.default_rng(23)
    A, B = rng.standard_normal((90, 24)), rng.standard_normal((70, 24))
    c = lib.tt_ctx_create(1 << 28)
    X = lib.DeviceTT.from_factors(A, B)
    Y = lib.DeviceTT(90, 70, 24)
    w, _ = lib.tt_round(c, X, 0.0, 24, Y)
    assert not (w & lib.TT_WJACOBI)
    lib.tt_ctx_set_limits(c, 1, 8)
    w, _ = lib.tt_round(c, X, 0.0, 24, Y)
    assert w & lib.TT_WJACOBI
    c.close()


def test_reciprocal_divergent_series_is_an_error(lib):
    """x = 8 on one row and 1 elsewhere: |1 - x/mean| = 63/17 there, the Taylor terms grow
    and Algorithm 1 must fail with TT_EDOMAIN (the oracle raises SeriesDiverges on the same
    input); a convergent input still works on the same context."""
    _say("reciprocal divergence")
    n1, n2 = 10, 4
    col = np.ones((n1, 1))
    col[0] = 8.0
    with pytest.raises(ott.SeriesDiverges):
        ott.reciprocal(ott.TT(col, np.ones((n2, 1))), 1e-12, 200, 10)
    c = lib.tt_ctx_create(1 << 28)
    X = lib.DeviceTT.from_factors(col, np.ones((n2, 1)))
    Y = lib.DeviceTT(n1, n2, 10)
    with pytest.raises(RuntimeError, match=r"\(-5\)"):
        lib.tt_reciprocal(c, X, 1e-12, 200, 10, Y)
    ok = np.full((n1, 1), 0.5)
    ok[5:] = 4.5
    X = lib.DeviceTT.from_factors(ok, np.ones((n2, 1)))
    w, err, terms = lib.tt_reciprocal(c, X, 1e-12, 200, 10, Y)
    assert err <= 1e-12 and np.allclose(Y.full(), 1.0 / (ok @ np.ones((1, n2))), rtol=1e-10)
    c.close()


def test_nonfinite_core_is_an_error(lib):
    """A NaN in a core reaches the singular values: rounding fails with TT_ENONFINITE."""
    _say("non-finite input")
    rng = np.random.default_rng(24)
    A, B = rng.standard_normal((50, 6)), rng.standard_normal((40, 6))
    A[7, 2] = np.nan
    c = lib.tt_ctx_create(1 << 28)
    X = lib.DeviceTT.from_factors(A, B)
    Y = lib.DeviceTT(50, 40, 6)
    with pytest.raises(RuntimeError, match=r"\(-4\)"):
        lib.tt_round(c, X, 1e-10, 6, Y)
    c.close()


@pytest.mark.parametrize("n1,n2,r,decay,eps,rmax", [
    (777, 1531, 60, 0.8, 1e-6, 64),      # rank set by eps
    (1024, 1024, 40, 0.9, 1e-12, 24),    # rank set by the cap
    (300, 97, 97, 0.7, 0.0, 64),         # eps 0: keep to the cap (rank 97 > the sketch)
])
def test_compress_full_field(lib, ctx, n1, n2, r, decay, eps, rmax):
    """tt_compress (randomized range finder on a dense field) against the oracle's truncated
    SVD of the same matrix: same rank, rel difference <= 1e-10, and the TT_WRANKCAP warning
    exactly when the cap set the rank."""
    import torch
    _say(f"compress {n1}x{n2} r={r} decay={decay} eps={eps} rmax={rmax}")
    rng = np.random.default_rng(n1 + n2)
    U, _ = np.linalg.qr(rng.standard_normal((n1, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n2, r)))
    F = (U * decay ** np.arange(r)) @ V.T
    Ft = torch.tensor(F, dtype=torch.float64, device="cuda").contiguous()
    y, w, sig = lib.tt_compress(ctx, Ft, eps, rmax)
    ref = ott.from_full(F, eps, rmax)
    _say(f"  rank gpu {y.rank} oracle {ref.rank} warn {w}")
    assert y.rank == ref.rank
    assert rel(y.full(), ref.A @ ref.B.T) < 1e-10
    capped = ref.rank == rmax and np.linalg.norm(F - ref.A @ ref.B.T) > eps * np.linalg.norm(F)
    assert bool(w & 1) == capped
    s_ref = np.linalg.svd(F, compute_uv=False)[:y.rank]
    assert np.allclose(sig, s_ref, rtol=1e-9, atol=1e-13 * s_ref[0])


def test_compress_dam_break_front(lib, ctx):
    """The dam break's initial depth at 512^2 (a tanh front of width 0.01: slowly decaying
    spectrum) at eps 1e-8, cap 64, through tt_compress: as the oracle's truncated SVD."""
    import torch
    import synth
    st = synth.dam_break(seed=0, n=512, rmax=64, eps=1e-8)
    F = st.fields[0]
    y, w, sig = lib.tt_compress(ctx, torch.tensor(F, dtype=torch.float64,
                                                  device="cuda").contiguous(), 1e-8, 64)
    ref = ott.from_full(F, 1e-8, 64)
    _say(f"dam break front: rank gpu {y.rank} oracle {ref.rank} warn {w}")
    assert y.rank == ref.rank
    assert rel(y.full(), ref.A @ ref.B.T) < 1e-10


def _bump_tt():
    """Smooth rank-3 part plus a narrow bump in 6 of 400 columns, as exact factors (rank 5)."""
    n1, n2 = 300, 400
    x = np.linspace(0, 1, n1)
    y = np.linspace(0, 1, n2)
    A = np.stack([np.sin(3 * x), np.cos(3 * x), 0.5 * np.cos(5 * x), x,
                  1e-3 * np.exp(-((x - 0.7) / 0.02) ** 2)], axis=1)
    B = np.stack([np.cos(2 * y), np.sin(2 * y), np.sin(4 * y), y,
                  (np.abs(y - 0.33) < 0.007).astype(float)], axis=1)
    return A, B


def test_cross_residual_enrichment(lib):
    """Residual enrichment (TT_ENRICH_RESIDUAL) in tt_cross against the oracle's cross with
    enrich="residual" on the same matrix: same final column set and result over 6 keys; over
    12 keys it recovers the narrow feature at least as often as seeded kicks."""
    _say("cross residual enrichment")
    A, B = _bump_tt()
    F = A @ B.T
    X = lib.DeviceTT.from_factors(A, B)
    T = ott.TT(A, B)

    class Fun:
        def cols(self, J):
            return T.A @ T.B[np.asarray(J)].T

        def rows(self, I):
            return T.A[np.asarray(I)] @ T.B.T

    J0 = [0, 133, 266, 399]
    wins = {"kicks": 0, "residual": 0}
    for mode in wins:
        c = lib.tt_ctx_create(1 << 28)
        lib.tt_ctx_set_enrichment(c, mode)
        for key in range(12):
            Y = lib.DeviceTT(300, 400, 20)
            w, J = lib.tt_cross(c, lib.TT_FN_IDENTITY, [X], [], 300, 400, J0, 1e-12, 20, 3, 4,
                                key, Y)
            wins[mode] += rel(Y.full(), F) < 1e-9
            if mode == "residual" and key < 6:
                ref, J_ref = ott.cross(Fun(), 300, 400, np.array(J0), 1e-12, 20, 3, 4,
                                       key=key, enrich="residual")
                assert sorted(J.tolist()) == sorted(J_ref.tolist()), key
                assert rel(Y.full(), ref.A @ ref.B.T) < 1e-9
        c.close()
    _say(f"  feature recovered: {wins}")
    assert wins["residual"] >= wins["kicks"]


@pytest.mark.parametrize("n1,n2,r,eps,rmax,decay", [
    (1000, 3000, 300, 1e-6, 32, 0.8),
    (777, 1531, 1024, 1e-5, 16, 0.8),
    (2049, 6144, 400, 1e-8, 40, 0.8),
    (1000, 3000, 300, 1e-6, 16, 0.97),   # slow spectrum: stops unconverged, keeps the sketch
])
def test_round_sketched_equals_the_oracle_sketch(lib, ctx, n1, n2, r, eps, rmax, decay):
    """The randomized path of tt_round against the oracle's independent implementation of the
    same seeded sketch (same generator, same steps; oracle.tt.tt_round_sketched): agreement to
    round-off (1e-12 of the norm).  On the slow spectrum the iterations stop before the leak
    bound, both keep the sketch's answer, and it differs from the exact rounding by far more
    than from the oracle's sketch."""
    _say(f"round sketched {n1}x{n2} r={r} eps={eps} rmax={rmax}")
    rng = np.random.default_rng(r)
    A, B = decaying_tt(rng, n1, n2, r, decay=decay)
    x = lib.DeviceTT.from_factors(A, B)
    y = lib.DeviceTT(n1, n2, rmax)
    w, _ = lib.tt_round(ctx, x, eps, rmax, y)
    ref = ott.tt_round_sketched(ott.TT(A, B), eps, rmax)
    ex = ott.tt_round(ott.TT(A, B), eps, rmax)
    F = y.full()
    d_sk = np.linalg.norm(F - ref.A @ ref.B.T) / np.linalg.norm(ref.A @ ref.B.T)
    d_ex = np.linalg.norm(F - ex.A @ ex.B.T) / np.linalg.norm(ex.A @ ex.B.T)
    _say(f"  rank gpu {y.rank} sketch oracle {ref.rank}; vs sketch {d_sk:.2e}, vs exact {d_ex:.2e}")
    assert y.rank == ref.rank
    assert d_sk < 1e-12
    if decay > 0.9:
        assert w & 4 and d_ex > 1e3 * max(d_sk, 1e-16)   # TT_WSKETCH; far from the exact one
