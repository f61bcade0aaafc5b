"""Cholesky QR on the matrix cores (the orthogonalisation inside TT rounding, Section 3.2) on
inputs that break plain Cholesky QR: graded spectra down to 1e-30, zero, repeated and
rank-one columns, the Khatri-Rao core of a product h o h.  Each rounding is compared with the
oracle's (truncated SVD of the full matrix) and with the Householder path; a pass limit too
small to converge forces the Householder redo, which must give the Householder result."""
import sys

import numpy as np
import pytest

from oracle import tt as ott

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


def _cases(rng):
    n1, n2 = 1000, 700
    U, _ = np.linalg.qr(rng.standard_normal((n1, 80)))
    V, _ = np.linalg.qr(rng.standard_normal((80, 80)))
    graded = (U * np.logspace(0, -30, 80)) @ V.T
    yield "graded to 1e-30", graded, rng.standard_normal((n2, 80))
    A = rng.standard_normal((n1, 72))
    A[:, 5] = 0.0
    A[:, 40] = A[:, 3]
    yield "zero and repeated columns", A, rng.standard_normal((n2, 72))
    yield "rank one", np.ones((n1, 90)), np.ones((n2, 90))
    h1, h2 = 1.0 + 0.1 * rng.standard_normal((n1, 9)), rng.standard_normal((n2, 9))
    kr1 = np.einsum("ia,ib->iab", h1, h1).reshape(n1, 81)
    kr2 = np.einsum("ia,ib->iab", h2, h2).reshape(n2, 81)
    yield "Khatri-Rao h o h", kr1, kr2
    sk = rng.standard_normal((n1, 12)) @ rng.standard_normal((12, 96))
    yield "96 columns of rank 12", sk, rng.standard_normal((n2, 96))


@pytest.mark.parametrize("eps", [1e-10, 1e-13])
def test_cholesky_qr_rounding_matches_oracle_and_householder(lib, eps):
    rng = np.random.default_rng(5)
    cc = lib.tt_ctx_create(1 << 30)
    ch = lib.tt_ctx_create(1 << 30)
    lib.tt_ctx_set_qr(cc, "cholesky")
    lib.tt_ctx_set_qr(ch, "householder")
    try:
        for name, A, B in _cases(rng):
            n1, n2, r = A.shape[0], B.shape[0], A.shape[1]
            X = lib.DeviceTT.from_factors(A, B)
            Yc, Yh = lib.DeviceTT(n1, n2, 96), lib.DeviceTT(n1, n2, 96)
            lib.tt_round(cc, X, eps, 96, Yc)
            lib.tt_round(ch, X, eps, 96, Yh)
            ref = ott.tt_round(ott.TT(A, B), eps, 96)
            F, Fr, Fh = Yc.full(), ref.full(), Yh.full()
            nr = np.linalg.norm(Fr)
            e_o = np.linalg.norm(F - Fr) / nr
            e_h = np.linalg.norm(F - Fh) / nr
            Ac = Yc.factors()[0]
            orth = np.max(np.abs(Ac.T @ Ac - np.eye(Yc.rank)))
            _say(f"  {name}, eps {eps:g}: rank {Yc.rank} (oracle {ref.rank}, householder "
                 f"{Yh.rank}), vs oracle {e_o:.1e}, vs householder {e_h:.1e}, first core "
                 f"orthonormal to {orth:.1e}")
            assert Yc.rank == ref.rank == Yh.rank
            assert e_o <= 10 * eps + 1e-13 and e_h <= 10 * eps + 1e-13
            assert orth <= 1e-12
    finally:
        cc.close()
        ch.close()


def test_unconverged_cholesky_qr_is_redone_with_householder(lib):
    """Two passes (the Gram of Y and one multiplication) leave the columns of these inputs
    short of orthonormal: every such call sets Q and R to NaN and the rounding is redone with
    Householder QR, giving the Householder result (no NaN reaches the output)."""
    rng = np.random.default_rng(6)
    cc = lib.tt_ctx_create(1 << 30)
    ch = lib.tt_ctx_create(1 << 30)
    lib.tt_ctx_set_qr(cc, "cholesky", max_passes=2)
    lib.tt_ctx_set_qr(ch, "householder")
    try:
        for name, A, B in _cases(rng):
            n1, n2 = A.shape[0], B.shape[0]
            X = lib.DeviceTT.from_factors(A, B)
            Yc, Yh = lib.DeviceTT(n1, n2, 96), lib.DeviceTT(n1, n2, 96)
            lib.tt_round(cc, X, 1e-10, 96, Yc)
            lib.tt_round(ch, X, 1e-10, 96, Yh)
            F, Fh = Yc.full(), Yh.full()
            d = np.linalg.norm(F - Fh) / np.linalg.norm(Fh)
            _say(f"  {name}: ranks {Yc.rank} {Yh.rank}, redo vs householder {d:.1e}")
            assert np.all(np.isfinite(F)) and Yc.rank == Yh.rank and d <= 1e-14
    finally:
        cc.close()
        ch.close()


def test_step_with_cholesky_qr_matches_oracle(lib):
    """One nonlinear Upwind5 step (48^2, periodic, cap 16) with every QR by Cholesky QR."""
    import synth
    from oracle import tt_fv as otf
    st = synth.nonlinear_bumps(seed=3, n=48, rmax=16, eps=1e-10)
    dev = [lib.DeviceTT.from_factors(f.A, f.B, cap=16) for f in st.tt]
    s = lib.tt_fv_init(48, "upwind5", True, True, dev, g=st.g, eps=1e-10, r_max=16,
                       taylor_terms=8, arena_bytes=1 << 28, qr="cholesky")
    lib.tt_fv_step(s, st.dt, 1)
    Qg = lib.tt_fv_get_state(s)
    stats = lib.tt_fv_get_stats(s)
    s.close()
    ts = otf.TTSolver(48, "upwind5", True, True, g=st.g, eps=1e-10, rmax=16, taylor_terms=8)
    Qo = ts.step([ott.TT(f.A, f.B) for f in st.tt], st.dt)
    rel = [np.linalg.norm(g.full() - o.full()) / np.linalg.norm(o.full()) for g, o in zip(Qg, Qo)]
    _say(f"  step rel {rel}, householder redos {stats['qr_redos']}")
    assert max(rel) <= 1e-9
