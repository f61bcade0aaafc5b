"""GPU d-core TT rounding (tt_round_nd; Sections 3.1-3.2 extended to d cores) against the
oracle's (oracle/tt_nd.py), through the C ABI."""
import sys

import numpy as np
import pytest

from oracle import tt_nd

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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("modes,ranks,eps,rmax", [
    ((64, 48, 80, 32), (8, 12, 6), 1e-6, 32),
    ((7, 9, 11, 13, 5), (5, 9, 9, 4), 1e-3, 32),
    ((16, 16, 16), (12, 10), 0.0, 6),            # cap binds
])
def test_round_nd_matches_the_oracle(lib, ctx, modes, ranks, eps, rmax):
    _say(f"round nd {modes} {ranks} eps={eps} rmax={rmax}")
    rng = np.random.default_rng(sum(modes))
    X = tt_nd.random_tt(rng, modes, ranks, decay=0.6)
    ref, sig_ref = tt_nd.tt_round(X, eps, rmax)
    y, w, sig = lib.tt_round_nd(ctx, lib.DeviceTTnd.from_cores(X), eps, rmax)
    got = y.to_cores()
    _say(f"  ranks gpu {y.r} oracle {[1] + [c.shape[2] for c in ref]} warn {w}")
    assert y.r == [1] + [c.shape[2] for c in ref]
    F = tt_nd.full(X)
    assert _rel(tt_nd.full(got), tt_nd.full(ref)) < 1e-10
    if eps > 0.0:
        assert _rel(tt_nd.full(got), F) <= eps
    assert np.allclose(sig, np.concatenate(sig_ref), rtol=1e-9, atol=1e-13 * np.max(sig))
    assert bool(w & 1) == (rmax < max(ranks) and eps == 0.0)


@pytest.mark.parametrize("d", [6, 10])
def test_round_nd_redundant_qtt_sum(lib, ctx, d):
    """A QTT-like train (modes 2) summed with itself and subtracted again: ranks triple, the
    wide unfoldings at both ends lower them in the orthogonalisation, and the rounding returns
    the original ranks and tensor."""
    rng = np.random.default_rng(d)
    ranks = [min(2 ** min(k + 1, d - k - 1), 4) for k in range(d - 1)]
    X = tt_nd.random_tt(rng, (2,) * d, ranks, decay=1.0)
    Y = tt_nd.add(tt_nd.add(X, X), [(-1.0 if k == 0 else 1.0) * c for k, c in enumerate(X)])
    y, w, sig = lib.tt_round_nd(ctx, lib.DeviceTTnd.from_cores(Y), 1e-12, 16)
    ref, _ = tt_nd.tt_round(Y, 1e-12, 16)
    _say(f"qtt d={d}: ranks in {[1] + [c.shape[2] for c in Y]} out {y.r}")
    assert y.r == [1] + [c.shape[2] for c in ref]
    assert _rel(tt_nd.full(y.to_cores()), tt_nd.full(X)) < 1e-10


def test_round_nd_zero(lib, ctx):
    rng = np.random.default_rng(1)
    X = [0.0 * c for c in tt_nd.random_tt(rng, (5, 6, 7), (3, 4))]
    y, w, sig = lib.tt_round_nd(ctx, lib.DeviceTTnd.from_cores(X), 1e-8, 4)
    assert y.r == [1, 1, 1, 1] and not np.any(tt_nd.full(y.to_cores()))
