"""Pins for the d-core TT rounding (Sections 3.1-3.2 extended to d cores): against the
full tensor's sequential truncated SVDs (TT-SVD of the dense array, computed here by numpy on
small cases), the error bound, and the exact recovery of known ranks."""
import math

import numpy as np
import pytest

from oracle import tt_nd


def _tt_svd_dense(X, eps, rmax):
    """Sequential truncated SVDs of the dense tensor's unfoldings (the plain TT-SVD)."""
    d = X.ndim
    delta = eps / math.sqrt(d - 1) * np.linalg.norm(X)
    ranks, C, r = [], X.copy(), 1
    for k in range(d - 1):
        C = C.reshape(r * X.shape[k], -1)
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        tail = np.concatenate([np.sqrt(np.cumsum((s * s)[::-1])[::-1]), [0.0]])
        keep = next(kk for kk in range(1, len(s) + 1) if tail[kk] <= delta)
        keep = min(keep, rmax)
        ranks.append(keep)
        C = s[:keep, None] * Vt[:keep]
        r = keep
    return ranks


@pytest.mark.parametrize("modes,ranks", [((6, 5, 7, 4), (3, 5, 2)), ((3, 3, 3, 3, 3), (2, 4, 4, 2)),
                                         ((2,) * 8, (2, 4, 4, 4, 4, 4, 2))])
def test_round_recovers_a_redundant_sum(modes, ranks):
    """X + X - X (ranks tripled, exactly rank of X) rounds back to X's ranks and to X."""
    rng = np.random.default_rng(len(modes))
    X = tt_nd.random_tt(rng, modes, ranks, decay=1.0)
    Y = tt_nd.add(tt_nd.add(X, X), [(-1.0 if k == 0 else 1.0) * c for k, c in enumerate(X)])
    Z, _ = tt_nd.tt_round(Y, 1e-12, 64)
    F = tt_nd.full(X)
    assert np.linalg.norm(tt_nd.full(Z) - F) <= 1e-10 * np.linalg.norm(F)
    assert [c.shape[2] for c in Z[:-1]] == _tt_svd_dense(F, 1e-12, 64)


def test_round_error_bound_and_dense_ranks():
    """A graded TT at eps = 1e-3 and 1e-6: the ranks equal the dense TT-SVD's, the error is
    within eps ||X||, and the kept bond singular values are the dense unfoldings' ones."""
    rng = np.random.default_rng(9)
    X = tt_nd.random_tt(rng, (5, 6, 7, 5), (5, 6, 4), decay=0.5)
    F = tt_nd.full(X)
    for eps in (1e-3, 1e-6):
        Z, sig = tt_nd.tt_round(X, eps, 64)
        assert [c.shape[2] for c in Z[:-1]] == _tt_svd_dense(F, eps, 64)
        assert np.linalg.norm(tt_nd.full(Z) - F) <= eps * np.linalg.norm(F)
        s1 = np.linalg.svd(F.reshape(5, -1), compute_uv=False)
        assert np.allclose(sig[0], s1[:len(sig[0])], rtol=1e-10)
    assert tt_nd.norm(X) == pytest.approx(np.linalg.norm(F), rel=1e-12)


def test_round_rank_cap_and_zero():
    rng = np.random.default_rng(3)
    X = tt_nd.random_tt(rng, (4, 4, 4, 4), (4, 8, 4), decay=0.9)
    Z, _ = tt_nd.tt_round(X, 0.0, 3)
    assert max(c.shape[2] for c in Z[:-1]) == 3
    zero = [0.0 * c for c in X]
    Z, sig = tt_nd.tt_round(zero, 1e-8, 5)
    assert all(c.shape[0] == 1 and c.shape[2] == 1 for c in Z) and not np.any(tt_nd.full(Z))
