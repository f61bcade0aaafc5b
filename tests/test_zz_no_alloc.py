"""The allocation-free rounding entry point against tt_round (through the C ABI, on the GPU)."""
import sys

import numpy as np
import pytest

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


def _decaying(rng, n1, n2, r, decay):
    return rng.standard_normal((n1, r)) * decay ** np.arange(r), rng.standard_normal((n2, r))


def test_round_noalloc_equals_tt_round_on_two_calls(lib):
    """Two calls in a row, the second smaller (the scratch keeps the first call's contents):
    the range-finder path (rank 1024 > 96) at the throughput workload's Hadamard shape, then
    the exact path; each against tt_round with its own context: same rank, singular values
    and reconstructed matrix to 1e-12 relative."""
    rng = np.random.default_rng(41)
    ctx = lib.tt_ctx_create(1 << 30)
    try:
        for n1, n2, r, eps, rmax in ((1024, 3072, 1024, 1e-10, 32), (333, 517, 40, 1e-12, 24)):
            _say(f"noalloc round {n1}x{n2} rank {r} eps {eps} rmax {rmax}")
            A, B = _decaying(rng, n1, n2, r, 0.97)
            X = lib.DeviceTT.from_factors(A, B)
            Y0, Y1 = lib.DeviceTT(n1, n2, rmax), lib.DeviceTT(n1, n2, rmax)
            w0, s0 = lib.tt_round(ctx, X, eps, rmax, Y0)
            w1, s1 = lib.tt_round_noalloc(X, eps, rmax, Y1)
            F0, F1 = Y0.full(), Y1.full()
            e = np.linalg.norm(F1 - F0) / np.linalg.norm(F0)
            _say(f"  ranks {Y0.rank} {Y1.rank}, warnings {w0} {w1}, rel {e:.2e}")
            assert Y1.rank == Y0.rank and w1 == w0
            assert np.max(np.abs(s1 - s0)) <= 1e-12 * s0[0]
            assert e <= 1e-12
    finally:
        ctx.close()


def test_round_noalloc_rejects_oversized_shapes(lib):
    """Shapes whose temporaries could exceed the fixed scratch are refused before any work
    is enqueued, with TT_ENOMEM and a message naming both sizes; the output is untouched."""
    import torch
    n, r = 20000, 2000
    X = lib.DeviceTT(n, n, r)
    X.g1.normal_()
    X.g2.normal_()
    X.rank = r
    Y = lib.DeviceTT(n, n, 32)
    Y.g1.fill_(7.0)
    with pytest.raises(RuntimeError, match=r"\(-2\).*scratch"):
        lib.tt_round_noalloc(X, 1e-10, 32, Y)
    torch.cuda.synchronize()
    assert bool((Y.g1 == 7.0).all())
