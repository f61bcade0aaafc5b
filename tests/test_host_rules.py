"""The library's host-side decision rules (no GPU) against the oracle's independent ones: the
kept rank of a rounding (Section 3.2) and the seeded fresh columns of a cross sweep
(Section 3.3).  The same C++ definitions run inside the fixed-shape kernels, so these pins
cover the device-side decisions of graph mode as well."""
import os

import numpy as np
import pytest

from oracle import tt as ott

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2408_03483_amd", "libttfv.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libttfv.so not built")


@pytest.fixture(scope="module")
def lib():
    from paper_2408_03483_amd import ttfv
    ttfv.load_library()
    return ttfv


def test_trunc_rank_equals_the_oracle(lib):
    """Random graded spectra (values above the norm floor): the rank and the cap flag equal the
    oracle's tail rule, for tolerances from coarse to zero and caps that bind or not."""
    rng = np.random.default_rng(0)
    checked = 0
    for _ in range(400):
        m = int(rng.integers(1, 97))
        decay = float(rng.uniform(0.3, 0.99))
        s = np.sort(decay ** np.arange(m) * rng.uniform(0.5, 1.5, m))[::-1]
        s = np.maximum(s, 1e-14 * s[0])
        eps = float(rng.choice([1e-1, 1e-3, 1e-6, 1e-10, 1e-14, 0.0]))
        rmax = int(rng.integers(1, 100))
        k, capped = lib.tt_rule_trunc_rank(s, eps, rmax)
        assert k == ott.trunc_rank(s, eps, rmax), (m, eps, rmax)
        k_free = ott.trunc_rank(s, eps, 10 ** 6)
        assert capped == (k_free > rmax), (m, eps, rmax)
        checked += 1
    assert checked == 400


def test_trunc_rank_norm_floor(lib):
    """Reading of the truncation floor: directions at or below max(1e-17, floor_rel) ||s|| are
    never kept, even at eps = 0 (the Jacobi SVD leaves them unrotated); a zero spectrum keeps
    one (the caller writes the zero TT)."""
    s = np.array([1.0, 1e-3, 1e-9, 1e-16, 1e-19, 0.0])
    assert lib.tt_rule_trunc_rank(s, 0.0, 10)[0] == 4          # 1e-19 <= 1e-17 ||s||
    assert lib.tt_rule_trunc_rank(s, 0.0, 10, floor_rel=1e-12)[0] == 3
    assert lib.tt_rule_trunc_rank(s, 0.0, 2) == (2, True)
    assert lib.tt_rule_trunc_rank(np.zeros(5), 1e-10, 3)[0] == 1
    with pytest.raises(RuntimeError):
        lib.tt_rule_trunc_rank(np.ones(129), 0.0, 4)


def test_kicks_equal_the_oracle(lib):
    """Seeded fresh columns for random existing sets, sizes, counts and keys: the same indices
    in the same order as the oracle's SplitMix64 draws, including sets that nearly fill n."""
    rng = np.random.default_rng(1)
    for _ in range(300):
        n = int(rng.integers(1, 400))
        nhave = int(rng.integers(0, min(n, 96) + 1))
        have = rng.choice(n, size=nhave, replace=False).tolist()
        count = int(rng.integers(0, 20))
        key = int(rng.integers(0, 2 ** 63)) ^ (int(rng.integers(0, 2 ** 31)) << 32)
        got = lib.tt_rule_kicks(have, n, count, key)
        want = ott.kick_indices(have, n, count, key)
        assert got == want, (n, nhave, count, key)
        assert not set(got) & set(have) and len(set(got)) == len(got)
