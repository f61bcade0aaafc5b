"""Pins for the exact reconstruction constants of the oracle (Section 2.3)."""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import stencils
from oracle.stencils import QSqrt

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "printed_constants.json")))


def fr(s):
    return float(Fr(s))


def test_step1_textbook_face_stencils():
    # Step 1 combined stencils: Upwind3 (-1, 5, 2)/6 and 5th order (2, -13, 47, 27, -3)/60
    t3 = stencils.tables("upwind3")
    assert np.allclose(t3["face_full"], np.array([-1, 5, 2]) / 6, atol=1e-15)
    t5 = stencils.tables("upwind5")
    assert np.allclose(t5["face_full"], np.array([2, -13, 47, 27, -3]) / 60, atol=1e-15)


def test_step1_candidates_and_weights_match_printed():
    for sch, key_c, key_w in (("upwind3", "step1_upwind3_candidates", "step1_upwind3_weights"),
                              ("upwind5", "step1_5th_candidates", "step1_5th_weights")):
        t = stencils.tables(sch)
        k = t["k"]
        cells = GOLD[key_c]["cells"]
        for r, row in enumerate(GOLD[key_c]["rows"]):
            printed = {c: fr(v) for c, v in zip(cells, row)}
            for l, w in enumerate(t["face_sub"][r]):
                assert abs(w - printed[-r + l]) < 1e-15
        assert np.allclose(t["face_gamma"], [fr(x) for x in GOLD[key_w]], atol=1e-15)
        assert k in (1, 2)


def test_step2_matrices_match_printed_approximations():
    # the printed entries are rational approximations: agree to 2e-6, not exactly
    t3 = stencils.tables("upwind3")
    for m, key in enumerate(("m1", "m2")):
        P = np.array([[fr(x) for x in row] for row in GOLD["step2_upwind3_C"][key]])
        assert np.max(np.abs(np.array(t3["quad_sub"][m]) - P)) < 2e-6
    assert np.allclose(t3["quad_gamma"][0], [0.5, 0.5], atol=1e-15)
    t5 = stencils.tables("upwind5")
    for m, key in enumerate(("m1", "m2", "m3")):
        P = np.array([[fr(x) for x in row] for row in GOLD["step2_5th_C"][key]])
        assert np.max(np.abs(np.array(t5["quad_sub"][m]) - P)) < 2e-6
    for m, key in ((0, "m1"), (2, "m3")):
        P = np.array([fr(x) for x in GOLD["step2_5th_gamma"][key]])
        assert np.max(np.abs(np.array(t5["quad_gamma"][m]) - P)) < 2e-6


def test_exact_values_differ_from_printed_rational():
    # 808/627 is not 1 + sqrt(3)/6: the printed value is an approximation (error ~1e-6)
    t3 = stencils.tables("upwind3")
    exact = 1 + np.sqrt(3) / 6
    assert abs(t3["quad_sub"][0][0][0] - exact) < 1e-15
    assert 1e-7 < abs(808 / 627 - exact) < 2e-6


def test_split_weights_are_exact_rationals():
    g = stencils.linear_weights(2, QSqrt(0))
    assert all(x.b == 0 for x in g)
    assert [x.a for x in g] == [Fr(-9, 80), Fr(49, 40), Fr(-9, 80)]
    gp, gm, sp, sm = stencils.split_weights_exact(g)
    S = GOLD["step2_5th_split"]
    assert gp == [Fr(x) for x in S["gamma_plus"]]
    assert gm == [Fr(x) for x in S["gamma_minus"]]
    assert sp == Fr(S["sigma_plus"]) and sm == Fr(S["sigma_minus"])
    assert sp - sm == 1


@pytest.mark.parametrize("scheme", ["upwind3", "upwind5"])
def test_polynomial_exactness(scheme):
    """Every stencil reproduces point values of polynomials of its degree from exact averages."""
    t = stencils.tables(scheme)
    k = t["k"]
    rng = np.random.default_rng(0)
    pts = [0.5] + t["gl_points"]
    ws = [t["face_full"]] + t["quad_full"]
    deg = 2 * k
    for _ in range(5):
        c = rng.standard_normal(deg + 1)
        P = np.polynomial.Polynomial(c)
        Pi = P.integ()
        avg = np.array([Pi(o + 0.5) - Pi(o - 0.5) for o in range(-k, k + 1)])
        for x0, w in zip(pts, ws):
            assert abs(np.dot(w, avg) - P(x0)) < 1e-12 * max(1.0, np.abs(c).sum())
        # candidate stencils are exact to degree k
        for m, x0 in enumerate(t["gl_points"]):
            Pk = np.polynomial.Polynomial(c[:k + 1])
            Pki = Pk.integ()
            for r in range(k + 1):
                offs = stencils.substencil_offsets(k, r)
                a = np.array([Pki(o + 0.5) - Pki(o - 0.5) for o in offs])
                assert abs(np.dot(t["quad_sub"][m][r], a) - Pk(x0)) < 1e-12 * max(1, np.abs(c).sum())


@pytest.mark.parametrize("scheme", ["upwind3", "upwind5"])
def test_linear_weights_recombine_full_stencil(scheme):
    t = stencils.tables(scheme)
    k = t["k"]
    for m in range(t["nq"]):
        comb = np.zeros(2 * k + 1)
        for r in range(k + 1):
            for l in range(k + 1):
                comb[(-r + l) + k] += t["quad_gamma"][m][r] * t["quad_sub"][m][r][l]
        assert np.allclose(comb, t["quad_full"][m], atol=1e-14)
        assert abs(sum(t["quad_gamma"][m]) - 1.0) < 1e-14
        assert abs(sum(t["quad_full"][m]) - 1.0) < 1e-14


def test_gauss_legendre_exactness():
    for nq, deg in ((2, 3), (3, 5)):
        pts, wts = stencils.gauss_points(nq)
        x = np.array([float(p) for p in pts])
        w = np.array([float(v) for v in wts])
        for p in range(deg + 1):
            exact = (0.5 ** (p + 1) - (-0.5) ** (p + 1)) / (p + 1)
            assert abs(np.dot(w, x ** p) - exact) < 1e-15
        assert abs(np.dot(w, x ** (deg + 1)) - (0.5 ** (deg + 2) * 2 / (deg + 2))) > 1e-8


def test_upwind5_middle_point_collapses_to_central_stencil():
    t = stencils.tables("upwind5")
    assert np.allclose(t["quad_full"][1], np.array([3 / 640, -29 / 480, 1067 / 960, -29 / 480, 3 / 640]),
                       atol=1e-15)
