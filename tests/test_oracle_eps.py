"""Pins for the paper's tolerance rule (Section 4.4, eqs. eps-tt-formula and
modified-eps-tt-formula) and for the Coriolis term on Section 5.2's inertia-gravity wave.

The tolerance rule is pinned by what it is for rather than by its formula: the rounding of a
field at the per-variable tolerance must leave an L2 error (cell-area weighted) at most
C_eps V^(1/2) dx^(p - 1/2), and not far below it on a smoothly decaying spectrum; the
tolerance must scale inversely with the field and by 2^(p - 1/2) under refinement, and clip
at 1e-3.  The Coriolis term is pinned by the closed-form solution with f != 0."""
import math

import numpy as np
import pytest

import synth
from oracle import fv_grid
from oracle.tt import TT, norm, tt_round
from oracle.tt_fv import TTSolver, paper_tolerances


def _graded_tt(rng, n, r, decay):
    A, _ = np.linalg.qr(rng.standard_normal((n, r)))
    B, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return TT(A * (decay ** np.arange(r))[None, :], B)


def test_tolerance_scaling_refinement_and_clip():
    rng = np.random.default_rng(0)
    n = 64
    Q = [_graded_tt(rng, n, 6, 0.5) for _ in range(3)]
    norms = [norm(q) for q in Q]
    eps, eq = paper_tolerances(norms, n, 5, 1.0)
    # eq. eps-tt-formula uses the largest norm, so it is the smallest of the unclipped ones
    assert eps == pytest.approx(min(eq), rel=1e-15)
    # tolerances scale like 1/||q||
    eps2, eq2 = paper_tolerances([7.0 * v for v in norms], n, 5, 1.0)
    assert eps2 == pytest.approx(eps / 7.0, rel=1e-14)
    assert eq2 == pytest.approx([e / 7.0 for e in eq], rel=1e-14)
    # same L2 norm on the twice finer grid (Frobenius norm of the array doubles): the
    # absolute L2 tolerance falls by 2^(p - 1/2)
    for p, scheme_order in ((3, 3), (5, 5)):
        e1, _ = paper_tolerances(norms, n, scheme_order, 1.0)
        e2, _ = paper_tolerances([2.0 * v for v in norms], 2 * n, scheme_order, 1.0)
        assert (e1 * norms[0] / n) / (e2 * 2 * norms[0] / (2 * n)) == \
            pytest.approx(2.0 ** (p - 0.5), rel=1e-12)
    # linear in C_eps
    eps3, _ = paper_tolerances(norms, n, 5, 250.0)
    assert eps3 == pytest.approx(250.0 * eps, rel=1e-14)
    # clip of the modified formula, for a tiny variable and for an exactly zero one
    eps4, eq4 = paper_tolerances([norms[0], 1e-30, 0.0], n, 3, 1.0)
    assert eq4[1] == 1e-3 and eq4[2] == 1e-3
    assert eps4 == pytest.approx(paper_tolerances([norms[0]], n, 3, 1.0)[0], rel=1e-15)
    assert paper_tolerances([0.0, 0.0, 0.0], n, 5, 1.0) == (1e-3, [1e-3, 1e-3, 1e-3])


@pytest.mark.parametrize("order,c_eps", [(3, 1.0), (5, 1.0), (5, 1000.0)])
def test_rounding_at_the_tolerance_meets_the_l2_target(order, c_eps):
    """The quantity the rule controls: with eps_q, round(q) is within C V^(1/2) dx^(p-1/2) of q
    in the cell-area L2 norm, and (spectrum decaying by 0.6 per index) within a small factor of
    that target, so a mis-scaled norm (a factor n or dx) fails one side."""
    rng = np.random.default_rng(order + int(c_eps))
    for n in (40, 96):
        dx = 1.0 / n
        target = c_eps * dx ** (order - 0.5)
        # amplitude chosen so that the tolerance lands well inside the spectrum
        r = 40
        q = _graded_tt(rng, n, r, 0.6)
        q = TT(q.A * (target * 0.6 ** -16 / dx), q.B)
        _, eq = paper_tolerances([norm(q), norm(q), norm(q)], n, order, c_eps)
        assert eq[0] < 1e-3
        y = tt_round(q, eq[0], r)
        err = dx * float(np.linalg.norm(q.A @ q.B.T - y.A @ y.B.T))
        assert err <= target * (1 + 1e-12), (err, target)
        assert err >= 0.25 * target, (err, target)


def _igw_state(n, t, f, g, H):
    fac = synth.inertia_gravity_exact(n, t, f, g, H, modes=((0.5, 1.0), (1.0, 2.0)))
    return [X @ Y.T for X, Y in fac], fac


def _rel(U, V):
    return math.sqrt(sum(float(np.sum((a - b) ** 2)) for a, b in zip(U, V)) /
                     sum(float(np.sum(b * b)) for b in V))


def test_inertia_gravity_coriolis_full_grid():
    """Section 5.2's closed form with f != 0 (nondimensional Table 2 scales): the scheme with
    the Coriolis term follows it; dropping the term or flipping its sign does not."""
    g, H, f, t_ref = synth.nondim("inertia_gravity", 1000.0)
    T = 3.0 * 3600.0 / t_ref
    n = 24
    c = math.sqrt(g * H)
    nsteps = int(math.ceil(T / (0.3 / n / c)))
    dt = T / nsteps
    U0, _ = _igw_state(n, 0.0, f, g, H)
    ref, _ = _igw_state(n, T, f, g, H)
    errs = {}
    for ff in (f, 0.0, -f):
        s = fv_grid.GridSolver(n, "upwind5", nonlinear=False, periodic=True, g=g, H=H, f=ff)
        errs[ff] = _rel(s.run(U0, dt, nsteps), ref)
    assert errs[f] < 5e-3, errs
    assert errs[0.0] > 50 * errs[f] and errs[-f] > 50 * errs[f], errs


def test_inertia_gravity_tt_oracle_paper_tolerances():
    """The TT oracle with the Section 4.4 tolerances and C_eps of Table 1 tracks the full-grid
    oracle on the f != 0 wave: the roundings stay far below the discretisation error, and the
    ranks stay at the exact rank 4 of the two plane-wave modes."""
    g, H, f, t_ref = synth.nondim("inertia_gravity", 1000.0)
    T = 3.0 * 3600.0 / t_ref
    n = 24
    c = math.sqrt(g * H)
    nsteps = int(math.ceil(T / (0.3 / n / c)))
    dt = T / nsteps
    U0, fac = _igw_state(n, 0.0, f, g, H)
    Q = [TT(X, Y) for X, Y in fac]
    Q = [tt_round(q, 1e-15, 16) for q in Q]
    s = TTSolver(n, "upwind5", nonlinear=False, periodic=True, g=g, H=H, f=f, rmax=16,
                 eps_rule="paper", c_eps=synth.TABLE1["inertia_gravity"]["upwind5"][1])
    Qn = s.run(Q, dt, nsteps)
    grid = fv_grid.GridSolver(n, "upwind5", nonlinear=False, periodic=True, g=g, H=H, f=f)
    Un = grid.run(U0, dt, nsteps)
    assert _rel([q.A @ q.B.T for q in Qn], Un) < 1e-10
    assert all(r <= 4 for rr in s.stats["ranks"] for r in rr), s.stats["ranks"]
    # the recorded per-step tolerances are those of the step's starting state
    assert len(s.stats["eps"]) == nsteps
    e0, eq0 = s.stats["eps"][0]
    assert (e0, eq0) == paper_tolerances([norm(q) for q in Q], n, 5, 1.0)
