"""Pins for the full-grid finite-volume oracle (Sections 2.2-2.4, 4.4, 5)."""
import math

import numpy as np
import pytest

from oracle import fv_grid, stencils


def _cell_avg_plane(n, kx, ky, phase):
    """Exact cell averages of cos(kx x + ky y - phase) on an n x n grid of [0,1]^2."""
    dx = 1.0 / n
    xc = (np.arange(n) + 0.5) * dx
    sx = np.sinc(kx * dx / (2 * np.pi)) if kx else 1.0     # np.sinc(t) = sin(pi t)/(pi t)
    sy = np.sinc(ky * dx / (2 * np.pi)) if ky else 1.0
    return sx * sy * np.cos(kx * xc[:, None] + ky * xc[None, :] - phase)


def plane_wave(n, t, g=9.81, H=1.0, amp=0.01, kk=(1, 1)):
    """Linear SWE, f = 0: eta = a cos(k.x - w t), u = g a kx/w cos(.), v = g a ky/w cos(.)
    (the inertia-gravity solution of Section 5.2 with f = 0)."""
    kx, ky = 2 * np.pi * kk[0], 2 * np.pi * kk[1]
    w = math.sqrt(g * H * (kx * kx + ky * ky))
    base = _cell_avg_plane(n, kx, ky, w * t)
    return [amp * base, g * amp * kx / w * base, g * amp * ky / w * base]


def _err(U, V):
    return math.sqrt(sum(float(np.sum((a - b) ** 2)) for a, b in zip(U, V)) / U[0].size)


@pytest.mark.parametrize("scheme,order,expo", [("upwind3", 3, 1.0), ("upwind5", 5, 5.0 / 3.0),
                                               ("weno5", 5, 5.0 / 3.0)])
def test_linear_plane_wave_convergence(scheme, order, expo):
    """Formal orders 3 / 5 / 5 on the closed-form linear wave (Sections 5.1-5.3)."""
    T = 0.04
    errs = []
    for n in (16, 32):
        dx = 1.0 / n
        dt0 = 0.25 * dx ** expo
        nsteps = int(math.ceil(T / dt0))
        dt = T / nsteps
        s = fv_grid.GridSolver(n, scheme, nonlinear=False, periodic=True)
        U = s.run(plane_wave(n, 0.0), dt, nsteps)
        errs.append(_err(U, plane_wave(n, T)))
    rate = math.log2(errs[0] / errs[1])
    assert rate > order - 0.35, (errs, rate)


def test_lake_at_rest_and_constant_states():
    for periodic in (True, False):
        for scheme in ("upwind3", "upwind5", "weno5"):
            s = fv_grid.GridSolver(10, scheme, nonlinear=True, periodic=periodic)
            U = [np.full((10, 10), 1.3), np.zeros((10, 10)), np.zeros((10, 10))]
            L = s.rhs(U)
            assert max(float(np.max(np.abs(l))) for l in L) < 1e-12
            if periodic:
                U = [np.full((10, 10), 1.3), np.full((10, 10), 0.2), np.full((10, 10), -0.1)]
                L = s.rhs(U)
                assert max(float(np.max(np.abs(l))) for l in L) < 1e-12


def test_flux_consistency():
    """LLF(U, U) = F(U) for both directions and both equation sets."""
    rng = np.random.default_rng(3)
    for nonlinear in (True, False):
        U = [1.0 + 0.1 * rng.random(7), 0.1 * rng.standard_normal(7), 0.1 * rng.standard_normal(7)]
        for d in (0, 1):
            F = fv_grid.physical_flux(U, nonlinear, 9.81, 1.0, d)
            Fh = fv_grid.llf(U, U, nonlinear, 9.81, 1.0, d)
            for a, b in zip(F, Fh):
                assert np.allclose(a, b, atol=1e-15)


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("scheme", ["upwind5", "weno5"])
def test_mass_conservation(periodic, scheme):
    rng = np.random.default_rng(5)
    n = 16
    x = (np.arange(n) + 0.5) / n
    h = 1.0 + 0.05 * np.exp(-((x[:, None] - 0.4) ** 2 + (x[None, :] - 0.6) ** 2) / 0.02)
    U = [h, 0.01 * rng.standard_normal((n, n)), 0.01 * rng.standard_normal((n, n))]
    s = fv_grid.GridSolver(n, scheme, nonlinear=True, periodic=periodic)
    m0 = float(U[0].sum())
    U = s.run(U, 2e-3, 5)
    assert abs(float(U[0].sum()) - m0) < 1e-13 * n * n


def test_weno5_equals_upwind5_on_linear_data():
    """On linear data every smoothness indicator is equal, so the nonlinear weights equal the
    linear weights and WENO5 reduces to Upwind5 (Section 2.3)."""
    rng = np.random.default_rng(1)
    t = stencils.tables("weno5")
    base = rng.standard_normal(4)
    offs = np.arange(-2, 3)
    vals = {int(o): base[0] + base[1] * o + 0 * base[2] for o in offs}
    for which in ["face", 0, 1, 2]:
        w = fv_grid.recon_point(vals, t, which, "weno5", 1e-6)
        u = fv_grid.recon_point(vals, t, which, "upwind5", 1e-6)
        assert abs(w - u) < 1e-13


def test_weno5_essentially_non_oscillatory_across_a_step():
    """At a jump the WENO5 face value stays within the data range; Upwind5 overshoots."""
    t = stencils.tables("weno5")
    vals = {-2: 0.0, -1: 0.0, 0: 0.0, 1: 1.0, 2: 1.0}
    w = fv_grid.recon_point(vals, t, "face", "weno5", 1e-6)
    u = fv_grid.recon_point(vals, t, "face", "upwind5", 1e-6)
    assert -1e-3 < w < 1.0 + 1e-3
    assert abs(u - (47 * 0 + 27 * 1 - 3 * 1) / 60) < 1e-15   # 0.4: linear answer
    vals = {-2: 0.0, -1: 0.0, 0: 1.0, 1: 1.0, 2: 1.0}
    w = fv_grid.recon_point(vals, t, "face", "weno5", 1e-6)
    assert abs(w - 1.0) < 1e-3                                 # takes the smooth stencil
    u = fv_grid.recon_point(vals, t, "face", "upwind5", 1e-6)
    assert u > 1.0 + 1e-3                                      # linear overshoot


def _gaussian_linear_exact(n, t, centre, g=9.81, H=1.0, amp=0.01, w=0.05, kmax=40):
    """Exact cell averages of the linear SWE solution from a periodised Gaussian eta, u=v=0.

    eta_hat_k(t) = eta_hat_k(0) cos(c|k| t), u_hat_k = -i g kx eta_hat_k(0) sin(c|k|t)/(c|k|).
    """
    c = math.sqrt(g * H)
    dx = 1.0 / n
    ks = np.arange(-kmax, kmax + 1)
    kap = 2 * np.pi * ks
    a = w * math.sqrt(2 * math.pi) * np.exp(-0.5 * (kap * w) ** 2)    # Fourier coefficients
    sinc = np.where(ks == 0, 1.0, np.sinc(kap * dx / (2 * np.pi)))
    xc = (np.arange(n) + 0.5) * dx
    Ex = np.exp(1j * kap[None, :] * (xc[:, None] - centre[0])) * (a * sinc)[None, :]
    Ey = np.exp(1j * kap[None, :] * (xc[:, None] - centre[1])) * (a * sinc)[None, :]
    KX, KY = np.meshgrid(kap, kap, indexing="ij")
    K = np.sqrt(KX ** 2 + KY ** 2)
    cosw = np.cos(c * K * t)
    with np.errstate(invalid="ignore", divide="ignore"):
        sfac = np.where(K > 0, np.sin(c * K * t) / (c * K), 0.0)
    eta = amp * (Ex @ cosw @ Ey.T).real
    u = amp * (Ex @ (-1j * g * KX * sfac) @ Ey.T).real
    v = amp * (Ex @ (-1j * g * KY * sfac) @ Ey.T).real
    return [eta, u, v]


def test_linear_gaussian_against_fourier_solution():
    """The 64^2 linear Gaussian workload: the full-grid oracle follows the exact solution and
    refines at the third-order rate."""
    centre = (0.37, 0.61)
    T = 0.05
    errs = []
    for n in (64, 128):
        c = math.sqrt(9.81)
        dt0 = 0.4 / (2 * c * n)
        nsteps = int(math.ceil(T / dt0))
        dt = T / nsteps
        U0 = _gaussian_linear_exact(n, 0.0, centre)
        s = fv_grid.GridSolver(n, "upwind3", nonlinear=False)
        U = s.run(U0, dt, nsteps)
        ex = _gaussian_linear_exact(n, T, centre)
        errs.append(np.linalg.norm(U[0] - ex[0]) / np.linalg.norm(ex[0]))
    assert errs[0] < 0.05
    assert math.log2(errs[0] / errs[1]) > 2.5


def test_ssprk3_amplification_of_one_mode():
    """For the linear scheme a single Fourier mode is an eigenvector of the spatial operator;
    one SSP-RK3 step multiplies it by 1 + z + z^2/2 + z^3/6 (z = dt * eigenvalue)."""
    n = 16
    s = fv_grid.GridSolver(n, "upwind5", nonlinear=False)
    # scalar probe: eta-only mode of the linear system is not an eigenvector, use the
    # (eta + u/c) characteristic combination of a wave moving in x
    kx = 2 * np.pi
    c = math.sqrt(9.81)
    x = (np.arange(n) + 0.5) / n
    e = np.exp(1j * kx * x)[:, None] * np.ones((1, n))
    U = [e.real * 0.01, (c * e.real) * 0.01, np.zeros((n, n))]     # right-moving: u = c eta
    Ui = [e.imag * 0.01, (c * e.imag) * 0.01, np.zeros((n, n))]
    L = s.rhs(U)
    Li = s.rhs(Ui)
    z_field = (L[0] + 1j * Li[0]) / (0.01 * e)
    z = complex(np.mean(z_field))
    assert np.allclose(z_field, z, atol=1e-10)
    dt = 2e-3
    Un = s.step(U, dt)
    Uni = s.step(Ui, dt)
    amp = (Un[0] + 1j * Uni[0]) / (0.01 * e)
    zz = dt * z
    assert np.allclose(amp, 1 + zz + zz ** 2 / 2 + zz ** 3 / 6, atol=1e-12)


# Hand-derived one-face LLF values (Section 2.2, equation LLF; Section 2.4 for the system).
# g = 4 keeps every wave speed rational: sqrt(g h) = 2 at h = 1 and 1 at h = 1/4.
#   minus state U- = (h, hu, hv) = (1, 1/2, -3):   u- = 1/2,  v- = -3
#   plus  state U+ = (1/4, -1/2, 1/4):             u+ = -2,   v+ = 1
# x: |u-| + c- = 5/2, |u+| + c+ = 3  -> lambda = 3 (decided by the plus side, where u < 0)
# y: |v-| + c- = 5,   |v+| + c+ = 2  -> lambda = 5 (decided by the minus side, where v < 0)
# Dropping |.|, using one side, g h instead of sqrt(g h), or the wrong momentum changes both.
_G4 = 4.0
_UM = [np.array([1.0]), np.array([0.5]), np.array([-3.0])]
_UP = [np.array([0.25]), np.array([-0.5]), np.array([0.25])]


def test_llf_eigenvalue_hand_values():
    lx = fv_grid.llf_eigenvalue(_UM, _UP, True, _G4, 1.0, 0)
    ly = fv_grid.llf_eigenvalue(_UM, _UP, True, _G4, 1.0, 1)
    assert float(lx[0]) == 3.0 and float(ly[0]) == 5.0
    # swapping the sides gives the same speed (the max is symmetric)
    assert float(fv_grid.llf_eigenvalue(_UP, _UM, True, _G4, 1.0, 0)[0]) == 3.0
    # linear SWE: the constant sqrt(g H)
    assert fv_grid.llf_eigenvalue(_UM, _UP, False, 9.0, 4.0, 0) == 6.0


def test_llf_flux_hand_values():
    """F-hat = (F(U-) + F(U+))/2 - lambda (U+ - U-)/2 worked out by hand for the states above:
    F(U-) = (1/2, 9/4, -3/2), F(U+) = (-1/2, 9/8, -1/2), lambda = 3 -> (9/8, 51/16, -47/8);
    G(U-) = (-3, -3/2, 11), G(U+) = (1/4, -1/2, 3/8), lambda = 5 -> (1/2, 3/2, -39/16)."""
    Fx = fv_grid.llf(_UM, _UP, True, _G4, 1.0, 0)
    Gy = fv_grid.llf(_UM, _UP, True, _G4, 1.0, 1)
    assert [float(f[0]) for f in Fx] == [9 / 8, 51 / 16, -47 / 8]
    assert [float(f[0]) for f in Gy] == [1 / 2, 3 / 2, -39 / 16]
