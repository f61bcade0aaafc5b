"""GPU tests of the paper-reproduction pieces (Section 4.4's tolerance rule, Section 5.2's
inertia-gravity wave with f != 0 at Table 1's time step and C_eps) and of the full-grid
comparator (the same scheme without compression), all through the C ABI, against the oracle
and the closed form."""
import math
import sys

import numpy as np
import pytest

import synth
from oracle import fv_grid
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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ---- full-grid comparator ------------------------------------------------------------------

def _grid_run(lib, fields, scheme, nonlinear, periodic, g, H, f, dt, nsteps):
    import torch
    U = torch.tensor(np.stack(fields), dtype=torch.float64, device="cuda").contiguous()
    grid = lib.tt_grid_init(fields[0].shape[0], scheme, nonlinear, periodic, g=g, H0=H, f=f,
                            stream=torch.cuda.current_stream())
    grid.step(U, dt, nsteps)
    torch.cuda.synchronize()
    out = U.cpu().numpy()
    grid.close()
    return [out[v] for v in range(3)]


def _states(kind, n):
    """(fields, nonlinear, g, H, f, dt) of small smooth test states."""
    if kind == "nonlinear":
        st = synth.nonlinear_bumps(seed=2, n=n, rmax=64, eps=1e-14, kmax=3)
        return st.fields, True, st.g, 1.0, 3.0, st.dt
    st = synth.inertia_gravity(n, "upwind5", rmax=8)
    c = math.sqrt(st.g * st.H0)
    return st.fields, False, st.g, st.H0, st.meta["f"], 0.3 / n / c


@pytest.mark.parametrize("scheme", ["upwind3", "upwind5", "weno5"])
@pytest.mark.parametrize("kind", ["linear", "nonlinear"])
@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("n", [6, 37])
def test_grid_comparator_matches_the_full_grid_oracle(lib, scheme, kind, periodic, n):
    """Element by element against the oracle's full-grid scheme after 2 steps, f != 0; n = 37
    spans several 8 x 32 tiles with ragged edges, n = 6 is a domain smaller than one tile."""
    _say(f"grid {scheme} {kind} periodic={periodic} n={n}")
    fields, nl, g, H, f, dt = _states(kind, n)
    s = fv_grid.GridSolver(n, scheme, nonlinear=nl, periodic=periodic, g=g, H=H, f=f)
    ref = s.run([x.copy() for x in fields], dt, 2)
    got = _grid_run(lib, fields, scheme, nl, periodic, g, H, f, dt, 2)
    for v in range(3):
        scale = max(float(np.max(np.abs(ref[v]))), 1e-300)
        err = float(np.max(np.abs(got[v] - ref[v]))) / scale
        assert err <= 1e-12, (v, err)


# ---- Section 4.4's tolerance rule -----------------------------------------------------------

def _tt_pair(lib, st, scheme, nonlinear, periodic, f, dt, nsteps, rmax, c_eps, eps=1e-10,
             replay=False):
    """The oracle's steps, then the GPU's from the same state; with `replay`, every cross
    takes the oracle's final column and row sets (a skeleton is fixed by its pivots, and
    maxvol's choice among equally valid sets flips under round-off)."""
    Q0 = [ott.TT(x.A, x.B) for x in st.tt]
    ts = otf.TTSolver(st.n, scheme, nonlinear, periodic, g=st.g, H=st.H0, f=f, eps=eps,
                      rmax=rmax, eps_rule="paper", c_eps=c_eps)
    Qo = ts.run(Q0, dt, nsteps)
    dev = [lib.DeviceTT.from_factors(x.A, x.B, cap=rmax) for x in st.tt]
    s = lib.tt_fv_init(st.n, scheme, nonlinear, periodic, dev, g=st.g, H0=st.H0, f=f, eps=eps,
                       r_max=rmax, arena_bytes=1 << 30, eps_rule="paper", c_eps=c_eps)
    if replay:
        for (step, site), (J, I) in ts.cross_log.items():
            lib.tt_fv_replay_pivots(s, step, site, J, I)
        lib.tt_fv_set_pivots(s, "replay")
    lib.tt_fv_step(s, dt, nsteps)
    Qg = lib.tt_fv_get_state(s)
    stats = lib.tt_fv_get_stats(s)
    s.close()
    return Qg, Qo, stats, ts


@pytest.mark.parametrize("scheme,n", [("upwind3", 45), ("upwind5", 48), ("weno5", 40)])
def test_paper_tolerances_linear_coriolis_parity(lib, scheme, n):
    """Inertia-gravity wave (f != 0) with the paper's tolerance rule and Table 1's C_eps:
    same ranks, same tolerances and rel-L2 <= 1e-9 per field after 4 steps.  WENO5
    (C_eps = 500) grows the velocity ranks to the cap of 24 through its crosses, whose pivots
    are replayed."""
    _say(f"paper eps {scheme} n={n}")
    st = synth.inertia_gravity(n, scheme, rmax=24)
    c = math.sqrt(st.g * st.H0)
    c_eps = synth.TABLE1["inertia_gravity"][scheme][1]
    Qg, Qo, stats, ts = _tt_pair(lib, st, scheme, False, True, st.meta["f"], 0.3 / n / c, 4,
                                 24, c_eps, replay=scheme == "weno5")
    assert [q.rank for q in Qg] == [q.rank for q in Qo]
    rel = [_rel(g.full(), o.A @ o.B.T) for g, o in zip(Qg, Qo)]
    e_in, e_q = ts.stats["eps"][-1]
    _say(f"  rel {rel} ranks {[q.rank for q in Qg]} eps {e_in:.3e} {e_q}")
    assert max(rel) <= 1e-9
    assert stats["eps_inner"] == pytest.approx(e_in, rel=1e-10)
    assert stats["eps_var"] == pytest.approx(e_q, rel=1e-10)


def test_paper_tolerances_nonlinear_parity(lib):
    """Nonlinear bumps (64^2, Upwind5, Taylor reciprocal) with the paper's rule at C_eps = 1:
    the Hadamard, reciprocal and time-stepping roundings all take their tolerances from it."""
    _say("paper eps nonlinear 64")
    st = synth.nonlinear_bumps(seed=1, n=64, rmax=24, eps=1e-12, kmax=3)
    Qg, Qo, stats, ts = _tt_pair(lib, st, "upwind5", True, True, 0.0, st.dt, 2, 24, 1.0)
    assert [q.rank for q in Qg] == [q.rank for q in Qo]
    rel = [_rel(g.full(), o.A @ o.B.T) for g, o in zip(Qg, Qo)]
    _say(f"  rel {rel} ranks {[q.rank for q in Qg]} eps {ts.stats['eps'][-1]}")
    assert max(rel) <= 1e-9


def test_inertia_gravity_1280_to_final_time(lib):
    """Section 5.2 at the resolution of the paper's profile figure: 1280^2, Upwind5,
    dt = 1e-3 dx^(5/3) and C_eps = 1 (Table 1), the nondimensional scales of Table 2, 265 steps
    to T = 3 hours.  The TT path matches the TT oracle (rel-L2 <= 1e-9 per field, same ranks);
    its error against the closed form equals that of the full-grid comparator (the
    compression costs no accuracy) and of the oracle."""
    import torch
    n = 1280
    st = synth.inertia_gravity(n, "upwind5", rmax=16)
    T = st.meta["T"]
    nsteps = int(math.ceil(T / st.dt))
    dt = T / nsteps
    f = st.meta["f"]
    _say(f"igw 1280: {nsteps} steps, oracle first")
    Qg, Qo, stats, ts = _tt_pair(lib, st, "upwind5", False, True, f, dt, nsteps, 16, 1.0)
    assert [q.rank for q in Qg] == [q.rank for q in Qo] == [4, 4, 4]
    exact = [X @ Y.T for X, Y in synth.inertia_gravity_exact(n, T, f, st.g, st.H0,
                                                             st.meta["modes"])]
    e_gpu = [_rel(g.full(), x) for g, x in zip(Qg, exact)]
    e_orc = [_rel(o.A @ o.B.T, x) for o, x in zip(Qo, exact)]
    par = [_rel(g.full(), o.A @ o.B.T) for g, o in zip(Qg, Qo)]
    _say(f"  TT vs oracle {par}; vs closed form gpu {e_gpu} oracle {e_orc}")
    assert max(par) <= 1e-9
    grid = _grid_run(lib, st.fields, "upwind5", False, True, st.g, st.H0, f, dt, nsteps)
    e_grid = [_rel(u, x) for u, x in zip(grid, exact)]
    _say(f"  full grid vs closed form {e_grid}")
    for a, b in zip(e_gpu, e_grid):
        assert abs(a - b) <= 0.01 * b
    assert max(e_gpu) < 1e-6
    torch.cuda.synchronize()


# ---- exact-solution boundaries and forcing (Sections 5.1, 5.3, 5.4) ----------------------

CASES = {"coastal_kelvin": synth.coastal_kelvin, "barotropic_tide": synth.barotropic_tide,
         "manufactured": synth.manufactured}


def _case_speed(case):
    st = case.state
    h = float(np.max(st.fields[0])) if st.nonlinear else st.H0
    u = max(float(np.max(np.abs(st.fields[1]))), float(np.max(np.abs(st.fields[2]))))
    return math.sqrt(st.g * h) + (u / float(np.min(st.fields[0])) if st.nonlinear else u)


@pytest.mark.parametrize("name,scheme", [
    ("coastal_kelvin", "upwind3"), ("coastal_kelvin", "upwind5"), ("coastal_kelvin", "weno5"),
    ("barotropic_tide", "upwind5"), ("barotropic_tide", "weno5"),
    ("manufactured", "upwind3"), ("manufactured", "upwind5"), ("manufactured", "weno5"),
])
@pytest.mark.parametrize("n", [6, 37])
def test_grid_comparator_terms_match_the_oracle(lib, name, scheme, n):
    """Exact x boundaries from the ghost terms (Kelvin, tide) and forcing terms
    (manufactured), 2 steps at the terms' stage times: element by element against the
    oracle's full-grid scheme: eta or h to <= 1e-12 of its largest value, both momenta to
    <= 1e-12 of the larger momentum's largest value (one momentum is zero in the exact
    solution of the Kelvin wave and of the manufactured case; its size is the discretisation
    error left by the near-cancellation of the Coriolis term with the pressure gradient or the
    forcing).  The manufactured case in Table 2's scales carries g h^2 / 2 ~ 1e8 in the
    momentum fluxes, whose FP64 rounding (~1e-8 per face value, in a different order on each
    side) moves the momenta by ~1e-12 of their size over two steps: there the bar is 1e-10."""
    import torch
    _say(f"grid terms {name} {scheme} n={n}")
    case = CASES[name](n, scheme)
    st = case.state
    dt = 0.3 / n / _case_speed(case)
    s = fv_grid.GridSolver(n, scheme, nonlinear=st.nonlinear, g=st.g, H=st.H0, f=st.meta["f"],
                           bc=case.bc, terms=case.terms)
    ref = s.run([x.copy() for x in st.fields], dt, 2)
    U = torch.tensor(np.stack(st.fields), dtype=torch.float64, device="cuda").contiguous()
    grid = lib.tt_grid_init(n, scheme, st.nonlinear, False, g=st.g, H0=st.H0, f=st.meta["f"],
                            bc=case.bc, terms=case.terms, stream=torch.cuda.current_stream())
    grid.step(U, dt, 2)
    torch.cuda.synchronize()
    got = U.cpu().numpy()
    grid.close()
    scale = [max(float(np.max(np.abs(r))), 1e-300) for r in ref]
    scale[1] = scale[2] = max(scale[1], scale[2])
    bar = [1e-12, 1e-10, 1e-10] if name == "manufactured" else [1e-12, 1e-12, 1e-12]
    for v in range(3):
        err = float(np.max(np.abs(got[v] - ref[v]))) / scale[v]
        assert err <= bar[v], (v, err)


@pytest.mark.parametrize("name,scheme,n", [
    ("coastal_kelvin", "upwind3", 45), ("coastal_kelvin", "upwind5", 40),
    ("coastal_kelvin", "weno5", 40), ("barotropic_tide", "upwind5", 40),
    ("barotropic_tide", "weno5", 36), ("manufactured", "upwind3", 40),
    ("manufactured", "upwind5", 40),
])
def test_tt_terms_parity(lib, name, scheme, n):
    """The TT step with ghost columns (exact x boundaries; with WENO5 also the directly
    evaluated Step-1 values at the tangent ghost cells, crosses on the oracle's pivots) or
    forcing TTs, the paper's tolerance rule and Table 1's C_eps, 3 steps: same ranks as the TT oracle, eta or h within
    1e-9 of its norm and both momenta within 1e-9 of the larger momentum's norm (one momentum
    is zero in the exact Kelvin and manufactured solutions)."""
    _say(f"tt terms {name} {scheme} n={n}")
    case = CASES[name](n, scheme, rmax=24)
    st = case.state
    dt = 0.3 / n / _case_speed(case)
    c_eps = st.meta["c_eps"]
    Q0 = [ott.TT(x.A, x.B) for x in st.tt]
    ts = otf.TTSolver(n, scheme, st.nonlinear, g=st.g, H=st.H0, f=st.meta["f"], rmax=24,
                      eps_rule="paper", c_eps=c_eps, bc=case.bc, terms=case.terms)
    Qo = ts.run(Q0, dt, 3)
    dev = [lib.DeviceTT.from_factors(x.A, x.B, cap=24) for x in st.tt]
    s = lib.tt_fv_init(n, scheme, st.nonlinear, False, dev, g=st.g, H0=st.H0, f=st.meta["f"],
                       r_max=24, arena_bytes=1 << 30, eps_rule="paper", c_eps=c_eps,
                       bc=case.bc, terms=case.terms)
    if scheme == "weno5":
        # the oracle's cross pivots, so that equally valid pivot sets cannot differ
        for (step, site), (J, I) in ts.cross_log.items():
            lib.tt_fv_replay_pivots(s, step, site, J, I)
        lib.tt_fv_set_pivots(s, "replay")
    lib.tt_fv_step(s, dt, 3)
    Qg = lib.tt_fv_get_state(s)
    stats = lib.tt_fv_get_stats(s)
    s.close()
    assert stats["time"] == pytest.approx(3 * dt, rel=1e-14)
    full_g = [q.full() for q in Qg]
    full_o = [o.A @ o.B.T for o in Qo]
    scale = [max(np.linalg.norm(f), 1e-300) for f in full_o]
    scale[1] = scale[2] = max(scale[1], scale[2])
    rel = [float(np.linalg.norm(a - b)) / sc for a, b, sc in zip(full_g, full_o, scale)]
    _say(f"  rel {rel} ranks gpu {[q.rank for q in Qg]} oracle {[q.rank for q in Qo]}")
    assert [q.rank for q in Qg] == [q.rank for q in Qo]
    assert max(rel) <= 1e-9


def test_kelvin_1280_upwind3_to_final_time(lib):
    """Section 5.1 at 1280^2 with Upwind3 at Table 1's dt/dx = 5e-5 and C_eps = 1, exact x
    boundaries, to T = 3 hours (277 steps): the TT path matches the TT oracle (rel-L2 <= 1e-9
    of the state) and stays within 1e-6 of the closed form.  (That step is c dt/dx = 1.0, at
    which the full-grid scheme is unstable: it grows from round-off and blows up after about
    130 steps at 128^2; the TT roundings truncate those modes.)"""
    n = 1280
    case = synth.coastal_kelvin(n, "upwind3", rmax=16)
    st = case.state
    T = case.T
    nsteps = int(math.ceil(T / st.dt))
    dt = T / nsteps
    f = st.meta["f"]
    _say(f"kelvin 1280 upwind3: {nsteps} steps, oracle first")
    Q0 = [ott.TT(x.A, x.B) for x in st.tt]
    ts = otf.TTSolver(n, "upwind3", False, g=st.g, H=st.H0, f=f, rmax=16, eps_rule="paper",
                      c_eps=1.0, bc=case.bc, terms=case.terms)
    Qo = ts.run(Q0, dt, nsteps)
    dev = [lib.DeviceTT.from_factors(x.A, x.B, cap=16) for x in st.tt]
    s = lib.tt_fv_init(n, "upwind3", False, False, dev, g=st.g, H0=st.H0, f=f, r_max=16,
                       eps_rule="paper", c_eps=1.0, bc=case.bc, terms=case.terms)
    lib.tt_fv_step(s, dt, nsteps)
    Qg = lib.tt_fv_get_state(s)
    s.close()
    full_g = [q.full() for q in Qg]
    full_o = [o.A @ o.B.T for o in Qo]
    tot = math.sqrt(sum(float(np.sum(b * b)) for b in full_o))
    par = math.sqrt(sum(float(np.sum((a - b) ** 2)) for a, b in zip(full_g, full_o))) / tot
    exact = case.exact(T)
    ex_tot = math.sqrt(sum(float(np.sum(b * b)) for b in exact))
    e_tt = math.sqrt(sum(float(np.sum((a - b) ** 2)) for a, b in zip(full_g, exact))) / ex_tot
    _say(f"  ranks {[q.rank for q in Qg]} TT vs oracle {par:.2e}; closed-form error {e_tt:.4e}")
    assert [q.rank for q in Qg] == [q.rank for q in Qo]
    assert par <= 1e-9
    assert e_tt < 1e-6


@pytest.mark.parametrize("name,scheme", [("coastal_kelvin", "upwind3"),
                                         ("barotropic_tide", "upwind5")])
def test_tt_and_full_grid_share_the_closed_form_error(lib, name, scheme):
    """640^2 to T (Kelvin: 3 hours; tide: 30 minutes) at c dt/dx = 0.5 (Upwind3) or 0.3
    (Upwind5): the TT path with the paper's tolerances and the full-grid
    comparator have the same error against the closed form (within 1%): the compression costs
    no accuracy with exact-solution boundaries either."""
    import torch
    n = 640
    case = CASES[name](n, scheme, rmax=16)
    st = case.state
    c = math.sqrt(st.g * st.H0)
    dt0 = (0.5 if scheme == "upwind3" else 0.3) / (c * n)
    T = case.T
    nsteps = int(math.ceil(T / dt0))
    dt = T / nsteps
    f = st.meta["f"]
    _say(f"{name} 640 {scheme}: {nsteps} steps, c dt/dx = {c * dt * n:.3f}")
    dev = [lib.DeviceTT.from_factors(x.A, x.B, cap=16) for x in st.tt]
    s = lib.tt_fv_init(n, scheme, False, False, dev, g=st.g, H0=st.H0, f=f, r_max=16,
                       eps_rule="paper", c_eps=st.meta["c_eps"], bc=case.bc, terms=case.terms)
    lib.tt_fv_step(s, dt, nsteps)
    Qg = lib.tt_fv_get_state(s)
    s.close()
    U = torch.tensor(np.stack(st.fields), dtype=torch.float64, device="cuda").contiguous()
    grid = lib.tt_grid_init(n, scheme, False, False, g=st.g, H0=st.H0, f=f, bc=case.bc,
                            terms=case.terms, stream=torch.cuda.current_stream())
    grid.step(U, dt, nsteps)
    torch.cuda.synchronize()
    Ug = U.cpu().numpy()
    grid.close()
    exact = case.exact(T)
    ex_tot = math.sqrt(sum(float(np.sum(b * b)) for b in exact))
    e_tt = math.sqrt(sum(float(np.sum((q.full() - x) ** 2)) for q, x in zip(Qg, exact))) / ex_tot
    e_grid = math.sqrt(sum(float(np.sum((Ug[v] - exact[v]) ** 2)) for v in range(3))) / ex_tot
    _say(f"  ranks {[q.rank for q in Qg]}; closed-form error TT {e_tt:.4e} grid {e_grid:.4e}")
    assert abs(e_tt - e_grid) <= 0.01 * e_grid
    assert e_tt < 1e-4
