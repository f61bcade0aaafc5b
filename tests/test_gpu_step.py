"""GPU parity of the full TT-FV SSP-RK3 step against the CPU oracle (through the C ABI)."""
import sys

import numpy as np
import pytest

import synth
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


def field_rel(Qg, Qo):
    return [np.linalg.norm(g.full() - o.full()) / max(np.linalg.norm(o.full()), 1e-300)
            for g, o in zip(Qg, Qo)]


def run_both(lib, st, scheme, nonlinear, periodic, eps, rmax, nsteps, taylor=8, recip="taylor",
             precision="f64"):
    Q0 = [ott.TT(f.A, f.B) for f in st.tt]
    ts = otf.TTSolver(st.n, scheme, nonlinear, periodic, g=st.g, H=st.H0, eps=eps, rmax=rmax,
                      taylor_terms=taylor, recip=recip)
    Qo = ts.run(Q0, st.dt, nsteps)
    dev = [lib.DeviceTT.from_factors(f.A, f.B, cap=rmax) for f in st.tt]
    s = lib.tt_fv_init(st.n, scheme, nonlinear, periodic, dev, g=st.g, H0=st.H0, eps=eps,
                       r_max=rmax, taylor_terms=taylor, recip=recip, arena_bytes=1 << 30,
                       precision=precision)
    lib.tt_fv_step(s, st.dt, nsteps)
    Qg = lib.tt_fv_get_state(s)
    stats = lib.tt_fv_get_stats(s)
    s.close()
    return Qg, Qo, stats, ts


def test_linear_gaussian_64_parity(lib):
    """64^2 linear Gaussian, Upwind3, rank cap 8, tol 1e-12, the whole run of 100 steps
    (trajectory parity): rel-L2 <= 1e-9 per field."""
    _say("linear 64 upwind3, 100 steps")
    st = synth.linear_gaussian(seed=0)
    Qg, Qo, stats, ts = run_both(lib, st, "upwind3", False, True, 1e-12, 8, 100)
    assert [q.rank for q in Qg] == [q.rank for q in Qo]
    r = field_rel(Qg, Qo)
    _say(f"  rel {r}")
    assert max(r) <= 1e-9


@pytest.mark.parametrize("periodic", [True, False])
def test_nonlinear_upwind5_parity(lib, periodic):
    """Nonlinear bumps on 96^2 (several tiles, ragged), Upwind5, Taylor 8 terms, rank cap 16."""
    _say(f"nonlinear 96 upwind5 periodic={periodic}")
    st = synth.nonlinear_bumps(seed=1, n=96, rmax=16, eps=1e-10)
    Qg, Qo, stats, ts = run_both(lib, st, "upwind5", True, periodic, 1e-10, 16, 2)
    r = field_rel(Qg, Qo)
    _say(f"  rel {r} ranks {[q.rank for q in Qg]} vs {[q.rank for q in Qo]}")
    assert max(r) <= 1e-9


def _full_rank_state(n, seed):
    rng = np.random.default_rng(seed)
    U = [1.0 + 0.02 * rng.standard_normal((n, n)), 0.01 * rng.standard_normal((n, n)),
         0.01 * rng.standard_normal((n, n))]
    tts = []
    for F in U:
        u, s, vt = np.linalg.svd(F)
        tts.append(synth.Factored(u * s, vt.T.copy()))
    return U, tts


@pytest.mark.parametrize("periodic,recip", [(True, "taylor"), (False, "taylor"),
                                            (False, "cross")])
def test_weno5_unique_parity(lib, periodic, recip):
    """WENO5 on a 16^2 grid with full-rank states: every cross sees all columns, so the
    cross is exact, the result is unique, and GPU and oracle must agree tightly."""
    _say(f"weno5 16 full rank periodic={periodic} recip={recip}")
    n = 16
    U, tts = _full_rank_state(n, 11)
    st = synth.State("full", n, True, periodic, 9.81, 1.0, U, tts, 2e-4, {})
    Qg, Qo, stats, ts = run_both(lib, st, "weno5", True, periodic, 1e-14, 64, 1, taylor=30,
                                 recip=recip)
    r = field_rel(Qg, Qo)
    _say(f"  rel {r}")
    assert max(r) <= 1e-9


def run_replayed(lib, st, scheme, periodic, eps, rmax, nsteps, recip="taylor",
                 precision="f64", cross_drop=1e-13, taylor=8):
    """The oracle's steps, then the GPU's from the same state with every cross given the
    oracle's final column and row sets (Section 3.3: a skeleton is fixed by its pivots).  At
    the rank cap several pivot sets are equally valid and maxvol's choice among them flips
    under round-off, so replaying one set is what makes the two steps comparable."""
    Q0 = [ott.TT(f.A, f.B) for f in st.tt]
    ts = otf.TTSolver(st.n, scheme, True, periodic, g=st.g, H=st.H0, eps=eps, rmax=rmax,
                      taylor_terms=taylor, recip=recip, cross_drop=cross_drop)
    Qo = ts.run(Q0, st.dt, nsteps)
    dev = [lib.DeviceTT.from_factors(f.A, f.B, cap=rmax) for f in st.tt]
    s = lib.tt_fv_init(st.n, scheme, True, periodic, dev, g=st.g, H0=st.H0, eps=eps,
                       r_max=rmax, taylor_terms=taylor, recip=recip, arena_bytes=1 << 30,
                       precision=precision)
    for (step, site), (J, I) in ts.cross_log.items():
        lib.tt_fv_replay_pivots(s, step, site, J, I)
    lib.tt_fv_set_pivots(s, "replay")
    lib.tt_fv_step(s, st.dt, nsteps)
    Qg = lib.tt_fv_get_state(s)
    s.close()
    return Qg, Qo, ts


def pivot_agreement(lib, st, scheme, periodic, eps, rmax, ts, recip="taylor"):
    """One plain GPU step (its own maxvol pivots): the fraction of cross sites whose final
    column sets and row sets equal the oracle's, and the GPU state."""
    dev = [lib.DeviceTT.from_factors(f.A, f.B, cap=rmax) for f in st.tt]
    s = lib.tt_fv_init(st.n, scheme, True, periodic, dev, g=st.g, H0=st.H0, eps=eps,
                       r_max=rmax, recip=recip, arena_bytes=1 << 30)
    lib.tt_fv_step(s, st.dt, 1)
    same_j = same_i = total = 0
    for (step, site), (J, I) in ts.cross_log.items():
        if step != 0:
            continue
        g = lib.tt_fv_get_pivots(s, site)
        total += 1
        same_j += set(g[0].tolist()) == set(J.tolist())
        same_i += set(g[1].tolist()) == set(I.tolist())
    Qg = lib.tt_fv_get_state(s)
    s.close()
    return same_j / total, same_i / total, total, Qg


@pytest.mark.parametrize("periodic", [True, False])
def test_weno5_capped_replay_parity(lib, periodic):
    """Nonlinear bumps on 64^2, WENO5 by crosses with the rank cap (24) binding, tol 1e-8,
    two steps.  With the oracle's pivots replayed the GPU must match it to 1e-9 per field.
    Without replay (the GPU's own maxvol pivots) the result must be as close to the
    full-grid scheme as the oracle's: within twice its distance plus 20 eps."""
    from oracle import fv_grid
    _say(f"weno5 64 capped, replayed pivots, periodic={periodic}")
    st = synth.nonlinear_bumps(seed=2, n=64, rmax=24, eps=1e-8)
    Qg, Qo, ts = run_replayed(lib, st, "weno5", periodic, 1e-8, 24, 2)
    r = field_rel(Qg, Qo)
    _say(f"  replayed rel {r} ranks {[q.rank for q in Qg]} vs {[q.rank for q in Qo]}")
    assert max(r) <= 1e-9
    # the GPU's own pivots: agreement with the oracle's, and accuracy against the grid
    ts1 = otf.TTSolver(st.n, "weno5", True, periodic, g=st.g, eps=1e-8, rmax=24)
    Qo1 = ts1.run([ott.TT(f.A, f.B) for f in st.tt], st.dt, 1)
    aj, ai, nsite, Qp = pivot_agreement(lib, st, "weno5", periodic, 1e-8, 24, ts1)
    Ug = fv_grid.GridSolver(st.n, "weno5", True, periodic, g=st.g).step(
        [f.full() for f in st.tt], st.dt)
    _say(f"  own pivots: {nsite} sites, equal column sets {aj:.2f}, equal row sets {ai:.2f}")
    for c in range(3):
        ref = np.linalg.norm(Ug[c])
        e_o = np.linalg.norm(Qo1[c].full() - Ug[c]) / ref
        e_g = np.linalg.norm(Qp[c].full() - Ug[c]) / ref
        _say(f"  var {c}: oracle-vs-grid {e_o:.3e} gpu-vs-grid {e_g:.3e}")
        assert e_g <= 2.0 * e_o + 20 * 1e-8


def test_dam_break_cross_reciprocal_replay_parity(lib):
    """Dam break (h from 0.5 to 1.5, walls) on 48^2: WENO5 crosses and 1/h by cross (reading
    R7), cap 24, tol 1e-8, two steps, the oracle's pivots replayed: rel-L2 <= 1e-9 per
    field, and for h also on its deviation from the mean."""
    _say("dam break 48 weno5 cross reciprocal, replayed pivots")
    st = synth.dam_break(seed=0, n=48, rmax=24, eps=1e-8, width=0.05)
    Qg, Qo, ts = run_replayed(lib, st, "weno5", False, 1e-8, 24, 2, recip="cross")
    r = field_rel(Qg, Qo)
    hg, ho = Qg[0].full(), Qo[0].full()
    dh = np.linalg.norm(hg - ho) / np.linalg.norm(ho - ho.mean())
    _say(f"  rel {r}, h deviation {dh:.2e}, ranks {[q.rank for q in Qg]}")
    assert max(r) <= 1e-9 and dh <= 1e-9


def test_dam_break_fp32_contractions_replay(lib):
    """Mixed precision on the 48^2 dam break (WENO5 crosses, 1/h by cross, walls, cap 24, tol
    1e-8, two steps): FP32 contractions against the FP64 oracle with the same cross drop
    rule (1e-6, reading R12) and its pivots replayed.  Gate: rel-L2 <= 1e-4 per field, and
    for h also on its deviation from the mean."""
    _say("dam break 48 weno5 cross reciprocal fp32, replayed pivots")
    st = synth.dam_break(seed=0, n=48, rmax=24, eps=1e-8, width=0.05)
    Qg, Qo, ts = run_replayed(lib, st, "weno5", False, 1e-8, 24, 2, recip="cross",
                              precision="f32", cross_drop=1e-6)
    r = field_rel(Qg, Qo)
    hg, ho = Qg[0].full(), Qo[0].full()
    dh = np.linalg.norm(hg - ho) / np.linalg.norm(ho - ho.mean())
    _say(f"  per-field rel {r}, h deviation {dh:.2e}")
    assert max(r) <= 1e-4 and dh <= 1e-4


def test_nonlinear_upwind5_fp32_contractions(lib):
    """Mixed precision: FP32 contractions, FP64 SVD / Taylor scalars, on the 96^2 bumps
    (Upwind5, periodic, cap 24, tol 1e-10, 2 steps).  Gate: rel-L2 <= 1e-4 per field against
    the FP64 oracle, and for h also on the deviation from its mean."""
    _say("nonlinear 96 upwind5 fp32")
    st = synth.nonlinear_bumps(seed=1, n=96, rmax=24, eps=1e-10)
    Qg, Qo, stats, ts = run_both(lib, st, "upwind5", True, True, 1e-10, 24, 2, precision="f32")
    r = field_rel(Qg, Qo)
    hg, ho = Qg[0].full(), Qo[0].full()
    dev = np.linalg.norm(hg - ho) / np.linalg.norm(ho - ho.mean())
    _say(f"  rel {r}, h deviation {dev:.2e}, ranks {[q.rank for q in Qg]}")
    assert max(r) <= 1e-4 and dev <= 1e-4


@pytest.mark.parametrize("scheme,recip", [("upwind5", "taylor"), ("weno5", "cross")])
def test_lake_at_rest_is_preserved(lib, scheme, recip):
    """Degenerate state: h = 1, hu = hv = 0 (rank-1 and zero TTs) between walls stays at rest
    to round-off after two steps (the flux differences of a constant state vanish)."""
    _say(f"lake at rest 40^2 {scheme} {recip}")
    n = 40
    ones = np.ones((n, 1))
    tts = [synth.Factored(ones, ones), synth.Factored(np.zeros((n, 1)), np.zeros((n, 1))),
           synth.Factored(np.zeros((n, 1)), np.zeros((n, 1)))]
    U = [np.ones((n, n)), np.zeros((n, n)), np.zeros((n, n))]
    st = synth.State("rest", n, True, False, 9.81, 1.0, U, tts, 1e-3, {})
    dev = [lib.DeviceTT.from_factors(f.A, f.B, cap=8) for f in st.tt]
    s = lib.tt_fv_init(n, scheme, True, False, dev, g=st.g, eps=1e-10, r_max=8, recip=recip,
                       arena_bytes=1 << 28)
    lib.tt_fv_step(s, st.dt, 2)
    Qg = lib.tt_fv_get_state(s)
    s.close()
    assert np.max(np.abs(Qg[0].full() - 1.0)) <= 1e-13
    assert np.max(np.abs(Qg[1].full())) <= 1e-13 and np.max(np.abs(Qg[2].full())) <= 1e-13


def test_dam_break_2048_mass_and_positivity(lib):
    """The 2048^2 dam break of the throughput run (WENO5 crosses, 1/h by cross, walls, cap 64,
    tol 1e-8, FP64), one step in the bench's launch configuration.  The oracle cannot take
    this step in test time, so properties that hold at any size are checked: the walls
    conserve mass up to the roundings' relative changes (a few eps per stage, bound 1e-6),
    h stays within its initial range up to 1e-3 (WENO5 is essentially non-oscillatory),
    and the ranks respect the cap."""
    _say("dam break 2048 one step: mass, range, ranks")
    st = synth.dam_break(seed=0, n=2048, rmax=64, eps=1e-8)
    dev = [lib.DeviceTT.from_factors(f.A, f.B, cap=64) for f in st.tt]
    s = lib.tt_fv_init(2048, "weno5", True, False, dev, g=st.g, eps=1e-8, r_max=64,
                       recip="cross")
    lib.tt_fv_step(s, st.dt, 1)
    Qg = lib.tt_fv_get_state(s)
    s.close()
    h0 = st.tt[0].A @ st.tt[0].B.T
    h1 = Qg[0].full()
    m0, m1 = h0.sum(), h1.sum()
    dh = np.max(np.abs(h1 - h0))
    _say(f"  mass drift {abs(m1 - m0) / m0:.2e}, max |dh| {dh:.2e}, "
         f"h in [{h1.min():.6f}, {h1.max():.6f}], ranks {[q.rank for q in Qg]}")
    assert dh > 1e-6                       # the step moved the front
    assert abs(m1 - m0) / m0 <= 1e-6
    assert h1.min() >= h0.min() - 1e-3 and h1.max() <= h0.max() + 1e-3
    assert all(1 <= q.rank <= 64 for q in Qg)


def test_bumps_1024_restart_parity_full_size(lib):
    """The throughput workload itself (1024^2 bumps, Upwind5, Taylor 8 terms, cap 32, tol
    1e-10, FP64) with the default launch configuration (8 worker streams, helper streams for
    the Taylor sums): one step from the initial state against the oracle's step, rel-L2 per
    field <= 1e-9, and for h also on its deviation from the mean."""
    _say("bumps 1024 restart parity (oracle step ~30 s)")
    st = synth.nonlinear_bumps(seed=0, n=1024, rmax=32, eps=1e-10)
    Qg, Qo, stats, ts = run_both(lib, st, "upwind5", True, True, 1e-10, 32, 1)
    r = field_rel(Qg, Qo)
    hg, ho = Qg[0].full(), Qo[0].full()
    dh = np.linalg.norm(hg - ho) / np.linalg.norm(ho - ho.mean())
    _say(f"  rel {r}, h deviation {dh:.2e}, ranks {[q.rank for q in Qg]} vs "
         f"{[q.rank for q in Qo]}")
    assert max(r) <= 1e-9 and dh <= 1e-9


def test_bumps_trajectory_and_restart_parity(lib):
    """The throughput workload's scheme on 64^2 bumps (Upwind5, Taylor 8 terms, cap 24
    binding, tol 1e-10, periodic).  Trajectory parity: the GPU's 12 steps against the
    oracle's at steps 4, 8 and 12.  Restart parity: the oracle's states at steps 4 and 8
    fed to a fresh GPU solver and a fresh oracle solver for one step.  Gate 1e-9 per field
    throughout, and for h also on its deviation from the mean."""
    _say("bumps 64 trajectory (12 steps) and restarts at steps 4 and 8")
    n, rmax, eps = 64, 24, 1e-10
    st = synth.nonlinear_bumps(seed=5, n=n, rmax=rmax, eps=eps)
    kw = dict(g=st.g, H=st.H0, eps=eps, rmax=rmax, taylor_terms=8)
    ts = otf.TTSolver(n, "upwind5", True, True, **kw)
    Q = [ott.TT(f.A, f.B) for f in st.tt]
    snaps = {}
    for k in range(1, 13):
        Q = ts.step(Q, st.dt)
        if k % 4 == 0:
            snaps[k] = Q

    def gpu_solver(tts):
        dev = [lib.DeviceTT.from_factors(t.A, t.B, cap=rmax) for t in tts]
        return lib.tt_fv_init(n, "upwind5", True, True, dev, g=st.g, H0=st.H0, eps=eps,
                              r_max=rmax, taylor_terms=8, arena_bytes=1 << 30)

    def check(Qg, Qo, what):
        r = field_rel(Qg, Qo)
        hg, ho = Qg[0].full(), Qo[0].full()
        dh = np.linalg.norm(hg - ho) / np.linalg.norm(ho - ho.mean())
        _say(f"  {what}: rel {r}, h deviation {dh:.2e}")
        assert max(r) <= 1e-9 and dh <= 1e-9, what

    s = gpu_solver([ott.TT(f.A, f.B) for f in st.tt])
    for k in (4, 8, 12):
        lib.tt_fv_step(s, st.dt, 4)
        check(lib.tt_fv_get_state(s), snaps[k], f"trajectory step {k}")
    s.close()
    for k in (4, 8):
        ref = otf.TTSolver(n, "upwind5", True, True, **kw).step(snaps[k], st.dt)
        s = gpu_solver(snaps[k])
        lib.tt_fv_step(s, st.dt, 1)
        check(lib.tt_fv_get_state(s), ref, f"restart from step {k}")
        s.close()


@pytest.mark.parametrize("periodic", [True, False])
def test_lf_cross_flux_parity(lib, periodic):
    """LF-cross (the whole LLF flux vector of a direction by one cross over face x (component,
    quadrature column), the alternative Section 4.2 contrasts with its products): 64^2
    nonlinear bumps, Upwind5, cap 24, tol 1e-10, two steps, the oracle's pivots replayed:
    rel-L2 <= 1e-9 per field and equal ranks."""
    _say(f"lf-cross 64 periodic={periodic}")
    st = synth.nonlinear_bumps(seed=5, n=64, rmax=24, eps=1e-10, kmax=3)
    Q0 = [ott.TT(f.A, f.B) for f in st.tt]
    ts = otf.TTSolver(64, "upwind5", True, periodic, g=st.g, eps=1e-10, rmax=24,
                      flux="lf_cross")
    Qo = ts.run(Q0, st.dt, 2)
    dev = [lib.DeviceTT.from_factors(f.A, f.B, cap=24) for f in st.tt]
    s = lib.tt_fv_init(64, "upwind5", True, periodic, dev, g=st.g, eps=1e-10, r_max=24,
                       arena_bytes=1 << 30, flux="lf_cross")
    for (step, site), (J, I) in ts.cross_log.items():
        lib.tt_fv_replay_pivots(s, step, site, J, I)
    lib.tt_fv_set_pivots(s, "replay")
    lib.tt_fv_step(s, st.dt, 2)
    Qg = lib.tt_fv_get_state(s)
    stats = lib.tt_fv_get_stats(s)
    s.close()
    r = field_rel(Qg, Qo)
    _say(f"  rel {r} ranks {[q.rank for q in Qg]} vs {[q.rank for q in Qo]}, "
         f"crosses {stats['crosses']}, roundings {stats['roundings']}")
    assert [q.rank for q in Qg] == [q.rank for q in Qo]
    assert max(r) <= 1e-9


def test_cfl_from_the_tts(lib):
    """tt_fv_max_speed / tt_fv_cfl_dt (rook pivoting on the TTs from h's maxvol columns) equal
    the oracle's estimate and the maxima of the TT state's cell values on the 1024^2 bumps
    workload, and on its state after 3 steps; the step they give matches the workload's CFL 0.4
    step (computed from the uncompressed cell averages, 1e-10 away)."""
    _say("cfl from the tts, 1024 bumps")
    st = synth.nonlinear_bumps(seed=0, n=1024, rmax=32, eps=1e-10)
    dev = [lib.DeviceTT.from_factors(f.A, f.B, cap=32) for f in st.tt]
    s = lib.tt_fv_init(1024, "upwind5", True, True, dev, g=st.g, eps=1e-10, r_max=32)
    ts = otf.TTSolver(1024, "upwind5", True, True, g=st.g, eps=1e-10, rmax=32)
    Q0 = [ott.TT(f.A, f.B) for f in st.tt]
    sx, sy = lib.tt_fv_max_speed(s)
    h, hu, hv = [q.A @ q.B.T for q in Q0]          # the TT state's own cell values
    true = (float(np.max(np.abs(hu / h) + np.sqrt(st.g * h))),
            float(np.max(np.abs(hv / h) + np.sqrt(st.g * h))))
    orc = (ts.max_speed(Q0, 0), ts.max_speed(Q0, 1))
    _say(f"  gpu {sx, sy} oracle {orc} full field {true}")
    assert (sx, sy) == pytest.approx(orc, rel=1e-13)
    assert (sx, sy) == pytest.approx(true, rel=1e-12)
    assert lib.tt_fv_cfl_dt(s, 0.4) == pytest.approx(st.dt, rel=1e-9)
    lib.tt_fv_step(s, st.dt, 3)
    Qg = lib.tt_fv_get_state(s)
    F = [q.full() for q in Qg]
    true3 = float(np.max(np.abs(F[1] / F[0]) + np.sqrt(st.g * F[0])))
    s3 = lib.tt_fv_max_speed(s)[0]
    s.close()
    assert s3 == pytest.approx(true3, rel=1e-12)
