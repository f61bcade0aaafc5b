"""Batched ensemble: members stepped together equal the same members stepped alone."""
import sys

import numpy as np
import pytest

import synth

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


def _members(lib, workers):
    specs = [(synth.nonlinear_bumps(seed=1001, n=48, rmax=12, eps=1e-10), "upwind5", True, 12),
             (synth.nonlinear_bumps(seed=1002, n=64, rmax=20, eps=1e-10), "upwind5", False, 20),
             (synth.linear_gaussian(seed=1003, n=40, rmax=8), "upwind3", True, 8),
             (synth.nonlinear_bumps(seed=1004, n=32, rmax=16, eps=1e-8), "weno5", True, 16)]
    out = []
    for st, scheme, periodic, r in specs:
        dev = [lib.DeviceTT.from_factors(f.A, f.B, cap=r) for f in st.tt]
        s = lib.tt_fv_init(st.n, scheme, st.nonlinear, periodic, dev, g=st.g, H0=st.H0,
                           eps=1e-10 if scheme != "weno5" else 1e-8, r_max=r, workers=workers,
                           arena_bytes=1 << 28)
        out.append((s, st.dt))
    return out


def test_ensemble_equals_members_alone(lib):
    _say("ensemble of 4 members vs alone")
    alone = _members(lib, 4)
    for s, dt in alone:
        lib.tt_fv_step(s, dt, 2)
    ref = [[q.full() for q in lib.tt_fv_get_state(s)] for s, _ in alone]
    for s, _ in alone:
        s.close()
    ens = lib.tt_ens_create(workers=6, arena_bytes_per_worker=1 << 28)
    members = _members(lib, -1)
    lib.tt_ens_step(ens, [m for m, _ in members], [dt for _, dt in members], nsteps=2,
                    concurrency=3)
    for (s, _), r in zip(members, ref):
        got = [q.full() for q in lib.tt_fv_get_state(s)]
        for a, b in zip(got, r):
            assert np.array_equal(a, b)
        with pytest.raises(RuntimeError, match="ensemble"):
            lib.tt_fv_step(s, 1e-4, 1)          # workers = -1: steps only inside an ensemble
        s.close()
    ens.close()
