#!/usr/bin/env python3
"""Throughput of the tensor-train finite-volume SSP-RK3 step on one MI355X.

Workload: nonlinear shallow water on [0,1]^2, 1024 x 1024 cells, periodic, Upwind5 with
3-point Gauss-Legendre faces, Taylor reciprocal of h (8 terms), TT rank cap 32, rounding
tolerance 1e-10, FP64; initial state h = 1 + 4 Gaussian bumps, u, v smooth random Fourier
fields (seed 0), dt from CFL 0.4.

One "step" is one full SSP-RK3 step of the TT solver.  value = cells * steps / seconds over
the timed steps (cell-updates/s).  Before timing, one step from the initial state is
checked against the CPU oracle (relative L2 error per field), and that oracle step, timed on
the host, is the cpu_baseline.  The dominant kernel is timed live with HIP events on the
streams it runs on, which gives the roofline line.

    python bench.py [--gpus 1] [--steps 5] [--warmup 2] [--no-cpu] [--timed-kernel NAME]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per RK step at fixed rel-L2 vs FP64 oracle; % HBM/MFMA peak"
PEAK_FP64_VECTOR_TFLOPS = 78.6      # MI355X FP64 vector (no MFMA used by this kernel)
PEAK_HBM_GBS = 8000.0
PARITY_GATE = 1e-9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle step")
    ap.add_argument("--timed-kernel", default="jacobi",
                    help="kernel family timed with HIP events ('' = none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); a single TT-FV member "
              "does not shard across GPUs in this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_2408_03483_amd import ttfv

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    n, rmax, eps, K = args.n, 32, 1e-10, 8
    st = synth.nonlinear_bumps(seed=0, n=n, rmax=rmax, eps=eps)
    dev = [ttfv.DeviceTT.from_factors(f.A, f.B, cap=rmax) for f in st.tt]
    s = ttfv.tt_fv_init(n, "upwind5", True, True, dev, g=st.g, eps=eps, r_max=rmax,
                        taylor_terms=K)

    # step 1 from the initial state: parity against the oracle (and the CPU baseline)
    torch.cuda.synchronize()
    ttfv.tt_fv_step(s, st.dt, 1)
    torch.cuda.synchronize()
    parity = None
    cpu = None
    if not args.no_cpu:
        from oracle import tt as ott, tt_fv as otf
        try:
            from threadpoolctl import threadpool_info
            cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
        except Exception:
            cores = os.cpu_count()
        ts = otf.TTSolver(n, "upwind5", True, True, g=st.g, eps=eps, rmax=rmax, taylor_terms=K)
        Q0 = [ott.TT(f.A, f.B) for f in st.tt]
        t0 = time.perf_counter()
        Qo = ts.step(Q0, st.dt)
        t_cpu = time.perf_counter() - t0
        Qg = ttfv.tt_fv_get_state(s)
        rel = [float(np.linalg.norm(g.full() - o.full()) / np.linalg.norm(o.full()))
               for g, o in zip(Qg, Qo)]
        h0 = st.tt[0].A @ st.tt[0].B.T
        dh_g, dh_o = Qg[0].full() - h0, Qo[0].full() - h0
        rel_dh = float(np.linalg.norm(dh_g - dh_o) / np.linalg.norm(dh_o))
        parity = {"rel_l2": rel, "rel_l2_dh": rel_dh, "gate": PARITY_GATE,
                  "pass": bool(max(rel) <= PARITY_GATE), "ranks_gpu": [q.rank for q in Qg],
                  "ranks_oracle": [q.rank for q in Qo], "mode": "restart parity, step 1"}
        cpu = {"value": n * n / t_cpu, "unit": "cell-updates/s", "cores": int(cores),
               "kind": "oracle",
               "sample": f"one full SSP-RK3 step of the {n}^2 workload from its initial state "
                         f"({t_cpu:.1f} s, numpy/LAPACK)"}

    for _ in range(max(args.warmup - 1, 0)):
        ttfv.tt_fv_step(s, st.dt, 1)
    if args.timed_kernel:
        ttfv.tt_fv_time_kernel(s, args.timed_kernel)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ttfv.tt_fv_step(s, st.dt, args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stats = ttfv.tt_fv_get_stats(s)
    if args.timed_kernel:
        ttfv.tt_fv_time_kernel(s, None)
    value = n * n * args.steps / elapsed

    roof = None
    if stats["timed_launches"] > 0 and stats["timed_ms"] > 0:
        avg_ms = stats["timed_ms"] / stats["timed_launches"]
        fl = stats["timed_flops"] / stats["timed_launches"]
        achieved = fl / (avg_ms * 1e-3) / 1e12
        roof = {"kernel": args.timed_kernel, "bound": "alu", "achieved": achieved,
                "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_VECTOR_TFLOPS, "traffic": None,
                "avg_launch_us": avg_ms * 1e3, "launches": stats["timed_launches"],
                "share_of_step": stats["timed_ms"] / (elapsed * 1e3),
                "alg_flops_per_launch": fl}
    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"nonlinear_bumps_{n}", "grid": f"{n}x{n}", "scheme": "upwind5",
                   "bc": "periodic", "r_max": rmax, "eps": eps, "taylor_terms": K, "seed": 0,
                   "cfl": 0.4, "dt": st.dt},
        "roofline": roof, "cpu_baseline": cpu, "parity": parity,
        "ranks": stats["ranks"], "roundings_per_step": None,
    }
    print(json.dumps(out), flush=True)
    s.close()


if __name__ == "__main__":
    main()
