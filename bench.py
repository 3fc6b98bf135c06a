"""Benchmark: density-matrix leapfrog steps/s at N_orb = 4096 on one MI355X.

One step is the whole clamped-nuclei hot path on one density matrix:
Mulliken charges, SCC potential with the laser field, Hamiltonian
rebuild, S^-1 H, (S^-1 H)[Re rho | Im rho], leapfrog update and dipole.
Workload: seeded synthetic C938H344 armchair strip (N_orb = 4096) from
its SCC ground state, driven by a sin^2 laser (0.1 Ha, 0.005 au,
in-plane transverse), dt = 0.2 au. The ground state is computed on the
GPU and is not timed.

Prints one JSON line. `roofline` is for the dominant kernel, the
(S^-1 H)[Re rho | Im rho] product (4 n^3 algorithmic flop per launch),
timed with HIP events on the library's stream over the timed steps.
`cpu_baseline` times the CPU oracle on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X dense FP64 matrix peak
BF16_PEAK_TFLOPS = 2500.0    # MI355X dense BF16 matrix peak
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", choices=["fp64"], default="fp64")
    ap.add_argument("--cpu-steps", type=int, default=3,
                    help="oracle steps in the CPU-baseline sample (0 to skip)")
    ap.add_argument("--traffic", type=str, default="",
                    help="optional JSON file with measured HBM bytes per launch")
    return ap.parse_args()


def cpu_baseline(w, n_steps):
    """The CPU oracle, as it stands, on a bounded sample of the workload."""
    import oracle as O
    import workloads as W
    try:
        from threadpoolctl import threadpool_info
        threads = max((x.get("num_threads", 1) for x in threadpool_info()), default=1)
    except Exception:
        threads = os.cpu_count()
    s = w.system
    Sinv = O.inverse_overlap(s.S)
    r, i = W.random_hermitian_pair(s.n_orb, seed=5, scale=1e-3, base=np.eye(s.n_orb))
    t0 = time.perf_counter()
    O.propagate(s, r + 1j * i, n_steps, w.dt, Sinv=Sinv, field=w.field(0, n_steps),
                record_energy=False)
    el = time.perf_counter() - t0
    return {"value": n_steps / el, "unit": "steps/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n_steps} oracle leapfrog steps (charges, potential, H, three "
                      f"complex128 products, update) at N_orb={s.n_orb} on a seeded Hermitian "
                      f"density, numpy/OpenBLAS; S^-1 formed before timing; "
                      f"{el:.2f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    import workloads as W
    from paper_1912_03174_amd import tddftb as T

    w = W.workload(3)
    s = w.system
    n = s.n_orb
    total = args.warmup + args.steps
    field = w.field(0, total)

    t0 = time.perf_counter()
    p = T.Propagator(s, dt=w.dt, precision=T.TD_FP64, profile=True, scc_tol=1e-10)
    init_s = time.perf_counter() - t0
    info = p.info()

    if args.warmup:
        p.step(args.warmup, field[:args.warmup])
    p.reset_kernel_time()
    t0 = time.perf_counter()
    p.step(args.steps, field[args.warmup:])      # returns after the stream has drained
    elapsed = time.perf_counter() - t0
    mu = p.dipole()
    assert np.all(np.isfinite(mu))

    steps_per_s = args.steps / elapsed
    ms_step = 1e3 * elapsed / args.steps
    arho_ms, arho_n = p.kernel_time(T.TD_KT_GEMM_ARHO)
    sh_ms, sh_n = p.kernel_time(T.TD_KT_GEMM_SH)
    up_ms, up_n = p.kernel_time(T.TD_KT_UPDATE)
    ot_ms, ot_n = p.kernel_time(T.TD_KT_OTHER)
    p.close()

    flop_arho = 4.0 * n ** 3
    avg_arho = arho_ms / max(arho_n, 1)
    achieved = flop_arho / (avg_arho * 1e-3) / 1e12
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        traffic = json.load(open(args.traffic)).get("bytes_per_launch")
    step_tflops = 6.0 * n ** 3 * steps_per_s / 1e12

    out = {
        "metric": "density-matrix steps/s at N_orb=4096 (FP64 vs split-BF16 @1e-6 dipole err)",
        "value": steps_per_s,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "strip4096", "system": "C938H344 armchair strip (seeded)",
                   "n_orb": n, "n_atoms": s.n_atoms, "dt_au": w.dt,
                   "field": "sin^2 laser 0.1 Ha, 0.005 au, in-plane transverse",
                   "precision": "fp64", "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": "dgemm_nn<2>: (S^-1 H)[Re rho | Im rho], 4 n^3 flop/launch",
                     "avg_launch_ms": avg_arho, "launches": arho_n},
        "step_breakdown_ms": {"gemm_sinv_h": sh_ms / max(sh_n, 1), "gemm_a_rho": avg_arho,
                              "leapfrog_update": up_ms / max(up_n, 1),
                              "charges_potential_h": ot_ms / max(ot_n, 1)},
        "step_fp64_tflops": step_tflops,
        "step_fp64_frac": step_tflops / FP64_PEAK_TFLOPS,
        "trajectory_fs_per_s": steps_per_s * w.dt * 0.0241888432658,
        "init_s": init_s,
        "init": {k: info[k] for k in ("scc_iterations", "scc_residual",
                                      "purification_iterations", "inverse_iterations")},
    }
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
