"""Benchmark: density-matrix leapfrog steps/s at N_orb = 4096 on one MI355X.

One step is the whole clamped-nuclei hot path on one density matrix:
Mulliken charges, SCC potential with the laser field, Hamiltonian
rebuild, the two products of S^-1 H rho, the leapfrog update and the
dipole. Workload: seeded synthetic C938H344 armchair strip (N_orb = 4096)
from its SCC ground state (computed on the GPU, not timed), driven by a
sin^2 laser (0.1 Ha, 0.005 au, in-plane transverse), dt = 0.2 au.

Both precisions run the workload's whole laser run (10000 steps) from the
same ground state: FP64, and split-bf16 with S slices (error-free
splitting, fp32 accumulation, fp64 combination). The timed window is
--steps steps after --warmup steps of that run; the rest runs untimed so
that the split run's dipole can be compared with the FP64 run's over the
whole run. The split run is admissible only if that error stays within
1e-6; `value` is the faster admissible one. A split run that was not
checked over the whole run (--precision split, or --full-run shorter than
the workload) reports admissible null and is never `value`.

Prints one JSON line. `roofline` is for the dominant kernel of the
reported precision, the product (S^-1 H)[Re rho | Im rho] (FP64: 4 n^3
flop per launch) or its split form (issued bf16 flop per launch), timed
with HIP events on the library's stream over the timed steps.
`cpu_baseline` times the CPU oracle on a bounded sample of the workload.
`probe_batch` (beside the main line, not part of it) times a batch of 512
probe trajectories with N_orb ~ U[60, 800] against solo contexts.
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
DIPOLE_TOL = 1e-6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_strip4096.json")
COPY_PROBE_BYTES = 1 << 30
# dominant kernel of each precision: (kernel name stem, source file)
DOMINANT = {"fp64": ("dgemm_nn<2>", "paper_1912_03174_amd/csrc/gemm_f64.hip"),
            "split": ("sgemm_split<", "paper_1912_03174_amd/csrc/gemm_split_bf16.hip")}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", choices=["both", "fp64", "split"], default="both")
    ap.add_argument("--slices", type=int, default=4, choices=[3, 4, 5])
    ap.add_argument("--slices-dh", type=int, default=0, choices=[0, 3, 4, 5],
                    help="slices of the S^-1 dH product (0: --slices)")
    ap.add_argument("--full-run", type=int, default=-1,
                    help="steps of the laser run each precision completes (untimed beyond the "
                         "timed window) for the admissibility check; -1 = the workload's whole "
                         "run (10000), 0 = only the timed window (admissibility unknown)")
    ap.add_argument("--cpu-steps", type=int, default=20,
                    help="oracle steps in the CPU-baseline sample (0 to skip)")
    ap.add_argument("--traffic", type=str, default=TRAFFIC_FILE,
                    help="JSON file with the measured HBM bytes per launch of the dominant "
                         "kernels (reported only while the kernel source is unchanged)")
    ap.add_argument("--traffic-from", type=str, default="",
                    help="host only: read rocprofv3 --pmc csv output (pmc_FETCH_SIZE, "
                         "pmc_WRITE_SIZE, pmccopy_FETCH_SIZE, pmccopy_WRITE_SIZE under this "
                         "folder) and write the --traffic file")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device-to-device once (a plain copy kernel of "
                         "known size, to calibrate HBM byte counters)")
    ap.add_argument("--batched", type=int, default=0,
                    help="instead of the N_orb=4096 step: time a batch of this many probe "
                         "trajectories (N_orb ~ U[60, 800]) against solo runs of a sample")
    ap.add_argument("--batch-summary", type=int, default=512,
                    help="also time a probe batch of this many trajectories (0 to skip) and "
                         "report it beside the main line")
    ap.add_argument("--batch-flags", type=int, default=0,
                    help="td_batch_create flags for --batched (1 no graph, 2 / 4 force tiles)")
    ap.add_argument("--spectrum", type=str, default="",
                    help="instead of timing: kick the 2944-orbital ribbon, propagate 20000 steps "
                         "in FP64, compute its absorption spectrum on the GPU and write it to "
                         "this CSV path")
    ap.add_argument("--ehrenfest", action="store_true",
                    help="instead of the clamped-nuclei step: time moving-nuclei steps of the "
                         "499-atom strip (N_orb=1648) under the sin^2 pump (--steps, --warmup)")
    ap.add_argument("--ehrenfest-batch", type=int, default=0,
                    help="instead of the clamped-nuclei step: a batch of this many moving-nuclei "
                         "trajectories of the 499-atom strip (N_orb=1648, nuclei at 300 K, each "
                         "member its own velocity seed) under the sin^2 pump, against solo runs "
                         "of two of them (--steps, --warmup)")
    ap.add_argument("--plus-u", action="store_true",
                    help="instead of the main line: FP64 steps/s of the N_orb=4096 strip with the "
                         "DFTB+U (FLL) correction on the carbon p shells, against the same steps "
                         "without it (--steps, --warmup)")
    ap.add_argument("--probe-precisions", action="store_true",
                    help="one probe member per size (N_orb 150 .. 800): ms per step as a solo "
                         "context in FP64 and in split-bf16 (--slices), the measurement behind "
                         "running probe batches in FP64")
    ap.add_argument("--small", action="store_true",
                    help="the 112-orbital flake workload (500 steps, kick): solo context "
                         "against a one-member batch replayed from HIP graphs")
    ap.add_argument("--validate", type=int, default=0,
                    help="instead of timing: propagate this many steps in FP64 and in "
                         "split-bf16 (--slices) from the same ground state and print the "
                         "dipole relative error against FP64")
    return ap.parse_args()


def validate(args):
    """Dipole error of split-bf16 against FP64 over a long run of the workload."""
    import workloads as W
    from paper_1912_03174_amd import tddftb as T
    w = W.workload(3)
    n = args.validate
    field = w.field(0, n)
    chunk = 500
    series = {}
    for name, prec in (("fp64", T.TD_FP64), ("split", T.TD_SPLIT_BF16)):
        p = T.Propagator(w.system, dt=w.dt, precision=prec, n_slices=args.slices, scc_tol=1e-10,
                         n_slices_dh=args.slices_dh)
        mus = []
        t0 = time.perf_counter()
        for k in range(0, n, chunk):
            m = min(chunk, n - k)
            mus.append(p.step(m, field[k:k + m]))
            if (k // chunk) % 4 == 3:
                log(f"{name}: {k + m} steps, {time.perf_counter() - t0:.1f} s")
        p.close()
        series[name] = np.concatenate(mus)
    ref, got = series["fp64"], series["split"]
    scale = np.abs(ref - ref[0]).max()
    err = np.abs(got - ref).max(axis=1) / scale
    marks = [m for m in (100, 500, 1000, 2000, 5000, 10000, 20000) if m <= n]
    out = {"validate_steps": n, "slices": args.slices, "slices_dh": args.slices_dh or args.slices,
           "workload": "strip4096",
           "dipole_rel_err": float(err.max()),
           "dipole_rel_err_at": {str(m): float(err[:m].max()) for m in marks},
           "admissible": bool(err.max() <= DIPOLE_TOL),
           "signal_max_au": float(scale)}
    print(json.dumps(out), flush=True)


def source_digest(rel):
    import hashlib
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _pmc(folder, counter):
    """[(kernel name, grid size, counter value KiB)] of one rocprofv3 --pmc csv run."""
    import csv
    path = os.path.join(folder, "run_counter_collection.csv")
    with open(path) as f:
        return [(r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"]))
                for r in csv.DictReader(f) if r["Counter_Name"] == counter]


def write_traffic(root, out_path):
    """HBM bytes per launch of the dominant kernels from FETCH_SIZE / WRITE_SIZE runs.

    Each counter is scaled by bytes / counter of a plain device-to-device copy
    of COPY_PROBE_BYTES (read once, written once) measured with the same
    counter. The split path's dominant kernel is the larger-grid launch of
    sgemm_split (the second product)."""
    cal = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        rows = [v for k, g, v in _pmc(os.path.join(root, "pmccopy_" + ctr), ctr)
                if "copyBuffer" in k]
        if len(rows) != 1:
            raise SystemExit(f"expected one copy kernel in pmccopy_{ctr}, found {len(rows)}")
        cal[ctr] = {"kib": rows[0], "factor": COPY_PROBE_BYTES / (rows[0] * 1024.0)}
    out = {"workload": "strip4096", "copy_probe_bytes": COPY_PROBE_BYTES, "calibration": cal}
    for prec, (stem, src) in DOMINANT.items():
        per = {}
        for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
            rows = [(g, v) for k, g, v in _pmc(os.path.join(root, "pmc_" + ctr), ctr) if stem in k]
            if not rows:
                break
            gmax = max(g for g, _ in rows)
            vals = [v for g, v in rows if g == gmax]
            per[ctr] = {"launches": len(vals), "kib_avg": sum(vals) / len(vals),
                        "bytes": sum(vals) / len(vals) * 1024.0 * cal[ctr]["factor"]}
        if len(per) == 2:
            out[prec] = {"kernel": stem, "source": src, "source_sha256": source_digest(src),
                         "counters": per,
                         "bytes_per_launch": per["FETCH_SIZE"]["bytes"] + per["WRITE_SIZE"]["bytes"]}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out), flush=True)


def measured_traffic(path, prec):
    """Bytes per launch from the --traffic file, or None when absent or when the
    kernel source has changed since the counters were taken."""
    if not path or not os.path.exists(path):
        return None
    with open(path) as f:
        ent = json.load(f).get(prec)
    if not ent or ent.get("source_sha256") != source_digest(ent["source"]):
        return None
    return ent["bytes_per_launch"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


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
    out = {"value": n_steps / el, "unit": "steps/s", "cores": int(threads), "kind": "oracle",
           "sample": f"{n_steps} oracle leapfrog steps (charges, potential, H, three "
                     f"complex128 products, update) at N_orb={s.n_orb} on a seeded Hermitian "
                     f"density near the neutral rho = 1, numpy/OpenBLAS; S^-1 formed before "
                     f"timing; {el:.2f} s"}
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            O.propagate(s, r + 1j * i, 1, w.dt, Sinv=Sinv, field=w.field(0, 1),
                        record_energy=False)
            el1 = time.perf_counter() - t0
        out["one_thread"] = {"value": 1.0 / el1, "unit": "steps/s", "cores": 1,
                             "sample": f"1 oracle step, same input; {el1:.2f} s"}
    except ImportError:
        pass
    return out


def run(T, w, precision, slices, warmup, steps, field, total=0, slices_dh=0):
    """Warm-up, the timed window, then (untimed) the rest of a run of
    ``total`` steps; dipoles of every step are returned."""
    s = w.system
    n = s.n_orb
    t0 = time.perf_counter()
    p = T.Propagator(s, dt=w.dt, precision=precision, n_slices=slices, profile=True,
                     scc_tol=1e-10, n_slices_dh=slices_dh)
    init_s = time.perf_counter() - t0
    info = p.info()
    mus = []
    if warmup:
        mus.append(p.step(warmup, field[:warmup]))
    p.reset_kernel_time()
    t0 = time.perf_counter()
    mus.append(p.step(steps, field[warmup:warmup + steps]))   # returns once the stream drained
    elapsed = time.perf_counter() - t0
    times = {k: p.kernel_time(k) for k in range(4)}
    done = warmup + steps
    while done < total:
        m = min(2000, total - done)
        mus.append(p.step(m, field[done:done + m]))
        done += m
        log(f"  {done} of {total} steps")
    charges = p.charges()
    p.close()
    split = precision == T.TD_SPLIT_BF16
    pairs = slices * (slices + 1) // 2
    ms, cnt = times[T.TD_KT_GEMM_ARHO]
    avg = ms / max(cnt, 1)
    if split:
        flop = pairs * 6.0 * n ** 3          # issued bf16: K = 2n real half, K = n imaginary half
        peak = BF16_PEAK_TFLOPS
        name = f"sgemm_split<{slices}>: [S^-1 H | S^-1 dH][rho - rho_ref ; rho_ref]"
    else:
        flop = 4.0 * n ** 3
        peak = FP64_PEAK_TFLOPS
        name = "dgemm_nn<2>: (S^-1 H)[Re rho | Im rho]"
    achieved = flop / (avg * 1e-3) / 1e12
    return {
        "steps_per_s": steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "init_s": init_s,
        "init": {k: info[k] for k in ("scc_iterations", "scc_residual",
                                      "purification_iterations", "inverse_iterations")},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "kernel": name, "flop_per_launch": flop,
                     "avg_launch_ms": avg, "launches": cnt},
        "breakdown_ms": {"product_1": times[T.TD_KT_GEMM_SH][0] / max(times[0][1], 1),
                         "product_2": avg,
                         "update": times[T.TD_KT_UPDATE][0] / max(times[2][1], 1),
                         "other": times[T.TD_KT_OTHER][0] / max(times[3][1], 1)},
        "fp64_equivalent_tflops": 6.0 * n ** 3 * steps / elapsed / 1e12,
        "steps_run": done,
        "dipoles": np.concatenate(mus),
        "charges": charges,
    }


def spectrum(args):
    """Kicked 2944-orbital ribbon: dipole series and absorption spectrum."""
    import workloads as W
    from paper_1912_03174_amd import tddftb as T

    w = W.spectrum_workload()
    s = w.system
    t0 = time.perf_counter()
    p = T.Propagator(s, dt=w.dt, scc_tol=1e-10)
    init_s = time.perf_counter() - t0
    info = p.info()
    e0, axis = w.kick
    p.kick(e0, axis)
    mus = []
    chunk = 2000
    t0 = time.perf_counter()
    for k in range(0, w.n_steps, chunk):
        mus.append(p.step(min(chunk, w.n_steps - k)))
        log(f"{k + chunk} steps")
    el = time.perf_counter() - t0
    p.close()
    mu = np.concatenate(mus) @ np.asarray(axis, dtype=np.float64)
    omega = np.linspace(0.01, 0.6, 2360)
    tau = 10.0 * W.FS                        # 10 fs damping
    _, sigma = T.td_spectrum(mu, e0, w.dt, omega, tau=tau)
    sigma = sigma[0]
    with open(args.spectrum, "w") as f:
        f.write("omega_ha,sigma_au\n")
        for om, sg in zip(omega, sigma):
            f.write(f"{om:.6f},{sg:.9e}\n")
    inner = np.nonzero((sigma[1:-1] > sigma[:-2]) & (sigma[1:-1] > sigma[2:]))[0] + 1
    top = inner[np.argsort(sigma[inner])[::-1][:6]]
    print(json.dumps({
        "workload": w.name, "n_orb": s.n_orb, "steps": w.n_steps, "dt_au": w.dt,
        "steps_per_s": w.n_steps / el, "init_s": init_s,
        "scc_iterations": info["scc_iterations"], "scc_residual": info["scc_residual"],
        "damping_fs": 10.0, "peaks": [{"omega_ha": float(omega[i]), "omega_ev": float(omega[i] * 27.211386),
                                       "sigma_au": float(sigma[i])} for i in sorted(top)],
        "sigma_min": float(sigma.min()), "sigma_max": float(sigma.max()),
    }), flush=True)


def plus_u(args):
    """FP64 steps of strip4096 with the FLL correction (U_p(C) = 0.15 Ha)
    from its own GPU ground state, beside the uncorrected step."""
    import workloads as W
    from paper_1912_03174_amd import tddftb as T

    class PU:
        mode = "fll"

    w = W.workload(3)
    s = w.system
    PU.shell_offset, PU.shell_u = W.atomic_shells(s, {("C", "p"): 0.15})
    field = w.field(0, args.warmup + args.steps)
    out = {}
    for name, pu in (("plus_u", PU), ("plain", None)):
        t0 = time.perf_counter()
        p = T.Propagator(s, dt=w.dt, scc_tol=1e-10, plus_u=pu)
        init_s = time.perf_counter() - t0
        info = p.info()
        if args.warmup:
            p.step(args.warmup, field[:args.warmup])
        t0 = time.perf_counter()           # the warm-up's dipole read synchronised the stream
        mu = p.step(args.steps, field[args.warmup:])
        el = time.perf_counter() - t0
        out[name] = {"steps_per_s": args.steps / el, "ms_per_step": 1e3 * el / args.steps,
                     "init_s": init_s, "scc_iterations": info["scc_iterations"],
                     "energy": p.energy(), "dipole_end": [float(x) for x in mu[-1]]}
        p.close()
    print(json.dumps({
        "metric": "density-matrix steps/s with the DFTB+U correction (FP64)",
        "value": out["plus_u"]["steps_per_s"], "unit": "steps/s", "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": out["plus_u"]["ms_per_step"],
        "config": {"workload": "strip4096", "n_orb": s.n_orb, "plus_u": "FLL, U = 0.15 Ha on the "
                   "938 carbon p shells", "field": "sin^2 laser 0.1 Ha, 0.005 au"},
        "runs": out,
        "overhead_ms_per_step": out["plus_u"]["ms_per_step"] - out["plain"]["ms_per_step"],
    }), flush=True)


def ehrenfest(args):
    """Moving nuclei: steps/s of the pump run on the 499-atom strip, FP64 and
    (unless --precision fp64) split-bf16 products with rho from the same
    start, with the split run's dipole error against FP64 over its steps."""
    import workloads as W
    from paper_1912_03174_amd import tddftb as T

    w = W.ehrenfest_workload()
    s = w.system
    m = W.two_centre_model(s)
    vel = W.thermal_velocities(s, 300.0, seed=5000)
    field = w.field(0, args.warmup + args.steps)
    n = s.n_orb
    runs = {}
    precs = {"both": ("fp64", "split"), "fp64": ("fp64",), "split": ("split",)}[args.precision]
    for name in precs:
        prec = T.TD_FP64 if name == "fp64" else T.TD_SPLIT_BF16
        t0 = time.perf_counter()
        e = T.Ehrenfest(s, m, velocities=vel, dt=w.dt, scc_tol=1e-10, precision=prec,
                        n_slices=args.slices)
        init_s = time.perf_counter() - t0
        mus = []
        if args.warmup:
            mus.append(e.step(args.warmup, field[:args.warmup]))
        upd0 = e.info()["inverse_updates"]
        t0 = time.perf_counter()
        mus.append(e.step(args.steps, field[args.warmup:]))
        el = time.perf_counter() - t0
        info = e.info()
        ee, ek = e.energy_series(args.steps)
        e.close()
        runs[name] = {
            "steps_per_s": args.steps / el, "ms_per_step": 1e3 * el / args.steps,
            "trajectory_fs_per_s": args.steps / el * w.dt / W.FS,
            "product_tflops": 12.0 * n ** 3 * args.steps / el / 1e12,
            "init_s": init_s, "e_kin_start": float(ek[0]), "e_kin_end": float(ek[-1]),
            "e_total_change": float((ee[-1] + ek[-1]) - (ee[0] + ek[0])),
            "inverse_updates_per_step": (info["inverse_updates"] - upd0) / args.steps,
            "inverse_residual_last": info["inverse_residual"],
            "dipoles": np.concatenate(mus)}
    if "fp64" in runs and "split" in runs:
        ref = runs["fp64"]["dipoles"]
        runs["split"]["dipole_rel_err_vs_fp64"] = float(
            np.abs(runs["split"]["dipoles"] - ref).max() / np.abs(ref - ref[0]).max())
    first = runs[precs[0]]
    print(json.dumps({
        "metric": "moving-nuclei steps/s", "value": first["steps_per_s"], "unit": "steps/s",
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": first["ms_per_step"],
        "dtype": "f64" if precs[0] == "fp64" else "bf16",
        "config": {"workload": w.name, "n_orb": n, "n_atoms": s.n_atoms,
                   "field": "sin^2 pump 0.15 Ha, 0.01 au, 10 fs, across the strip",
                   "nuclei": "300 K"},
        "precisions": {k: {kk: vv for kk, vv in v.items() if kk != "dipoles"}
                       for k, v in runs.items()},
    }), flush=True)


def ehrenfest_batch(args):
    """Moving nuclei in a batch: member-steps/s of N trajectories of one system."""
    import workloads as W
    from paper_1912_03174_amd import tddftb as T

    w = W.ehrenfest_workload()
    s = w.system
    m = W.two_centre_model(s)
    nm = args.ehrenfest_batch
    vel = np.array([W.thermal_velocities(s, 300.0, seed=5000 + j) for j in range(nm)])
    field = w.field(0, args.warmup + args.steps)
    split = args.precision == "split"
    prec = T.TD_SPLIT_BF16 if split else T.TD_FP64
    t0 = time.perf_counter()
    b = T.EhrenfestBatch(s, m, nm, velocities=vel, dt=w.dt, scc_tol=1e-10, precision=prec,
                         n_slices=args.slices)
    init_s = time.perf_counter() - t0
    log(f"batch of {nm} created in {init_s:.1f} s")
    if args.warmup:
        b.step(args.warmup, field[:args.warmup])
    t0 = time.perf_counter()
    b.step(args.steps, field[args.warmup:])
    el = time.perf_counter() - t0
    mu_last = b.dipoles(nm - 1, args.steps)
    ee, ek = b.energy_series(0, args.steps)
    b.close()
    # two members alone, same steps
    solo_s = 0.0
    same = True
    for j in (0, nm - 1):
        e = T.Ehrenfest(s, m, velocities=vel[j], dt=w.dt, scc_tol=1e-10, precision=prec,
                        n_slices=args.slices)
        if args.warmup:
            e.step(args.warmup, field[:args.warmup])
        t1 = time.perf_counter()
        mu = e.step(args.steps, field[args.warmup:])
        solo_s += time.perf_counter() - t1
        e.close()
        if j == nm - 1:
            same = bool(np.array_equal(mu, mu_last))
    n = s.n_orb
    rate = nm * args.steps / el
    flop = 12.0 * n ** 3                      # S^-1 H, (S^-1 H) rho, S^-1 D, (S^-1 D) rho
    print(json.dumps({
        "metric": "moving-nuclei member-steps/s, batch of one system", "value": rate,
        "unit": "member-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True,
        "dtype": "bf16" if split else "f64", "data": "synthetic",
        "config": {"workload": f"{w.name} x{nm}", "members": nm, "n_orb": n,
                   "n_atoms": s.n_atoms,
                   "field": "sin^2 pump 0.15 Ha, 0.01 au, 10 fs, across the strip",
                   "nuclei": "300 K, velocity seeds 5000 ..", "parallelism": "single GPU"},
        "product_tflops": flop * rate / 1e12,
        "fp64_peak_frac": flop * rate / 1e12 / FP64_PEAK_TFLOPS,
        "solo_member_steps_per_s": 2 * args.steps / solo_s,
        "speedup_vs_solo": rate / (2 * args.steps / solo_s),
        "last_member_bitwise_equal_to_solo": same,
        "init_s": init_s, "e_total_change_member0": float((ee[-1] + ek[-1]) - (ee[0] + ek[0])),
    }), flush=True)


def batched(args):
    """Probe batch: member-steps/s of one batch against solo contexts.

    The batch steps all members together (grouped launches, graph replay);
    the solo figure is the same number of steps of a sample of the members,
    each in its own context, one after the other, scaled to the whole batch.
    """
    print(json.dumps(batched_measure(args.batched, args.steps, args.warmup, args.batch_flags)),
          flush=True)


def batched_measure(count, steps, warmup, flags=0):
    """The probe-batch measurement of ``batched`` as a dict."""
    import workloads as W
    from paper_1912_03174_amd import tddftb as T

    log(f"generating {count} probe molecules")
    systems, axes = W.probe_batch(count)
    ns = np.array([s.n_orb for s in systems], dtype=np.float64)
    flop_step = float(np.sum(6.0 * ns ** 3))
    t0 = time.perf_counter()
    b = T.Batch(systems, flags=flags)
    init_s = time.perf_counter() - t0
    log(f"batch created in {init_s:.1f} s")
    b.kick(np.full(count, 1e-3), axes)
    if warmup:
        b.step(warmup)
    t0 = time.perf_counter()
    b.step(steps)
    el = time.perf_counter() - t0
    info = b.info()
    b.close()
    rate = count * steps / el
    # solo contexts on an evenly spaced sample, same steps
    sample = list(range(0, count, max(1, count // 32)))
    solo_s = 0.0
    for m in sample:
        p = T.Propagator(systems[m])
        p.kick(1e-3, axes[m])
        if warmup:
            p.step(warmup)
        t0 = time.perf_counter()
        p.step(steps)
        solo_s += time.perf_counter() - t0
        p.close()
    solo_rate = len(sample) * steps / solo_s
    out = {
        "metric": "probe-trajectory steps/s, batch of N_orb ~ U[60, 800] (FP64)",
        "value": rate, "unit": "member-steps/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": 1e3 * el / steps, "higher_is_better": True,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"probe batch x{count}", "members": count,
                   "n_orb_min": int(ns.min()), "n_orb_max": int(ns.max()),
                   "n_orb_mean": float(ns.mean()), "flags": flags},
        "algorithmic_tflops": flop_step * steps / el / 1e12,
        "fp64_peak_frac": flop_step * steps / el / 1e12 / FP64_PEAK_TFLOPS,
        "solo_sample": {"members": len(sample), "member_steps_per_s": solo_rate},
        "speedup_vs_solo": rate / solo_rate,
        "init_s": init_s, "tiles": info["bucket_tile"], "bucket_members": info["bucket_members"],
        "tuning_ms": info["bucket_ms"],
    }
    return out


def probe_precisions(args):
    """Solo step time of single probe members in both precisions.

    A batch member runs the solo arithmetic in grouped launches, so the
    split-bf16 products could only pay in a batch if they beat FP64 on the
    members themselves; here each size is timed alone (kick, warm-up, then
    --steps steps, HIP events of the library's stream per kernel class)."""
    import workloads as W
    from paper_1912_03174_amd import tddftb as T

    steps = args.steps
    rows = []
    for target in (150, 300, 450, 600, 800):
        s = W.probe_molecule(target, seed=4100 + target)
        row = {"n_orb": s.n_orb}
        for name, prec in (("fp64", T.TD_FP64), ("split", T.TD_SPLIT_BF16)):
            p = T.Propagator(s, precision=prec, n_slices=args.slices, profile=True)
            p.kick(1e-3, (1.0, 0.0, 0.0))
            p.step(max(args.warmup, 1))
            p.reset_kernel_time()
            t0 = time.perf_counter()
            p.step(steps)
            el = time.perf_counter() - t0
            kt = {k: p.kernel_time(k) for k in range(4)}
            p.close()
            row[name] = {"ms_per_step": 1e3 * el / steps,
                         "products_ms": (kt[0][0] + kt[1][0]) / steps,
                         "other_ms": (kt[2][0] + kt[3][0]) / steps}
        row["split_over_fp64"] = row["split"]["ms_per_step"] / row["fp64"]["ms_per_step"]
        rows.append(row)
        log(f"n_orb {s.n_orb}: fp64 {row['fp64']['ms_per_step']:.3f} ms, "
            f"split {row['split']['ms_per_step']:.3f} ms per step")
    print(json.dumps({"workload": "probe members, N_orb 150 .. 800", "steps": steps,
                      "slices": args.slices, "members": rows}), flush=True)


def small(args):
    """The 112-orbital flake (FP64, kick 0.001 au along x, dt 0.2 au): one
    solo context against a one-member batch (the same trajectory bit for
    bit) whose steps replay HIP graphs. At this size a step is a handful of
    launches of a few microseconds, so launch overhead decides the rate.
    Both run the same sequence: kick, warm-up steps (the batch captures its
    graphs there), a second kick, then the timed steps."""
    import workloads as W
    from paper_1912_03174_amd import tddftb as T

    w = W.workload(1)
    s = w.system
    e0, axis = w.kick
    n = args.steps if args.steps != 200 else w.n_steps
    warm = max(args.warmup, 1)
    p = T.Propagator(s)
    rho0 = p.rho()[0]
    p.kick(e0, axis)
    p.step(warm)
    p.kick(e0, axis)
    t0 = time.perf_counter()
    mu_solo = p.step(n)
    solo_s = time.perf_counter() - t0
    p.close()
    b = T.Batch([s], rho0s=[rho0])
    b.kick(np.array([e0]), np.array([axis]))
    b.step(warm)
    b.kick(np.array([e0]), np.array([axis]))
    t0 = time.perf_counter()
    b.step(n)
    batch_s = time.perf_counter() - t0
    mu_batch = b.dipoles(0, n)
    b.close()
    print(json.dumps({
        "metric": "density-matrix steps/s, 112-orbital flake (FP64)", "value": n / solo_s,
        "unit": "steps/s", "n_gpus": 1, "steps": n, "warmup": warm,
        "ms_per_step": 1e3 * solo_s / n, "higher_is_better": True, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_orb": s.n_orb, "path": "solo context"},
        "trajectory_fs_per_s": n / solo_s * w.dt / W.FS,
        "graph_replay_steps_per_s": n / batch_s, "graph_speedup": solo_s / batch_s,
        "dipoles_bitwise_equal": bool(np.array_equal(mu_solo, mu_batch)),
    }), flush=True)


def main():
    args = parse()
    if args.traffic_from:
        write_traffic(args.traffic_from, args.traffic)
        return
    if args.copy_probe:
        import torch
        a = torch.empty(COPY_PROBE_BYTES, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": COPY_PROBE_BYTES}), flush=True)
        return
    if args.validate:
        validate(args)
        return
    if args.batched:
        batched(args)
        return
    if args.spectrum:
        spectrum(args)
        return
    if args.ehrenfest:
        ehrenfest(args)
        return
    if args.plus_u:
        plus_u(args)
        return
    if args.ehrenfest_batch:
        ehrenfest_batch(args)
        return
    if args.small:
        small(args)
        return
    if args.probe_precisions:
        probe_precisions(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    import workloads as W
    from paper_1912_03174_amd import tddftb as T

    w = W.workload(3)
    s = w.system
    total = w.n_steps if args.full_run < 0 else args.full_run
    total = max(total, args.warmup + args.steps)
    field = w.field(0, total)
    res = {}
    if args.precision in ("both", "fp64"):
        log("fp64 run")
        res["fp64"] = run(T, w, T.TD_FP64, args.slices, args.warmup, args.steps, field, total)
    if args.precision in ("both", "split"):
        log(f"split-bf16 x{args.slices} run")
        res["split"] = run(T, w, T.TD_SPLIT_BF16, args.slices, args.warmup, args.steps, field,
                           total, args.slices_dh)
    if "split" in res:
        res["split"]["admissible"] = None            # unknown unless checked below
    if "fp64" in res and "split" in res:
        ref = res["fp64"]["dipoles"]
        dev = np.abs(res["split"]["dipoles"] - ref).max(axis=1) / np.abs(ref - ref[0]).max()
        err = float(dev.max())
        lo, hi = args.warmup, args.warmup + args.steps
        win = ref[lo:hi]
        res["split"]["dipole_rel_err_vs_fp64"] = err
        res["split"]["dipole_rel_err_steps"] = total
        res["split"]["dipole_rel_err_at"] = {str(m): float(dev[:m].max())
                                             for m in (100, 1000, 2000, 5000, 10000)
                                             if m <= total}
        res["split"]["dipole_rel_err_timed_window"] = float(
            np.abs(res["split"]["dipoles"][lo:hi] - win).max() / np.abs(ref - ref[0]).max())
        # same form for the charges, over the final state (scaled by the largest
        # charge fluctuation, as no charge series is recorded)
        dq, dq_ref = res["split"]["charges"], res["fp64"]["charges"]
        res["split"]["charge_rel_err_vs_fp64"] = float(np.abs(dq - dq_ref).max()
                                                       / np.abs(dq_ref).max())
        if total >= w.n_steps:                       # the metric's bound holds over the whole run
            res["split"]["admissible"] = err <= DIPOLE_TOL
    best = "fp64" if "fp64" in res else "split"
    if "split" in res and "fp64" in res and res["split"]["admissible"]:
        if res["split"]["steps_per_s"] > res["fp64"]["steps_per_s"]:
            best = "split"
    r = res[best]
    for k, v in res.items():
        t = measured_traffic(args.traffic, k)
        v["roofline"]["traffic"] = t
        v["hbm_GBps"] = None if t is None else t / (v["roofline"]["avg_launch_ms"] * 1e-3) / 1e9
    roof = dict(r["roofline"])
    dtype = "f64" if best == "fp64" else "bf16"
    out = {
        "metric": "density-matrix steps/s at N_orb=4096 (FP64 vs split-BF16 @1e-6 dipole err)",
        "value": r["steps_per_s"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "arithmetic": ("float64 products" if best == "fp64" else
                       f"bf16 slices (x{args.slices}) on the matrix cores, fp32 accumulation, "
                       "float64 combination"),
        "data": "synthetic",
        "config": {"workload": "strip4096", "system": "C938H344 armchair strip (seeded)",
                   "n_orb": s.n_orb, "n_atoms": s.n_atoms, "dt_au": w.dt,
                   "field": "sin^2 laser 0.1 Ha, 0.005 au, in-plane transverse",
                   "precision": best, "parallelism": "single GPU"},
        "roofline": roof,
        "trajectory_fs_per_s": r["steps_per_s"] * w.dt * 0.0241888432658,
        "precisions": {k: {kk: vv for kk, vv in v.items() if kk not in ("dipoles", "charges")}
                       for k, v in res.items()},
    }
    if "split" in res:
        out["split_admissible"] = res["split"]["admissible"]
    if args.batch_summary > 0:
        log(f"probe batch of {args.batch_summary}")
        bm = batched_measure(args.batch_summary, 50, 5)
        out["probe_batch"] = {k: bm[k] for k in ("metric", "value", "unit", "ms_per_step",
                                                 "algorithmic_tflops", "fp64_peak_frac",
                                                 "speedup_vs_solo", "config", "tiles")}
    if args.cpu_steps > 0:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
