#!/usr/bin/env python3
"""Benchmark of the implicit DUGKS hot path on one MI355X.

One step is one implicit IDUGKS iteration (records, interface flux, predicted macroscopic
LU-SGS, micro LU-SGS sweeps, update, residual).  The headline workload is the largest
single-GPU configuration: the 128x128 lid-driven cavity at Kn = 10 with 101x101
Newton-Cotes velocities (Shakhov, 1.67e8 cell-velocity pairs) in the FP32-bulk /
FP64-moment form, resident in HBM before timing starts.  The 64x64 tanh cavity with 28x28
Gauss-Hermite velocities (FP64; small enough to stay in the Infinity Cache and latency
bound) is measured beside it.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell·velocity updates/s per LU-SGS iter; time-to-residual 1e-8; % HBM peak"
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per cell-velocity pair and launch (s = bytes per stored value,
# both species G and H; a cell has about two faces of its own, nf ~ 2 nc): the face
# partials read phi~ and write the reconstructed value at every face (one writer per face
# and velocity, 4s); the face records read those (4s); the flux reads each face value
# (once: the second cell of a face finds it in L2) and writes M; the forward sweep reads
# M and phi~ and writes the increment; the backward sweep reads the increment and phi~,
# writes phi~
ALGO_BYTES = {"face_partials": 6, "face_records": 4, "flux": 6, "sweep_lower": 6,
              "sweep_upper": 6, "raw_moments": 2, "explicit_update": 6}
# per cell: M_W (4), W (4), sound speed, 1/D, side codes, face nx, ny, S (12) in; dW (4) out
MACRO_DOUBLES_PER_CELL = 27


def measured_traffic(tag, kernel):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs
    summarised in profiles/traffic.json, or None if those counters were taken on other
    kernel sources or another workload."""
    import hashlib
    try:
        tj = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
        h = hashlib.sha256()
        for f in ("idugks_kernels.hip", "idugks_internal.hpp"):
            with open(os.path.join(ROOT, "paper_1709_01819_amd", "csrc", f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != tj["source_sha256"]:
            return None
        for e in tj["workloads"].get(tag, {}).values():
            if e["bench_kernel"] == kernel:
                return e["hbm_bytes"]
    except (OSError, KeyError, ValueError):
        return None
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp32")
    ap.add_argument("--workload", default="cavity_kn10")
    ap.add_argument("--secondary", default="cavity_kn0.075",
                    help="a second, small workload measured in FP64 beside the headline one; it "
                         "also carries the time-to-residual and explicit-vs-implicit runs "
                         "(empty: none)")
    ap.add_argument("--unstructured", default="cavity_kn10_hybrid",
                    help="a workload on an unstructured mesh measured like the headline one, in "
                         "the same precision (empty: none)")
    ap.add_argument("--sweep-order", type=int, choices=[0, 1, 2], default=None,
                    help="sweep_order of the structured headline workload: 0 the library's "
                         "choice (default), 1 levels, 2 i+j hyperplanes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-one-thread", action="store_true",
                    help="skip the single-thread oracle iteration of the CPU baseline")
    ap.add_argument("--no-ttr", action="store_true", help="skip the time-to-residual runs")
    ap.add_argument("--cpu-sample-iters", type=int, default=0,
                    help="oracle iterations of the CPU baseline (0 = 3 on workloads above "
                         "1e8 cell-velocity pairs, else sized to ~15 s)")
    ap.add_argument("--ttr-suite", default="couette,cavity_kn10,cylinder_ma5", metavar="NAMES",
                    help="time the solve to residual 1e-8 of these comma-separated workloads "
                         "in FP64 and FP32-mixed as well (name@CFL sets the implicit CFL, "
                         "name@CFL@START@GROWTH its start-up ramp; an empty string skips them)")
    ap.add_argument("--ttr-budget", type=float, default=20.0,
                    help="wall-clock seconds per solve of --ttr-suite")
    ap.add_argument("--no-explicit", action="store_true",
                    help="skip the explicit-vs-implicit wall-clock comparison")
    ap.add_argument("--explicit-cap", type=int, default=200000,
                    help="explicit step limit of that comparison")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times (the "
                         "reference kernel that scales the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def copy_calibration(mib):
    """Five copies of a MIB-MiB buffer: each reads and writes exactly MIB MiB."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ms = []
    for _ in range(5):
        ev[0].record()
        dst.copy_(src)
        ev[1].record()
        torch.cuda.synchronize()
        ms.append(ev[0].elapsed_time(ev[1]))
    assert torch.equal(dst, src)
    best = min(ms)
    print(json.dumps({"copy_MiB": mib, "bytes_read_per_copy": mib << 20,
                      "bytes_written_per_copy": mib << 20, "ms": ms,
                      "GB/s (read+write)": 2 * (mib << 20) / (best * 1e-3) / 1e9}))


# Table 2 of the paper: explicit steps, implicit iterations and wall-clock speedup to a
# residual of 5e-8 for the cavity cases run here at the same Knudsen numbers
TABLE2 = {"cavity_kn0.075": (11900, 230, 27.49), "cavity_kn1": (9600, 190, 26.80),
          "cavity_kn10": (34200, 640, 28.52)}
EXPLICIT_TOL = 5e-8


def explicit_vs_implicit(workload, cfg, cap):
    """Wall-clock time to steady state of explicit DUGKS (Eq. 21) and of the implicit
    iteration, same GPU, same configuration.

    Criterion 1 is the one of the paper's cost comparison: each run stops when the relative
    L2 change of the cell densities in one step falls below 5e-8 (explicit runs are
    checked every 10 steps, one stream wait each).  At that point the explicit state is
    still far from steady (its time step is the physical one), so criterion 2 continues
    the explicit run until its macroscopic residual (largest RMS of M_W / cell area over
    the conserved variables, Eq. 27) is no larger than the implicit solution's; it is
    checked every 2000 steps, and the clock stops during the checks."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_1709_01819_amd import Solver

    s = Solver(cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it, res, ok = s.solve(EXPLICIT_TOL, 20000)
    torch.cuda.synchronize()
    t_imp = time.perf_counter() - t0
    target = float(np.max(s.residual()))
    del s
    e = Solver(cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n, r = 0, 1.0
    while n < cap:
        r = e.step(wl.EXPLICIT, 10)
        n += 10
        if r < EXPLICIT_TOL:
            break
    torch.cuda.synchronize()
    t_exp = time.perf_counter() - t0
    steady = float(np.max(e.residual()))
    out = {"criterion": "relative L2 change of the cell densities in one step < 5e-8",
           "implicit": {"iterations": it, "seconds": t_imp, "converged": ok,
                        "steady_residual": target},
           "explicit": {"steps": n, "seconds": t_exp, "converged": r < EXPLICIT_TOL,
                        "ms_per_step": 1e3 * t_exp / max(n, 1), "steady_residual": steady},
           "speedup": t_exp / t_imp}
    if workload in TABLE2:
        ex, im, sp = TABLE2[workload]
        out["paper_table2"] = {"explicit_steps": ex, "implicit_steps": im, "speedup": sp}
    n2, t2 = n, t_exp
    while steady > target and n2 < cap:
        t0 = time.perf_counter()
        e.step(wl.EXPLICIT, 2000)
        torch.cuda.synchronize()
        t2 += time.perf_counter() - t0
        n2 += 2000
        steady = float(np.max(e.residual()))
    out["equal_steady_residual"] = {"target": target, "explicit_steps": n2,
                                    "explicit_seconds": t2, "reached": steady <= target,
                                    "speedup": t2 / t_imp}
    return out


FLOOR32 = 5e-8   # FP32 iterations hand over to FP64 below this relative density change


def ttr_suite(names, budget_s):
    """Time to residual 1e-8 of each named workload from its initial state: FP64, FP32-mixed,
    and FP32-mixed down to FLOOR32 (above the FP32 rounding floor) followed by FP64
    iterations from that state (mixed-precision refinement; the handover copies the state
    through the canonical FP64 layout).  Each solve runs in chunks of 50 iterations until converged or out of budget
    (then reported unconverged with the iterations done)."""
    import torch
    import workloads as wl
    from paper_1709_01819_amd import Solver

    def run(s, t0, budget, tol=1e-8):
        """Solve to tol in chunks of 50 iterations.  Returns (res, converged, error)."""
        res, ok, err = float("inf"), False, None
        try:
            while not ok and time.perf_counter() - t0 < budget:
                _, res, ok = s.solve(tol, 50)
        except RuntimeError as e:  # a diverged solve is reported, not raised
            err = str(e)
        return res, ok, err

    out = {}
    for spec in [n for n in names.split(",") if n]:
        # name@CFL overrides the workload's implicit CFL, name@CFL@START@GROWTH also sets the
        # start-up ramp of the CFL
        name, *ov = spec.split("@")

        def cfg_of(prec):
            cfg = dict(wl.case(name), precision=prec)
            if ov:
                cfg["cfl_imp"] = float(ov[0])
            if len(ov) == 3:
                cfg["cfl_start"], cfg["cfl_growth"] = float(ov[1]), float(ov[2])
            return cfg

        for pname in ("fp64", "fp32_mixed", "fp32_then_fp64"):
            cfg = cfg_of(wl.FP64 if pname == "fp64" else wl.FP32_MIXED)
            s = Solver(cfg)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            entry = {}
            if pname == "fp32_then_fp64":
                # FP32 iterations down to FLOOR32, FP64 ones from there
                res, ok32, err = run(s, t0, budget_s, tol=FLOOR32)
                it32 = int(s.info().iterations)
                entry["fp32_iterations"] = it32
                entry["fp32_res"] = res
                it, ok = it32, res < 1e-8
                if err is None and ok32 and not ok:
                    f = s.get_state()
                    del s
                    s = Solver(cfg_of(wl.FP64))
                    s.set_state(f)
                    res, ok, err = run(s, t0, budget_s)
                    entry["fp64_iterations"] = int(s.info().iterations)
                    it = it32 + entry["fp64_iterations"]
            else:
                res, ok, err = run(s, t0, budget_s)
                it = int(s.info().iterations)  # all of them, a diverged one included
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            out[f"{spec}:{pname}"] = dict(
                {"seconds": sec, "iterations": it, "res": res, "converged": ok,
                 "ms_per_iteration": 1e3 * sec / max(it, 1), "cells": s.nc, "velocities": s.nv,
                 "cfl_imp": cfg["cfl_imp"], "cfl_start": cfg.get("cfl_start", 0.0),
                 "cfl_growth": cfg.get("cfl_growth", 1.0)}, **entry)
            if err:
                out[f"{spec}:{pname}"]["error"] = err
            print(f"ttr {spec} {pname}: {it} iterations, {sec:.2f} s, res {res:.3e}, converged {ok}",
                  file=sys.stderr, flush=True)
            del s
            torch.cuda.empty_cache()
    return out


def cpu_baseline(cfg, nc, nv, budget_s=15.0, iters=0, one_thread=True):
    """The FP64 oracle on the host cores, a bounded sample of the same workload: the median
    of a few implicit iterations (after one untimed) from the uniform initial state, and
    one iteration on a single thread."""
    import statistics
    from oracle import Oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    o = Oracle(cfg)
    t0 = time.perf_counter()
    o.implicit_step(1)
    t1 = time.perf_counter() - t0
    big = nc * nv > 1e8
    n = iters if iters > 0 else (3 if big else max(3, min(200, int(budget_s / max(t1, 1e-3)))))
    if big:  # per iteration, median
        per = []
        for _ in range(n):
            t0 = time.perf_counter()
            o.implicit_step(1)
            per.append(time.perf_counter() - t0)
        dt = statistics.median(per)
        how = f"median of {n} implicit iterations"
    else:
        t0 = time.perf_counter()
        o.implicit_step(n)
        dt = (time.perf_counter() - t0) / n
        how = f"mean of {n} implicit iterations"
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    out = {"value": nc * nv / dt, "unit": "cell·vel/s", "cores": threads, "kind": "oracle",
           "sample": f"{how} (after 1 untimed) of the same {mesh_text(cfg)} x "
                     f"{nv}-velocity problem from its uniform initial state, FP64, OpenMP over "
                     f"independent cells/velocities",
           "s_per_iter": dt, "cpu_model": model}
    # the same oracle on one thread (one more iteration), through the OpenMP runtime the
    # oracle library runs on
    if one_thread:
        try:
            import ctypes
            gomp = ctypes.CDLL("libgomp.so.1")
            gomp.omp_set_num_threads(1)
            k = 1 if big else 3
            t0 = time.perf_counter()
            o.implicit_step(k)
            d1 = (time.perf_counter() - t0) / k
            gomp.omp_set_num_threads(threads)
            out["value_1_thread"] = nc * nv / d1
            out["s_per_iter_1_thread"] = d1
        except OSError:
            pass
    return out


def measure(cfg, workload, precision, steps, warmup):
    """Throughput of whole implicit iterations of one workload, resident in HBM.

    A first pass of `steps` iterations brackets every kernel with a HIP event pair (per-kernel
    means; each pair costs a few microseconds of launch gap, so this pass is not the timed
    one).  The timed region is exactly `steps` iterations with one event pair around the
    dominant kernel only, bracketed by stream synchronisations."""
    import torch
    import workloads as wl
    from paper_1709_01819_amd import Solver

    prec = cfg["precision"]
    g = Solver(cfg)
    nc, nv = g.nc, g.nv
    torch.cuda.synchronize()
    g.step(wl.IMPLICIT, warmup)
    torch.cuda.synchronize()
    prof = g.profile(wl.IMPLICIT, steps)
    torch.cuda.synchronize()
    kernels = {k: {"ms_avg": ms / n, "launches": n} for k, (ms, n) in prof.items() if n}
    dom = max(kernels, key=lambda k: kernels[k]["ms_avg"] * kernels[k]["launches"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    live = g.profile(wl.IMPLICIT, steps, kernels=[dom])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dom_ms, dom_n = live[dom]
    kernels[dom]["ms_avg_timed_region"] = dom_ms / dom_n
    s_bytes = 8 if prec == wl.FP64 else 4
    per_launch_bytes = ALGO_BYTES.get(dom, 0) * s_bytes * nc * nv
    if dom == "macro_lusgs":
        per_launch_bytes = nc * 8 * MACRO_DOUBLES_PER_CELL
    achieved = per_launch_bytes / (kernels[dom]["ms_avg_timed_region"] * 1e-3) / 1e9
    tag = f"{workload}:{precision}"
    roofline = {"bound": "hbm", "kernel": dom, "kernel_ms": kernels[dom]["ms_avg_timed_region"],
                "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(tag, dom),
                "algorithmic_bytes_per_launch": per_launch_bytes}
    if dom == "macro_lusgs" and cfg.get("mesh") is None and cfg.get("sweep_order", 0) != 1:
        steps_dep = 2 * (cfg["ni"] + cfg["nj"] - 1)
        roofline["note"] = ("one workgroup sweeps 2 x (ni+nj-1) dependent hyperplane steps: "
                            "bound by the step latency, not by bandwidth")
        roofline["dependent_steps_per_launch"] = steps_dep
        roofline["us_per_step"] = 1e3 * roofline["kernel_ms"] / steps_dep
    streaming = {}
    for k, per in ALGO_BYTES.items():
        if k in kernels:
            b = per * s_bytes * nc * nv
            gbs = b / (kernels[k]["ms_avg"] * 1e-3) / 1e9
            streaming[k] = {"ms": kernels[k]["ms_avg"], "GB/s": gbs, "frac": gbs / HBM_PEAK_GBS,
                            "algorithmic_bytes": b, "traffic": measured_traffic(tag, k)}
    del g
    torch.cuda.empty_cache()
    return {"value": nc * nv / (elapsed / steps), "ms_per_step": 1e3 * elapsed / steps,
            "cells": nc, "velocities": nv, "roofline": roofline, "streaming_kernels": streaming,
            "kernels_ms": {k: round(v["ms_avg"], 5) for k, v in kernels.items()}}


def mesh_text(cfg):
    m = cfg.get("mesh")
    if m is None:
        return f"{cfg['ni']}x{cfg['nj']} cells"
    ntri = int((m["cell_nodes"][:, 3] < 0).sum())
    return f"{len(m['cell_nodes'])} cells ({ntri} triangles, level-scheduled sweeps)"


def describe(workload, cfg, precision):
    return (f"{workload}: {mesh_text(cfg)}, {cfg['nvx']}x{cfg['nvy']} velocities, "
            f"{'Shakhov' if cfg['model'] == 1 else 'BGK'}, Kn={cfg['Kn']}, CFL={cfg['cfl_imp']}, "
            f"{'FP64' if precision == 'fp64' else 'FP32-mixed'}")


def case_cfg(name, prec):
    import workloads as wl
    return wl.case(name, precision=prec) if name != "couette" else dict(wl.case("couette"), precision=prec)


def main():
    args = parse()
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on exactly one GPU (--gpus 1); the "
                                   "velocity-sharded multi-GPU design is documented, not built"}))
        sys.exit(2)
    import torch
    import workloads as wl
    from paper_1709_01819_amd import Solver

    prec = wl.FP64 if args.precision == "fp64" else wl.FP32_MIXED
    cfg = case_cfg(args.workload, prec)
    if args.sweep_order is not None and cfg.get("mesh") is None:
        cfg["sweep_order"] = args.sweep_order
    head = measure(cfg, args.workload, args.precision, args.steps, args.warmup)
    print(f"headline {args.workload} {args.precision}: {head['ms_per_step']:.3f} ms per iteration",
          file=sys.stderr, flush=True)
    out = {"metric": METRIC, "value": head["value"], "unit": "cell·vel/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if prec == wl.FP64 else "f32+f64",
           "data": "synthetic",
           "config": {"workload": describe(args.workload, cfg, args.precision),
                      "cells": head["cells"], "velocities": head["velocities"],
                      "precision": args.precision},
           "roofline": head["roofline"], "streaming_kernels": head["streaming_kernels"],
           # means of a separate K-iteration pass with events around every kernel
           "kernels_ms": head["kernels_ms"]}
    # the same physics on a hybrid quadrilateral/triangle mesh (level-scheduled sweeps)
    if args.unstructured and args.unstructured != args.workload:
        uc = case_cfg(args.unstructured, prec)
        um = measure(uc, args.unstructured, args.precision, args.steps, args.warmup)
        print(f"unstructured {args.unstructured} {args.precision}: {um['ms_per_step']:.3f} ms per "
              f"iteration", file=sys.stderr, flush=True)
        out["unstructured"] = {"workload": describe(args.unstructured, uc, args.precision),
                               "value": um["value"], "unit": "cell·vel/s",
                               "ms_per_step": um["ms_per_step"], "cells": um["cells"],
                               "velocities": um["velocities"], "roofline": um["roofline"],
                               "streaming_kernels": um["streaming_kernels"],
                               "kernels_ms": um["kernels_ms"]}
    # the small benchmark-style cavity (cache resident and latency bound) beside it
    if args.secondary and args.secondary != args.workload:
        sec_prec = wl.FP64
        sc = case_cfg(args.secondary, sec_prec)
        sm = measure(sc, args.secondary, "fp64", args.steps, args.warmup)
        out["secondary"] = {"workload": describe(args.secondary, sc, "fp64"), "value": sm["value"],
                            "ms_per_step": sm["ms_per_step"], "roofline": sm["roofline"],
                            "kernels_ms": sm["kernels_ms"]}
    small = args.secondary
    if small and not args.no_ttr:
        ttr = {}
        for name, pr in (("fp64", wl.FP64), ("fp32_mixed", wl.FP32_MIXED)):
            s2 = Solver(case_cfg(small, pr))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            it, res, ok = s2.solve(1e-8, 5000)
            torch.cuda.synchronize()
            ttr[name] = {"seconds": time.perf_counter() - t0, "iterations": it, "res": res,
                         "converged": ok}
            del s2
        out["time_to_residual_1e-8"] = {"workload": small, **ttr}
        # the paper's second predictor (point relaxation, FP64): fewer outer iterations with
        # more Jacobi sweeps, and no serial hyperplane chain in the macroscopic step
        pr = {}
        for k in (16, 32, 64):
            cp = dict(case_cfg(small, wl.FP64), predictor=1, relax_sweeps=k)
            gk = Solver(cp)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            it, res, ok = gk.solve(1e-8, 20000)
            torch.cuda.synchronize()
            pr[f"sweeps_{k}"] = {"seconds": time.perf_counter() - t0, "iterations": it,
                                 "res": res, "converged": ok}
            del gk
        out["time_to_residual_1e-8_point_relaxation"] = {"workload": small, **pr}
    if args.ttr_suite and not args.no_ttr:
        out["time_to_residual_1e-8_suite"] = ttr_suite(args.ttr_suite, args.ttr_budget)
    if small and not args.no_explicit:
        ecfg = case_cfg(small, wl.FP64)
        if ecfg["ni"] * ecfg["nj"] * ecfg["nvx"] * ecfg["nvy"] <= 2e7:
            out["explicit_vs_implicit"] = explicit_vs_implicit(small, ecfg, args.explicit_cap)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case_cfg(args.workload, wl.FP64), head["cells"],
                                           head["velocities"], iters=args.cpu_sample_iters,
                                           one_thread=not args.no_cpu_one_thread)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
