"""Benchmark of the GRMHD substep on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 192] [--no-cpu]
                    [--precision both|fp64|mixed] [--accuracy-steps 200]

Workload: the static curved-spacetime blob on [-20,20]^3 at 192^3 cells
(isotropic Schwarzschild metric with softened radius, Gamma = 2, SSP-RK3),
synthetic seeded initial data already resident in HBM.  A step is one full
Runge-Kutta step (three substeps, every kernel of the path).  The metric is
zone-updates per second per Runge-Kutta substep.  Prints one JSON line: the
headline value is the FP64 run; the "mixed" object holds the mixed-precision
run of the same workload, its speedup over FP64 and its relative L1 distance
from the FP64 state after --accuracy-steps steps.

Per-kernel durations come from HIP events the library records around each
launch on its stream during the timed region.  The roofline entry is for the
kernel with the largest total time; its algorithmic bytes per launch are
given by algorithmic_bytes() below, and the measured HBM traffic per launch
(if profiles/traffic.json was taken on the current kernel sources) by two
rocprofv3 counter runs; copy_GBps is what a plain 1 GiB device-to-device
copy achieves on the same GPU (bytes read plus written), the practical
ceiling beside the 8 TB/s peak.  The CPU baseline times the plain oracle on
one full RK step of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "zone-updates/s per RK substep (FP64 vs mixed) at stated L1 error; adjoint/forward cost"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("paper_1102_5202_amd/csrc/grmhd_kernels.hip",
                  "paper_1102_5202_amd/csrc/grmhd_device.h")


def kernel_source_hash() -> str:
    """Hash of the kernel sources' code: comments and blank space are
    dropped first, so that the stored counters stay valid across edits that
    change no code."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def algorithmic_bytes(kernel: str, n, nsub: int, precision: str = "fp64") -> float:
    """Algorithmic HBM bytes of ONE launch of a kernel class on an n[0] x n[1] x n[2]
    grid (3D), each value that has to cross HBM counted once:
      flux_x / flux_y : the primitives once + one 9-value flux record per face;
      update          : the x and y face records (one unique record per cell and
                        axis), the primitives once (the z faces are computed in
                        the kernel) and the new primitives, U^n, the stage state
                        U^s read (all substeps but the first, which reads U^n)
                        and U^(s+1) written -- averaged over the substeps of a
                        step;
      bc              : read and write the 2-cell ghost slabs of the three axes.
    In mixed precision the primitive caches, face records and the intermediate
    stage state are FP32; U^n and the step's result U^(n+1) stay FP64."""
    N = n[0] * n[1] * n[2]
    wu = 8.0 * 9                     # bytes of one 9-variable FP64 record
    w = wu if precision == "fp64" else 4.0 * 9
    if kernel in ("flux_x", "flux_y", "flux_z"):
        d = "xyz".index(kernel[-1])
        nf = N // n[d] * (n[d] + 1)
        return w * N + w * nf
    if kernel == "update":
        fx = (n[0] + 1) / n[0]
        fy = (n[1] + 1) / n[1]
        inner = (nsub - 1) / nsub            # substeps that read / write the stage state
        return N * (w * (fx + fy + 1 + 1) + wu + w * inner + (w * inner + wu / nsub))
    if kernel == "bc":
        g = 2
        return w * 2 * g * (n[1] * n[2] + n[0] * n[2] + n[0] * n[1]) * 2
    return float("nan")


def load_traffic(kernel: str, workload: str, precision: str = "fp64"):
    """HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE
    (scaled by a copy-kernel calibration), if taken on the current sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(workload, {}).get(precision, {}).get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def _read_csv(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _short(name: str) -> str:
    """Kernel class of a demangled kernel name."""
    for key, short in (("k_flux_x", "flux_x"), ("k_flux_march<1", "flux_y"),
                       ("k_flux_march<2", "flux_z"), ("k_update", "update"), ("k_ghosts", "bc"),
                       ("k_cons", "cons"),
                       ("k_prim", "prim"), ("k_rhs", "rhs"), ("copyBuffer", "copy_probe")):
        if key in name:
            return short
    return name[:40]


def pmc_summary(fetch_csv: str, write_csv: str, probe_bytes: float, workload: str, precision: str,
                out_json: str):
    """Per-launch HBM bytes of each kernel class from two rocprofv3 --pmc runs
    (FETCH_SIZE and WRITE_SIZE, KiB per dispatch), each scaled by what the same
    counter reads for the copy probe of known size (probe_bytes read and written)."""
    per = {}
    for path, ctr in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        for r in _read_csv(path):
            if r.get("Counter_Name") != ctr:
                continue
            k = _short(r["Kernel_Name"])
            per.setdefault(k, {}).setdefault(ctr, []).append(float(r["Counter_Value"]))
    probe = per.get("copy_probe")
    if not probe:
        raise SystemExit("no copy-probe dispatch found in the counter files")
    # the probe is the largest copy dispatch (other copies are small host transfers)
    ff = (probe_bytes / 1024.0) / max(probe["FETCH_SIZE"])
    fw = (probe_bytes / 1024.0) / max(probe["WRITE_SIZE"])
    try:
        with open(out_json) as f:
            res = json.load(f)
    except (OSError, ValueError):
        res = {}
    res.setdefault(workload, {})
    for k in list(res[workload]):             # entries of an older layout
        if k not in ("fp64", "mixed"):
            del res[workload][k]
    cal = res.setdefault("calibration", {})
    for k in list(cal):
        if not isinstance(cal[k], dict):
            del cal[k]
    res[workload][precision] = {}
    res.setdefault("calibration", {})[workload + "/" + precision] = {
        "probe_bytes": probe_bytes, "fetch_factor": ff, "write_factor": fw}
    for k, c in per.items():
        if k not in ("bc", "flux_x", "flux_y", "flux_z", "update", "cons", "prim", "rhs"):
            continue
        if "FETCH_SIZE" not in c or "WRITE_SIZE" not in c:
            continue
        fk = sum(c["FETCH_SIZE"]) / len(c["FETCH_SIZE"])
        wk = sum(c["WRITE_SIZE"]) / len(c["WRITE_SIZE"])
        res[workload][precision][k] = {"fetch_KiB": fk, "write_KiB": wk,
                            "bytes_per_launch": 1024.0 * (fk * ff + wk * fw),
                            "dispatches": len(c["FETCH_SIZE"]), "source_hash": kernel_source_hash()}
    with open(out_json, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
    return res


GROUPS = (("D", (0,)), ("tau", (1,)), ("S", (2, 3, 4)), ("B", (5, 6, 7)), ("Phi", (8,)))


def accuracy(grmhd, w, P0, dev, nsteps):
    """Relative L1 distance of the mixed-precision state from the FP64 state
    after nsteps RK steps from the same initial data, per group of conserved
    variables: sum |U_m - U_d| over the group's components divided by the
    largest component L1 norm of the group in U_d.  "physical" is the maximum
    over D, tau, S and the densitised field; Phi (the cleaning scalar, whose
    size is set by the discretisation error of div B) is given apart."""
    import torch
    Us = {}
    for prec in ("fp64", "mixed"):
        s = grmhd.solver_for(w, device=dev, precision=prec)
        U = s.cons(P0)
        for _ in range(nsteps):
            s.step(U, w.dt)
        torch.cuda.synchronize()
        Us[prec] = U
        del s
    a, b = Us["mixed"], Us["fp64"]
    out = {}
    for name, g in GROUPS:
        num = sum(float((a[i] - b[i]).abs().sum()) for i in g)
        den = max(float(b[i].abs().sum()) for i in g)
        out[name] = num / den if den > 0 else num
    out["physical"] = max(out[k] for k in ("D", "tau", "S", "B"))
    return out


def copy_bandwidth(dev, mib: int = 1024, reps: int = 10) -> float:
    """Achieved GB/s (bytes read + bytes written) of a plain device-to-device
    copy of `mib` MiB, the mean of `reps` copies after a warm-up, timed with
    HIP events on the current stream."""
    import torch
    a = torch.ones(mib * 2 ** 20 // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * mib * 2 ** 20 / (ms * 1e-3) / 1e9


def adjoint_cost(grmhd, w, dev, steps: int, every: int = 10):
    """Cost of the adjoint on workload w (FP64), after a warm-up of every
    call, as mean durations over that of one grmhd_step:
    grmhd_step_adjoint, which recomputes its step's stages first (about one
    forward step); grmhd_step_record, a forward step that keeps its stages;
    and grmhd_step_adjoint_recorded, the reverse sweep of a recorded step.
    Also the wall time of a whole gradient (forward evolution with checkpoints
    every `every` steps, then the checkpointed reverse sweep, with the tape of
    recorded steps and without it) over that of the forward evolution alone."""
    import numpy as np
    import torch
    from paper_1102_5202_amd.adjoint import evolve
    s = grmhd.solver_for(w, device=dev, adjoint=True)
    st = grmhd.solver_for(w, device=dev, adjoint=True, tape_steps=every)
    P0 = torch.from_numpy(w.P).to(dev)
    tgt = (torch.from_numpy(np.ascontiguousarray(w.extra["target"])).to(dev) if "target" in w.extra
           else P0[0] * 1.01)

    def gradient(solver):
        Pq = P0.clone().requires_grad_(True)
        Pn = evolve(solver, Pq, w.dt, steps, every)
        ((Pn[0] - tgt) ** 2).sum().backward()
        return Pq.grad

    def forward_evolution():
        U = s.cons(P0)
        for _ in range(steps):
            s.step(U, w.dt)
        s.prim(U)

    def timed(fn, reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    U = s.cons(P0)
    for _ in range(2):
        s.step(U, w.dt)
    Ub = torch.randn_like(U)
    s.step_adjoint(U, Ub, w.dt)
    Ur = st.cons(P0)
    st.step_record(Ur, w.dt, 0)
    st.step_adjoint_recorded(0, Ub)
    g = gradient(s)                     # warm-up of every path
    gt = gradient(st)
    n = max(4, min(steps, 20))
    t_fwd = timed(lambda: s.step(U, w.dt), n)
    t_adj = timed(lambda: s.step_adjoint(U, Ub, w.dt), n)
    t_rec = timed(lambda: st.step_record(Ur, w.dt, 0), n)
    t_rev = timed(lambda: st.step_adjoint_recorded(0, Ub), n)
    t_evo = timed(forward_evolution, 2)
    t_grad = timed(lambda: gradient(s), 2)
    t_gradt = timed(lambda: gradient(st), 2)
    return {"workload": w.name, "steps": steps, "checkpoint_every": every,
            "forward_step_ms": round(1e3 * t_fwd, 4), "adjoint_step_ms": round(1e3 * t_adj, 4),
            "adjoint_over_forward": round(t_adj / t_fwd, 3),
            "record_step_ms": round(1e3 * t_rec, 4), "recorded_adjoint_step_ms": round(1e3 * t_rev, 4),
            "recorded_adjoint_over_forward": round(t_rev / t_fwd, 3),
            "gradient_ms": round(1e3 * t_gradt, 3), "gradient_untaped_ms": round(1e3 * t_grad, 3),
            "forward_evolution_ms": round(1e3 * t_evo, 3),
            "gradient_over_forward": round(t_gradt / t_evo, 3),
            "gradient_untaped_over_forward": round(t_grad / t_evo, 3),
            "finite": bool(torch.isfinite(g).all().item() and torch.isfinite(gt).all().item())}


def batch_throughput(grmhd, e, dev):
    """The batched ensemble e evolved to its end in one persistent launch per
    precision, after the launch-shape tuner: zone-updates per second per
    Runge-Kutta substep (sum over problems of cells x steps x substeps, over
    the wall time of the evolve call)."""
    import torch
    work = sum(n * s for n, s in zip(e.n, e.steps)) * e.rk_order
    out = {"workload": e.name, "problems": len(e.n), "cells": e.ncell, "zone_substeps": work}
    for prec in ("fp64", "mixed"):
        s = grmhd.batch_for(e, device=dev, precision=prec)
        P0 = s.pack(e.P)
        U = s.cons(P0)
        th, lds = s.tune(U, trial_steps=20)
        U = s.cons(P0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.evolve(U)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out[prec] = {"value": work / t, "seconds": round(t, 4), "threads": th, "lds_rows": lds,
                     "recovery": s.status(), "finite": bool(torch.isfinite(U).all().item())}
        del s, U
    out["mixed"]["speedup_vs_fp64"] = round(out["mixed"]["value"] / out["fp64"]["value"], 3)
    return out


def cpu_baseline(w, pb_kwargs):
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    oracle.set_threads(threads)
    pb = oracle.Problem(**pb_kwargs)
    U0 = oracle.prim2con(pb, w.P)
    t0 = time.perf_counter()
    oracle.step(pb, U0, w.P, w.dt, 1)
    dt = time.perf_counter() - t0
    subs = w.rk_order * w.ncell
    return {"value": subs / dt, "unit": "zone-updates/s", "cores": oracle.get_threads(),
            "kind": "oracle",
            "sample": "one full SSP-RK%d step (%d substeps) of the %s workload, %d cells, %.1f s wall"
                      % (w.rk_order, w.rk_order, w.name, w.ncell, dt)}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=192)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-timing", action="store_true", help="do not record per-kernel events")
    ap.add_argument("--no-variants", action="store_true", help="skip the scheme-variant legs")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-cost leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-ensemble leg")
    ap.add_argument("--accuracy-steps", type=int, default=200,
                    help="RK steps of the FP64-vs-mixed accuracy comparison")
    ap.add_argument("--precision", choices=("both", "fp64", "mixed"), default="both",
                    help="which precisions to time (a counter run takes one); with --pmc-summary, "
                         "the precision the counter files were taken on")
    ap.add_argument("--copy-probe", type=float, default=0.0, metavar="MIB",
                    help="first run one plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc counter files "
                         "(taken with --copy-probe) and exit")
    ap.add_argument("--probe-mib", type=float, default=1024.0)
    args = ap.parse_args(argv)

    if args.pmc_summary:
        if args.precision == "both":
            raise SystemExit("--pmc-summary needs --precision fp64 or mixed")
        res = pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.probe_mib * 2 ** 20,
                          "curved_blob_%d^3" % args.n, args.precision,
                          os.path.join(ROOT, "profiles", "traffic.json"))
        print(json.dumps(res, indent=1))
        return 0

    if args.gpus != 1:
        print("bench.py: the library runs on one GPU; --gpus %d is not supported "
              "(the multi-GPU halo exchange is a design note, not an implemented path)" % args.gpus,
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1102_5202_amd import grmhd, workloads

    dev = "cuda:0"
    if args.copy_probe > 0:
        nel = int(args.copy_probe * 2 ** 20) // 8
        a = torch.ones(nel, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    w = workloads.config3(n=args.n, nsteps=args.steps)
    wl_name = "curved_blob_%d^3" % args.n
    nsub = w.rk_order
    P0 = torch.from_numpy(w.P).to(dev)

    def timed_run(precision, stored=None, **over):
        s = grmhd.solver_for(w, device=dev, timing=not args.no_timing, precision=precision, **over)
        if stored is not None:
            s.set_metric(*stored)
        U = s.cons(P0)
        for _ in range(args.warmup):
            s.step(U, w.dt)
        torch.cuda.synchronize()
        s.timing(reset=True)
        s.status(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            s.step(U, w.dt)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        r = {"value": w.ncell * nsub * args.steps / elapsed,
             "ms_per_step": 1e3 * elapsed / args.steps,
             "recovery": s.status(), "finite": bool(torch.isfinite(U).all().item()),
             "kernels": {}, "roofline": None}
        if not args.no_timing:
            kernels = r["kernels"]
            for k, (ms, cnt) in s.timing().items():
                if cnt:
                    avg = ms / cnt
                    bk = algorithmic_bytes(k, w.n, nsub, precision)
                    kernels[k] = {"launches": cnt, "total_ms": round(ms, 4), "avg_ms": round(avg, 5),
                                  "alg_GBps": round(bk / (avg * 1e-3) / 1e9, 1) if bk == bk else None}
            dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
            bk = algorithmic_bytes(dom, w.n, nsub, precision)
            achieved = bk / (kernels[dom]["avg_ms"] * 1e-3) / 1e9
            r["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(achieved / HBM_PEAK_GBS, 4),
                             "traffic": load_traffic(dom, wl_name, precision),
                             "alg_bytes_per_launch": bk}
        del U, s
        return r

    fp64 = timed_run("fp64") if args.precision != "mixed" else None
    mixed = timed_run("mixed") if args.precision != "fp64" else None
    if not args.no_timing:
        # the practical denominator: a plain device-to-device copy of 1 GiB
        bw = copy_bandwidth(dev)
        for r in (fp64, mixed):
            if r and r["roofline"]:
                r["roofline"]["copy_GBps"] = round(bw, 1)
                r["roofline"]["frac_of_copy"] = round(r["roofline"]["achieved"] / bw, 4)
    if fp64 and mixed:
        mixed["speedup_vs_fp64"] = round(mixed["value"] / fp64["value"], 3)
        if args.accuracy_steps > 0:
            acc = accuracy(grmhd, w, P0, dev, args.accuracy_steps)
            mixed["rel_l1_vs_fp64"] = acc["physical"]
            mixed["rel_l1_vs_fp64_groups"] = acc
            mixed["rel_l1_steps"] = args.accuracy_steps
    main = fp64 or mixed

    out = {
        "metric": METRIC,
        "value": main["value"],
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if fp64 else "f32+f64 (mixed)",
        "data": "synthetic (seeded initial data)",
        "config": {"workload": wl_name + " static curved spacetime (isotropic Schwarzschild, "
                   "r_s = sqrt(r^2+1)), [-20,20]^3, Gamma=2, SSP-RK3, "
                   + ("FP64" if fp64 else "mixed precision"),
                   "cells": w.ncell, "substeps_per_step": nsub, "dt": w.dt},
        "roofline": main["roofline"],
        "kernels": main["kernels"],
        "recovery": main["recovery"],
        "finite": main["finite"],
        "mixed": mixed if fp64 else None,
    }
    if not args.no_adjoint and fp64:
        # the adjoint workload (64^3 periodic box, 50 RK2 steps, checkpoints every 10)
        out["adjoint"] = adjoint_cost(grmhd, workloads.config4(n=64, nsteps=50), dev, 50, 10)
    if not args.no_variants and fp64:
        # scheme variants on the same workload: the recovery's one-unknown
        # iteration; PPM reconstruction and flux-CT (three face kernels, for
        # flux-CT the edge and face corrections, then the cell update); the
        # same spacetime given on the grid (stored metric)
        out["variants"] = {}
        alpha, psi4 = workloads.sampled_isotropic_metric(w.n, w.lo, w.hi, w.M, w.r_min)
        stored = (torch.from_numpy(alpha).to(dev), torch.from_numpy(psi4).to(dev))
        for name, over in (("recovery_1d", {"recovery": "1d"}), ("ppm", {"reconstruction": "ppm"}),
                           ("fluxct", {"divergence": "fluxct"}),
                           ("stored_metric", {"metric": grmhd.STORED, "stored": stored})):
            v = timed_run("fp64", **over)
            out["variants"][name] = {
                "value": v["value"], "ms_per_step": v["ms_per_step"], "recovery": v["recovery"],
                "finite": v["finite"], "kernels_avg_ms": {k: x["avg_ms"] for k, x in v["kernels"].items()},
                "vs_default": round(v["value"] / fp64["value"], 3)}
    if not args.no_batch and fp64:
        # 256 magnetised 1D Riemann problems of 200..4000 cells, each to t = 0.4
        out["batch"] = batch_throughput(grmhd, workloads.config5(), dev)
    finite = all(r["finite"] for r in (fp64, mixed) if r)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, w.problem_kwargs())
    print(json.dumps(out), flush=True)
    return 0 if finite else 1


if __name__ == "__main__":
    sys.exit(main())
