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


# Algorithmic HBM bytes per cell and Runge-Kutta substep of a fully fused
# substep: read P^s and U^n, write U^(s+1) and P^(s+1), 36 values; the stage
# state U^s is recomputable from P^s and the metric is evaluated in closed
# form, so neither is counted.  FP64: 36 x 8 = 288 B; mixed precision with the
# primitives in FP32: 2 x 36 + 2 x 72 = 216 B.
SUBSTEP_BYTES = {"fp64": 288.0, "mixed": 216.0}


def design_bytes_per_cell(nsub: int, precision: str = "fp64") -> float:
    """Bytes per cell and substep that this design has to move at the least,
    averaged over the substeps of a step: the primitives read and written
    once (FP64 or FP32), U^n read, the stage state U^s read by every substep
    but the first (which reads U^n as its stage state) and U^(s+1) written
    (the intermediate stage states in FP32 in mixed precision, the step's
    result in FP64)."""
    wp = 72.0 if precision == "fp64" else 36.0
    ws = 72.0 if precision == "fp64" else 36.0
    inner = (nsub - 1) / nsub
    return 2 * wp + 72.0 + ws * inner + (ws * inner + 72.0 / nsub)


def algorithmic_bytes(kernel: str, n, nsub: int, precision: str = "fp64") -> float:
    """Algorithmic HBM bytes of ONE launch of a kernel class on an n[0] x n[1] x n[2]
    grid (3D), each value that has to cross HBM counted once:
      update          : the fused substep kernel (faces of all axes, flux
                        differences, sources, Runge-Kutta combination,
                        recovery): SUBSTEP_BYTES per cell;
      flux_x/y/z      : (1D/2D grids and scheme variants) the primitives once +
                        one 9-value flux record per face;
      bc              : read and write the 2-cell ghost slabs of the three axes."""
    N = n[0] * n[1] * n[2]
    w = 72.0 if precision == "fp64" else 36.0
    if kernel in ("flux_x", "flux_y", "flux_z"):
        d = "xyz".index(kernel[-1])
        nf = N // n[d] * (n[d] + 1)
        return w * N + w * nf
    if kernel == "update":
        return SUBSTEP_BYTES[precision] * N
    if kernel == "bc":
        g = 2
        return w * 2 * g * (n[1] * n[2] + n[0] * n[2] + n[0] * n[1]) * 2
    return float("nan")


def load_counters(kernel: str, workload: str, precision: str = "fp64"):
    """The counter entry of a kernel class (profiles/traffic.json: HBM bytes
    per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by a copy-kernel
    calibration, and VALU wave-instructions per launch), if taken on the
    current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(workload, {}).get(precision, {}).get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e


def _read_csv(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _short(name: str) -> str:
    """Kernel class of a demangled kernel name."""
    for key, short in (("k_substep", "update"), ("k_flux_x", "flux_x"), ("k_flux_march<1", "flux_y"),
                       ("k_flux_march<2", "flux_z"), ("k_update", "update"), ("k_ghosts", "bc"),
                       ("k_cons", "cons"),
                       ("k_prim", "prim"), ("k_rhs", "rhs"), ("copyBuffer", "copy_probe")):
        if key in name:
            return short
    return name[:40]


VALU_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_ADD_F64",
                 "SQ_INSTS_VALU_TRANS_F64")


def pmc_summary(fetch_csv: str, write_csv: str, probe_bytes: float, workload: str, precision: str,
                out_json: str, valu_csv: str = None):
    """Per-launch HBM bytes of each kernel class from two rocprofv3 --pmc runs
    (FETCH_SIZE and WRITE_SIZE, KiB per dispatch), each scaled by what the same
    counter reads for the copy probe of known size (probe_bytes read and
    written); with a third counter file, the VALU wave-instructions per launch
    (all, and the FP64 arithmetic ones)."""
    per = {}
    files = [(fetch_csv, ("FETCH_SIZE",)), (write_csv, ("WRITE_SIZE",))]
    if valu_csv:
        files.append((valu_csv, VALU_COUNTERS))
    for path, ctrs in files:
        for r in _read_csv(path):
            ctr = r.get("Counter_Name")
            if ctr not in ctrs:
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
        if all(v in c for v in VALU_COUNTERS):
            mean = {v: sum(c[v]) / len(c[v]) for v in VALU_COUNTERS}
            res[workload][precision][k]["valu_insts_per_launch"] = mean["SQ_INSTS_VALU"]
            res[workload][precision][k]["fp64_valu_insts_per_launch"] = sum(
                mean[v] for v in VALU_COUNTERS[1:])
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
    size is set by the discretisation error of div B) is given apart; "all"
    is the maximum over every group."""
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
    out["all"] = max(out["physical"], out["Phi"])
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
    recorded steps and without it) over that of the forward evolution alone,
    and with a tape as long as the run (every step recorded by the forward
    pass, nothing recomputed: memory for compute)."""
    import numpy as np
    import torch
    from paper_1102_5202_amd.adjoint import evolve
    s = grmhd.solver_for(w, device=dev, adjoint=True)
    st = grmhd.solver_for(w, device=dev, adjoint=True, tape_steps=every)
    sf = grmhd.solver_for(w, device=dev, adjoint=True, tape_steps=steps)
    P0 = torch.from_numpy(w.P).to(dev)
    tgt = (torch.from_numpy(np.ascontiguousarray(w.extra["target"])).to(dev) if "target" in w.extra
           else P0[0] * 1.01)

    def gradient(solver, seg=every):
        Pq = P0.clone().requires_grad_(True)
        Pn = evolve(solver, Pq, w.dt, steps, seg)
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
    gf = gradient(sf, steps)
    n = max(4, min(steps, 20))
    t_fwd = timed(lambda: s.step(U, w.dt), n)
    t_adj = timed(lambda: s.step_adjoint(U, Ub, w.dt), n)
    t_rec = timed(lambda: st.step_record(Ur, w.dt, 0), n)
    t_rev = timed(lambda: st.step_adjoint_recorded(0, Ub), n)
    t_evo = timed(forward_evolution, 2)
    t_grad = timed(lambda: gradient(s), 2)
    t_gradt = timed(lambda: gradient(st), 2)
    t_gradf = timed(lambda: gradient(sf, steps), 2)
    return {"workload": w.name, "steps": steps, "checkpoint_every": every,
            "forward_step_ms": round(1e3 * t_fwd, 4), "adjoint_step_ms": round(1e3 * t_adj, 4),
            "adjoint_over_forward": round(t_adj / t_fwd, 3),
            "record_step_ms": round(1e3 * t_rec, 4), "recorded_adjoint_step_ms": round(1e3 * t_rev, 4),
            "recorded_adjoint_over_forward": round(t_rev / t_fwd, 3),
            "gradient_ms": round(1e3 * t_gradt, 3), "gradient_untaped_ms": round(1e3 * t_grad, 3),
            "forward_evolution_ms": round(1e3 * t_evo, 3),
            "gradient_over_forward": round(t_gradt / t_evo, 3),
            "gradient_untaped_over_forward": round(t_grad / t_evo, 3),
            "gradient_full_tape_ms": round(1e3 * t_gradf, 3),
            "gradient_full_tape_over_forward": round(t_gradf / t_evo, 3),
            "full_tape_bytes": int(sf.workspace.numel() - s.workspace.numel()),
            "finite": bool(torch.isfinite(g).all().item() and torch.isfinite(gt).all().item()
                           and torch.isfinite(gf).all().item())}


def batch_throughput(grmhd, e, dev):
    """The batched ensemble e evolved to its end in one persistent launch per
    precision, after the launch-shape tuner: zone-updates per second per
    Runge-Kutta substep (sum over problems of cells x steps x substeps, over
    the wall time of the evolve call), and how busy the launch kept its
    workgroup slots (summed workgroup durations over slots x span, from the
    workgroups' own clock readings).  For comparison, FP64 once more with one
    workgroup per problem (the tuner's best shape without the split)."""
    import torch
    work = sum(n * s for n, s in zip(e.n, e.steps)) * e.rk_order
    out = {"workload": e.name, "problems": len(e.n), "cells": e.ncell, "zone_substeps": work}
    places = {0: "one workgroup per problem, rows in HBM", 1: "one workgroup per problem, rows in LDS",
              2: "problems split among workgroups by work"}

    def run(prec, shape=None):
        s = grmhd.batch_for(e, device=dev, precision=prec)
        P0 = s.pack(e.P)
        U = s.cons(P0)
        if shape is None:
            th, lds = s.tune(U, trial_steps=20)
        else:
            th, lds = shape
            s.set_shape(th, lds)
        U = s.cons(P0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.evolve(U)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        busy, slots = s.busy()
        r = {"value": work / t, "seconds": round(t, 4), "threads": th, "placement": places[lds],
             "busy_fraction": round(busy, 4), "wg_slots": slots,
             "recovery": s.status(), "finite": bool(torch.isfinite(U).all().item())}
        del s, U
        return r

    for prec in ("fp64", "mixed"):
        out[prec] = run(prec)
    out["mixed"]["speedup_vs_fp64"] = round(out["mixed"]["value"] / out["fp64"]["value"], 3)
    one = run("fp64", (1024, 0))
    out["fp64_one_workgroup_per_problem"] = {k: one[k] for k in ("value", "seconds", "threads", "placement",
                                                                   "busy_fraction", "wg_slots")}
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, small):
    """The plain CPU oracle (test infrastructure, never on the GPU path) timed
    on the host: one full RK step of the benchmark workload on all the cores
    OpenMP is given, and one full RK step of the same workload recipe at a
    smaller size on one thread (the per-cell rate does not depend on the
    size)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {}
    for wl, nth in ((w, threads), (small, 1)):
        oracle.set_threads(nth)
        pb = oracle.Problem(**wl.problem_kwargs())
        U0 = oracle.prim2con(pb, wl.P)
        t0 = time.perf_counter()
        oracle.step(pb, U0, wl.P, wl.dt, 1)
        dt = time.perf_counter() - t0
        out[nth == 1 and wl is small] = (wl.rk_order * wl.ncell / dt, oracle.get_threads(), dt, wl)
    v, cores, dt, wl = out[False]
    v1, _, dt1, wl1 = out[True]
    return {"value": v, "unit": "zone-updates/s", "cores": cores, "kind": "oracle",
            "sample": "one full SSP-RK%d step (%d substeps) of the %s workload, %d cells, %.1f s wall"
                      % (wl.rk_order, wl.rk_order, wl.name, wl.ncell, dt),
            "cpu_model": cpu_model(),
            "one_thread": {"value": v1, "cores": 1,
                           "sample": "one full SSP-RK%d step of the same workload at %d^3 (%d cells), %.1f s wall"
                                     % (wl1.rk_order, wl1.n[0], wl1.ncell, dt1)}}


def batch_accuracy(grmhd, e, dev, nsteps: int = None):
    """Relative L1 distance of the mixed-precision ensemble from the FP64 one
    after every problem ran to its end (both with the split placement where
    the device allows it), per problem (the largest over all 9 conserved
    variables, vector components normalised as in accuracy()): median, 90th
    percentile and maximum over the problems."""
    import numpy as np
    import torch
    res = {}
    for prec in ("fp64", "mixed"):
        s = grmhd.batch_for(e, device=dev, precision=prec)
        try:
            s.set_shape(256, 2)       # the placement the throughput leg measures
        except RuntimeError:
            pass
        U = s.cons(s.pack(e.P))
        s.evolve(U)
        torch.cuda.synchronize()
        res[prec] = [u.double().cpu().numpy() for u in s.unpack(U)]
        del s, U
    errs = []
    for a, b in zip(res["mixed"], res["fp64"]):
        e_b = 0.0
        for _, g in GROUPS:
            num = sum(np.abs(a[i] - b[i]).sum() for i in g)
            den = max(np.abs(b[i]).sum() for i in g)
            e_b = max(e_b, num / den if den > 0 else num)
        errs.append(e_b)
    errs = np.array(errs)
    return {"median": float(np.median(errs)), "p90": float(np.percentile(errs, 90)), "max": float(errs.max()),
            "problems_above_1e-5": int((errs > 1e-5).sum())}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--repeats", type=int, default=5, help="timed runs of --steps steps; the median is reported")
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
    ap.add_argument("--pmc-summary", nargs="+", metavar="CSV",
                    help="write profiles/traffic.json from rocprofv3 --pmc counter files: FETCH_SIZE, "
                         "WRITE_SIZE (taken with --copy-probe) and optionally the VALU counters; then exit")
    ap.add_argument("--probe-mib", type=float, default=1024.0)
    args = ap.parse_args(argv)

    if args.pmc_summary:
        if args.precision == "both":
            raise SystemExit("--pmc-summary needs --precision fp64 or mixed")
        if len(args.pmc_summary) not in (2, 3):
            raise SystemExit("--pmc-summary takes FETCH_CSV WRITE_CSV [VALU_CSV]")
        res = pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.probe_mib * 2 ** 20,
                          "curved_blob_%d^3" % args.n, args.precision,
                          os.path.join(ROOT, "profiles", "traffic.json"),
                          args.pmc_summary[2] if len(args.pmc_summary) == 3 else None)
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
    N = w.ncell

    def timed_run(precision, stored=None, repeats=None, **over):
        repeats = args.repeats if repeats is None else repeats
        s = grmhd.solver_for(w, device=dev, timing=not args.no_timing, precision=precision, **over)
        if stored is not None:
            s.set_metric(*stored)
        runs = []
        for _ in range(max(1, repeats)):
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
            runs.append((elapsed, s.timing(), s.status(), bool(torch.isfinite(U).all().item())))
            del U
        runs.sort(key=lambda r: r[0])
        elapsed, timing, status, finite = runs[len(runs) // 2]
        r = {"value": N * nsub * args.steps / elapsed,
             "ms_per_step": 1e3 * elapsed / args.steps,
             "ms_per_step_runs": [round(1e3 * x[0] / args.steps, 4) for x in runs],
             "recovery": status, "finite": all(x[3] for x in runs),
             "kernels": {}, "roofline": None}
        if not args.no_timing:
            kernels = r["kernels"]
            for k, (ms, cnt) in timing.items():
                if cnt:
                    avg = ms / cnt
                    bk = algorithmic_bytes(k, w.n, nsub, precision)
                    kernels[k] = {"launches": cnt, "total_ms": round(ms, 4), "avg_ms": round(avg, 5),
                                  "alg_GBps": round(bk / (avg * 1e-3) / 1e9, 1) if bk == bk else None}
            dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
            avg_s = kernels[dom]["avg_ms"] * 1e-3
            bk = algorithmic_bytes(dom, w.n, nsub, precision)
            achieved = bk / avg_s / 1e9
            sub_s = r["ms_per_step"] * 1e-3 / nsub
            cnt = load_counters(dom, wl_name, precision)
            rl = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                  "traffic": cnt["bytes_per_launch"] if cnt else None,
                  "alg_bytes_per_cell": SUBSTEP_BYTES[precision] if dom == "update" else bk / N,
                  "alg_bytes_per_launch": bk,
                  "whole_substep_frac": round(SUBSTEP_BYTES[precision] * N / sub_s / 1e9 / HBM_PEAK_GBS, 4),
                  "design_bytes_per_cell": round(design_bytes_per_cell(nsub, precision), 1),
                  "design_frac": round(design_bytes_per_cell(nsub, precision) * N / avg_s / 1e9 / HBM_PEAK_GBS,
                                       4)}
            if cnt:
                rl["traffic_bytes_per_cell"] = round(cnt["bytes_per_launch"] / N, 1)
                rl["traffic_frac"] = round(cnt["bytes_per_launch"] / avg_s / 1e9 / HBM_PEAK_GBS, 4)
                if "valu_insts_per_launch" in cnt:
                    # issue time of the counted wave-instructions (4 cycles each
                    # on a 16-lane SIMD) on all 1024 SIMDs at 2.4 GHz
                    issue = lambda x: x * 4.0 / (1024 * 2.4e9)
                    rl["valu_insts_per_cell"] = round(cnt["valu_insts_per_launch"] * 64 / N, 1)
                    rl["valu_busy"] = round(issue(cnt["valu_insts_per_launch"]) / avg_s, 4)
                    rl["fp64_valu_util"] = round(issue(cnt["fp64_valu_insts_per_launch"]) / avg_s, 4)
            r["roofline"] = rl
        del s
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
            # against the FP64 GPU path, which the parity tests hold to the
            # FP64 oracle at 1e-10 (the oracle takes minutes for this run)
            acc = accuracy(grmhd, w, P0, dev, args.accuracy_steps)
            mixed["rel_l1_vs_fp64"] = acc["all"]
            mixed["rel_l1_vs_fp64_groups"] = acc
            mixed["rel_l1_steps"] = args.accuracy_steps
            mixed["meets_1e-5"] = {"all_variables": acc["all"] <= 1e-5, "without_Phi": acc["physical"] <= 1e-5}
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
                   "cells": N, "substeps_per_step": nsub, "dt": w.dt,
                   "timing": "median of %d runs of %d steps" % (args.repeats, args.steps)},
        "roofline": main["roofline"],
        "kernels": main["kernels"],
        "ms_per_step_runs": main["ms_per_step_runs"],
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
            v = timed_run("fp64", repeats=1, **over)
            out["variants"][name] = {
                "value": v["value"], "ms_per_step": v["ms_per_step"], "recovery": v["recovery"],
                "finite": v["finite"], "kernels_avg_ms": {k: x["avg_ms"] for k, x in v["kernels"].items()},
                "vs_default": round(v["value"] / fp64["value"], 3)}
    if not args.no_batch and fp64:
        # 256 magnetised 1D Riemann problems of 200..4000 cells, each to t = 0.4
        e5 = workloads.config5()
        out["batch"] = batch_throughput(grmhd, e5, dev)
        out["batch"]["mixed"]["rel_l1_vs_fp64"] = batch_accuracy(grmhd, e5, dev)
    finite = all(r["finite"] for r in (fp64, mixed) if r)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, workloads.config3(n=96, nsteps=1))
    print(json.dumps(out), flush=True)
    return 0 if finite else 1


if __name__ == "__main__":
    sys.exit(main())
