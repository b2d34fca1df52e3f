#!/usr/bin/env python3
"""Benchmark of the chemistry hot path on one MI355X.

One step = integrating every cell of the workload over one CFD time step
(fresh initial states and a cold step size, restored from an HBM-resident copy
inside the step; the copy is ~0.03 GB and takes microseconds).  Prints one JSON
line: whole-job cells/s, the roofline of the integration kernel (FP64 ALU-bound:
algorithmic FLOPs per launch / launch time, against the 78.6 TFLOP/s FP64
vector peak) and the CPU oracle timed on a bounded sample of the same cells.
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

from paper_2105_12070_amd.inputs import WORKLOADS  # noqa: E402

FP64_PEAK_TFLOPS = 78.6
METRIC = "cells/s integrated over one CFD dt at rtol 1e-6; adjoint gradients/s"


def oracle_op_counts(name: str):
    """F_rhs and F_jac of a workload's mechanism as counted on the oracle
    (profiles/oracle_op_counts.md, written by oracle/op_counts_table.py), or None."""
    import re
    path = os.path.join(ROOT, "profiles", "oracle_op_counts.md")
    if not os.path.exists(path):
        return None
    base = "c2_54sp" if name == "zonal_54sp" else name
    got = dict(re.findall(rf"^{re.escape(base)} (f_rhs|f_jac): (\d+)", open(path).read(), flags=re.M))
    if set(got) != {"f_rhs", "f_jac"}:
        return None
    return int(got["f_rhs"]), int(got["f_jac"])


def flop_model(mech: dict, method_stages: int = 4, new_f: int = 2, name: str | None = None) -> dict:
    """Algorithmic FP64 operation counts of the method (transcendentals count 1).

    F_att: one step attempt = form M (N^2) + LU (N(N-1)/2 + (N-1)N(2N-1)/3) +
    s solves (2N^2 - N each) + new f evaluations + stage combinations (26N);
    F_step: the Jacobian pass (which also yields f(y_n)) of each accepted step.
    F_rhs and the Jacobian pass are the oracle's counts for the workload's
    mechanism (counting scalar; see oracle_op_counts); `hand` holds the
    earlier closed-form estimates of both, which count only the operations
    of the sparse formulation (third-body terms factored per row, constants
    folded) and are lower.
    """
    K = int(mech["n_species"])
    R = int(mech["n_reactions"])
    N = K + 1
    rtype = np.asarray(mech["rtype"])
    Rtb = int(np.sum(rtype >= 1))
    Rtroe = int(np.sum(rtype == 2))
    eff = np.asarray(mech["eff"])
    tb_entries = int(np.sum((eff != 1.0) & (rtype[:, None] >= 1)))
    L = 0
    for r in range(R):
        nu = {}
        for s in mech["reac"][r]:
            if s >= 0:
                nu[s] = nu.get(s, 0) - 1
        for s in mech["prod"][r]:
            if s >= 0:
                nu[s] = nu.get(s, 0) + 1
        L += sum(1 for v in nu.values() if v != 0)
    hand_rhs = 24 * R + 2 * tb_entries + Rtb + 37 * Rtroe + 2 * L + 41 * K + 10
    hand_jac = 45 * K + 36 * R + 60 * Rtroe + 22 * L + 16 * tb_entries + 6 * K * N
    counted = oracle_op_counts(name) if name else None
    f_rhs, f_jac = counted if counted else (hand_rhs, hand_jac)
    f_lu = N * (N - 1) // 2 + (N - 1) * N * (2 * N - 1) // 3
    f_solve = 2 * N * N - N
    f_att = N * N + f_lu + method_stages * f_solve + new_f * f_rhs + 26 * N
    hand_att = N * N + f_lu + method_stages * f_solve + new_f * hand_rhs + 26 * N
    return dict(f_rhs=f_rhs, f_lu=f_lu, f_solve=f_solve, f_att=f_att, f_step=f_jac, L=L,
                source="oracle op counts" if counted else "closed-form estimate",
                hand=dict(f_rhs=hand_rhs, f_step=hand_jac, f_att=hand_att))


def adjoint_flop_model(mech: dict, method_stages: int = 4, new_f: int = 3, name: str | None = None) -> dict:
    """Algorithmic FP64 operations of one reverse step (estimates, transcendentals count 1).

    With checkpoints every few steps, each accepted step has to be recomputed
    once from its checkpoint (Jacobian pass + one attempt); the kernel keeps
    that replay's factors and stages for the backward pass, replaying only the
    last step of each segment a second time, which is not counted.  The
    reverse step takes s transposed solves, s dual-number vector-Jacobian
    products of f (the second-order terms, costed as 3 first-order ones) and
    one first-order product per new f evaluation (stage sources); a
    first-order product of f costs ~3 f.
    """
    fm = flop_model(mech, name=name)
    f_vjp = 3 * fm["f_rhs"]
    f_rev = method_stages * (fm["f_solve"] + 3 * f_vjp) + new_f * f_vjp
    return dict(f_replay=fm["f_step"] + fm["f_att"], f_rev=f_rev, **fm)


KERNEL_SOURCES = ("chem_common.hpp", "chem_cell.hpp", "chem_wg.hpp", "chem.hip")
HOST_MARKER = "// ================================================================ host side"


def kernel_source_hash(root: str = ROOT) -> str:
    """sha256 over the device code of the integration kernels (the headers and
    the part of chem.hip before its host-side section) with comments, trailing
    blanks and empty lines removed: a change of kernel code changes it; host
    code and comments do not."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(root, "paper_2105_12070_amd", "csrc", f)) as fh:
            txt = fh.read()
        if f == "chem.hip":
            txt = txt.split(HOST_MARKER)[0]
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        txt = re.sub(r"//[^\n]*", "", txt)
        lines = [ln.rstrip() for ln in txt.split("\n")]
        h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()


def measured_traffic(workload: str, ncells: int, method: str = "ros4"):
    """HBM bytes per launch of the ROS4 kernel from the committed counter
    summary, or None when the kernel code changed since the counters were
    taken, no summary covers this workload, or another integrator (another
    kernel) is timed."""
    if method != "ros4":
        return None
    import re
    path = os.path.join(ROOT, "profiles", f"k_integrate_{workload}_hbm.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = {k: v for k, v in re.findall(r"^(\w+): (.+)$", txt, flags=re.M)}
    if m.get("source_sha256") != kernel_source_hash() or m.get("workload") != f"{workload} {ncells}":
        return None
    return float(m["fetch_bytes_per_launch"]) + float(m["write_bytes_per_launch"])


def cpu_baseline(w, mech, st0, target_s=12.0):
    import oracle
    oracle.build(force=False)
    nthreads = oracle.num_threads()
    # grow the sample (first n cells) until one run takes at least target_s
    n2, t2 = 32, 0.0
    while True:
        t0 = time.perf_counter()
        oracle.integrate(mech, st0[:, :n2], None, w.p_pa, w.dt, w.rtol, w.atol, nthreads=nthreads)
        t2 = time.perf_counter() - t0
        if t2 >= target_s or n2 >= min(65536, st0.shape[1]):
            break
        n2 = int(min(n2 * min(max(1.2 * target_s / max(t2, 1e-3), 2.0), 64.0), 65536, st0.shape[1]))
    # one core, on a smaller sample
    n1 = max(4, min(n2, int(n2 / max(nthreads, 1) / 2)))
    t0 = time.perf_counter()
    oracle.integrate(mech, st0[:, :n1], None, w.p_pa, w.dt, w.rtol, w.atol, nthreads=1)
    t3 = time.perf_counter() - t0
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": n2 / t2, "unit": "cells/s", "cores": nthreads, "kind": "oracle",
            "sample": f"first {n2} of the {st0.shape[1]} cells of {w.name}, same rtol/atol, "
                      f"OpenMP over cells, {t2:.1f} s",
            "note": "the plain test oracle (g++ -O3 -march=x86-64-v3, no floating-point contraction, its own "
                    "unblocked LU, no LAPACK, dense Jacobian loops), not a tuned CPU solver",
            "one_core": {"value": n1 / t3, "sample": f"first {n1} cells, {t3:.1f} s"},
            "host": {"cpus": os.cpu_count(), "model": model}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default=None, choices=sorted(WORKLOADS),
                    help="workload (default: the 262,144-cell batching workload; with --adjoint the "
                         "16,384-cell adjoint workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--graph", action="store_true", help="launch through the cached hipGraph (default for c3_batch)")
    ap.add_argument("--no-graph", action="store_true", help="plain stream launches")
    ap.add_argument("--method", default="ros4", choices=["ros4", "rodas3", "seulex"],
                    help="integrator (ROS4 is the headline; Seulex is the paper's integrator)")
    ap.add_argument("--cost-order", action="store_true",
                    help="persistent queue ordered by the previous call's step counts (default for c3_batch)")
    ap.add_argument("--no-cost-order", action="store_true", help="unordered persistent queue")
    ap.add_argument("--cells", type=int, default=0, help="integrate only the first CELLS cells (profiling)")
    ap.add_argument("--progress", action="store_true",
                    help="synchronise after every launch and report it on stderr (long launches under a profiler)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--ablation", action="store_true",
                    help="per-phase cost of the analytic vs finite-difference Jacobian and pivoted vs unpivoted "
                         "LU over an atol sweep (the shape of the paper's Figs. 2 and 3)")
    ap.add_argument("--adjoint", action="store_true",
                    help="time chem_integrate_adjoint (gradients of sum_cells[T + w.Y] w.r.t. lnA, b, theta)")
    ap.add_argument("--refmap", action="store_true",
                    help="zonal workload with and without reference-cell mapping of the ambient zone")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the cells are independent, and sharding them over "
              "several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2105_12070_amd import chem

    if args.calib_copy_mib:
        import torch
        n = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.ablation:
        return bench_ablation(args)
    if args.adjoint:
        return bench_adjoint(args)
    if args.refmap:
        return bench_refmap(args)
    args.config = args.config or "c3_batch"
    w = WORKLOADS[args.config]
    if args.config == "c3_batch":  # the batching workload is defined with the graph and the cost-ordered queue
        args.graph = args.graph or not args.no_graph
        args.cost_order = args.cost_order or not args.no_cost_order
    args.graph = args.graph and not args.no_graph
    args.cost_order = args.cost_order and not args.no_cost_order
    mech = w.mechanism()
    st0_np = w.states(mech)
    if args.cells:
        st0_np = np.ascontiguousarray(st0_np[:, :args.cells])
    dev = torch.device("cuda:0")
    m = chem.Mechanism(mech)
    nc = st0_np.shape[1]
    st0 = torch.tensor(st0_np, device=dev)
    state = st0.clone()
    h = torch.zeros(nc, dtype=torch.float64, device=dev)
    steps = torch.zeros(nc, dtype=torch.int32, device=dev)
    rejects = torch.zeros(nc, dtype=torch.int32, device=dev)
    status = torch.zeros(nc, dtype=torch.int32, device=dev)

    variant = None
    if not args.no_autotune:
        sub = min(nc, 65536)  # enough cells that throughput, not the slowest cell, decides
        variant, _ = chem.autotune(m, st0[:, :sub].contiguous(), torch.zeros(sub, dtype=torch.float64, device=dev),
                                   w.p_pa, w.dt, w.rtol, w.atol)
        print(f"# autotune on {sub} cells: {variant}", file=sys.stderr, flush=True)
    method = {"ros4": 0, "rodas3": 1, "seulex": 2}[args.method]
    opt = chem.Options(method=method, use_graph=1 if args.graph else 0, cost_order=1 if args.cost_order else 0)
    if args.graph or args.cost_order:
        opt.persistent = 1

    def one_step(ev=None):
        state.copy_(st0)
        h.zero_()
        if ev:
            ev[0].record()
        chem.integrate(m, state, h, w.p_pa, w.dt, w.rtol, w.atol, options=opt, steps=steps, rejects=rejects,
                       status=status)
        if ev:
            ev[1].record()

    def progress(msg):
        if args.progress:
            torch.cuda.synchronize()
            print(f"# {msg} done ({time.perf_counter() - t_start:.1f} s)", file=sys.stderr, flush=True)

    t_start = time.perf_counter()
    for i in range(args.warmup):
        one_step()
        progress(f"warmup {i}")
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        one_step(evs[i])
        progress(f"step {i}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_list = [a.elapsed_time(b) for a, b in evs]
    kern_ms = float(np.mean(kern_list))
    st = status.cpu().numpy()
    sp = steps.cpu().numpy().astype(np.int64)
    rj = rejects.cpu().numpy().astype(np.int64)
    if np.any(st != 0):
        print(f"# warning: {np.sum(st != 0)} cells with nonzero status {np.bincount(st)}", file=sys.stderr)
    fm = flop_model(mech, name=w.name)
    work = None
    flops_hand = None
    if args.method == "seulex":
        work = seulex_work(chem, m, st0, w, sp)
        flops = work.pop("flops")
    else:
        flops = float(np.sum((sp + rj) * fm["f_att"] + sp * fm["f_step"]))
        flops_hand = float(np.sum((sp + rj) * fm["hand"]["f_att"] + sp * fm["hand"]["f_step"]))
    achieved = flops / (kern_ms * 1e-3) / 1e12

    plain = None
    if not args.no_plain and w.N <= 64:  # the workgroup path (N > 64) has only the persistent launch
        popt = chem.Options(method=method, persistent=0, waves_per_block=1)
        state.copy_(st0)
        h.zero_()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        chem.integrate(m, state, h, w.p_pa, w.dt, w.rtol, w.atol, options=popt)
        b.record()
        torch.cuda.synchronize()
        plain = nc / (a.elapsed_time(b) * 1e-3)
        progress("plain launch")

    # a warm call: the same cells again from the step sizes the last call
    # returned (the flow solver calls the chemistry again within a time step)
    h_warm = h.clone()
    state.copy_(st0)
    h.copy_(h_warm)
    wa, wb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wa.record()
    chem.integrate(m, state, h, w.p_pa, w.dt, w.rtol, w.atol, options=opt, steps=steps, rejects=rejects,
                   status=status)
    wb.record()
    torch.cuda.synchronize()
    progress("warm call")
    warm = {"cells_per_s": nc / (wa.elapsed_time(wb) * 1e-3),
            "steps_mean": float(steps.float().mean()), "rejects_mean": float(rejects.float().mean())}

    value = nc * args.steps / elapsed
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generator: element-balanced Chemkin-form mechanism, random states)",
        "config": {"workload": f"{w.name}: {w.n_species} species / {w.n_reactions} reactions "
                               f"({w.n_thirdbody} third-body, {w.n_troe} Troe), {nc} cells, p = {w.p_pa:g} Pa, "
                               f"dt = {w.dt:g} s, rtol {w.rtol:g}, atol {w.atol:g}, {args.method.upper()}",
                   "n_cells": nc, "N": w.N, "variant": variant, "graph": bool(args.graph),
                   "cost_order": bool(args.cost_order)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": measured_traffic(w.name, nc, args.method),
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_bytes": nc * (16 * (w.N + 1) + 12),
                     "kernel_ms": kern_ms, "kernel_ms_median": float(np.median(kern_list)),
                     "flops_per_launch": flops, "flops_source": fm["source"],
                     "frac_closed_form_estimate": (flops_hand / (kern_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS
                                                   if flops_hand else None)},
        "steps_mean": float(sp.mean()), "rejects_mean": float(rj.mean()),
        "steps_percentiles_0_50_90_99_100": np.percentile(sp, [0, 50, 90, 99, 100]).tolist(),
        "plain_one_cell_per_block_cells_per_s": plain,
        "warm_call": warm,
    }
    if work:
        out["seulex_work"] = work
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, mech, st0_np)
    print(json.dumps(out), flush=True)


def seulex_work(chem, m, st0, w, steps_timed):
    """FLOPs of one Seulex launch from the instrumented kernel's counters
    (factorisations and substeps per cell), taken in an untimed run with the
    same arithmetic: per factorisation N^2 + F_LU (form M, LU); per substep
    F_solve + N; per substep after a column's first F_rhs + 3N (f and the
    extrapolation table); per attempt 10N (error norms); per step F_jac."""
    import torch
    mech = w.mechanism()
    fm = flop_model(mech, name=w.name)
    N = w.N
    nc = st0.shape[1]
    s = st0.clone()
    h = torch.zeros(nc, dtype=torch.float64, device=st0.device)
    steps = torch.zeros(nc, dtype=torch.int32, device=st0.device)
    rej = torch.zeros(nc, dtype=torch.int32, device=st0.device)
    pc = torch.zeros((nc, 8), dtype=torch.int64, device=st0.device)
    chem.integrate(m, s, h, w.p_pa, w.dt, w.rtol, w.atol, options=chem.Options(method=2, phase_cycles=pc),
                   steps=steps, rejects=rej)
    torch.cuda.synchronize()
    sp = steps.cpu().numpy().astype(np.int64)
    rj = rej.cpu().numpy().astype(np.int64)
    pcn = pc.cpu().numpy()
    nlu, nsub = pcn[:, 6].astype(np.float64), pcn[:, 7].astype(np.float64)
    if not np.array_equal(sp, steps_timed):
        raise RuntimeError("instrumented Seulex run took other steps than the timed run")
    flops = float(np.sum(nlu * (N * N + fm["f_lu"]) + nsub * (fm["f_solve"] + N)
                         + (nsub - nlu) * (fm["f_rhs"] + 3 * N) + (sp + rj) * 10 * N + sp * fm["f_step"]))
    return {"flops": flops, "lu_per_attempt": float(nlu.sum() / (sp + rj).sum()),
            "substeps_per_attempt": float(nsub.sum() / (sp + rj).sum())}


def bench_refmap(args):
    """The zonal workload (75% ambient-zone cells among reacting ones): cells/s
    with reference-cell mapping against the same integration without it, the
    share of cells mapped, and the mapping error (mapped cells against their
    own integration)."""
    import torch
    from paper_2105_12070_amd import chem

    w = WORKLOADS["zonal_54sp"]
    mech = w.mechanism()
    st0_np = w.states(mech)
    if args.cells:
        st0_np = np.ascontiguousarray(st0_np[:, :args.cells])
    nc = st0_np.shape[1]
    dev = torch.device("cuda:0")
    m = chem.Mechanism(mech)
    rm = w.refmap_params()
    st0 = torch.tensor(st0_np, device=dev)
    state = st0.clone()
    h = torch.zeros(nc, dtype=torch.float64, device=dev)
    steps = torch.zeros(nc, dtype=torch.int32, device=dev)
    status = torch.zeros(nc, dtype=torch.int32, device=dev)
    ref_of = torch.zeros(nc, dtype=torch.int32, device=dev)
    refmap = chem.RefMap(torch.tensor(rm["weight"], device=dev), rm["z0"], rm["z_max"], rm["dT"], ref_of)
    opts = {"mapped": chem.Options(refmap=refmap), "unmapped": chem.Options()}

    def timed(opt):
        for _ in range(args.warmup):
            state.copy_(st0)
            h.zero_()
            chem.integrate(m, state, h, w.p_pa, w.dt, w.rtol, w.atol, options=opt, steps=steps, status=status)
        torch.cuda.synchronize()
        el = 0.0
        for _ in range(args.steps):
            state.copy_(st0)
            h.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            chem.integrate(m, state, h, w.p_pa, w.dt, w.rtol, w.atol, options=opt, steps=steps, status=status)
            torch.cuda.synchronize()
            el += time.perf_counter() - t0
        return el, state.cpu().numpy(), steps.cpu().numpy(), status.cpu().numpy()

    el_m, out_m, steps_m, st_m = timed(opts["mapped"])
    rof = ref_of.cpu().numpy()
    el_u, out_u, steps_u, st_u = timed(opts["unmapped"])
    mapped = rof >= 0
    err = np.abs(out_m - out_u)[:, mapped]
    scale = w.rtol * np.abs(out_u[:, mapped]) + w.atol
    value = nc * args.steps / el_m
    out = {"metric": "cells/s with reference-cell mapping (zonal workload)", "value": value, "unit": "cells/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": el_m * 1e3 / args.steps,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"zonal_54sp: 54 species / 270 reactions, {nc} cells (75% ambient zone, "
                                  f"T jittered by 2 K), p = {w.p_pa:g} Pa, dt = {w.dt:g} s, rtol {w.rtol:g}, "
                                  f"atol {w.atol:g}, ROS4; zone: Y_{int(np.argmax(rm['weight']))} <= {rm['z_max']:g}, "
                                  f"dT = {rm['dT']:g} K"},
           "unmapped_cells_per_s": nc * args.steps / el_u, "speedup": el_u / el_m,
           "mapped_fraction": float(mapped.mean()),
           "steps_total": {"mapped_run": int(steps_m.astype(np.int64).sum()),
                           "unmapped_run": int(steps_u.astype(np.int64).sum())},
           "mapping_error": {"max_over_tol": float((err / scale).max()) if mapped.any() else 0.0,
                             "mean_over_tol": float((err / scale).mean()) if mapped.any() else 0.0,
                             "max_T_K": float(err[0].max()) if mapped.any() else 0.0},
           "failed_cells": int((st_m != 0).sum() + (st_u != 0).sum())}
    print(json.dumps(out), flush=True)


def bench_ablation(args):
    """The 53-species / 325-reaction mechanism (the size of GRI-3.0 in Figs. 2-3)
    at 13.5 atm and T = 1200 K over dt = 1e-6 s, rtol 1e-6, atol swept: cells/s
    and the share of each phase for the four combinations of analytic or
    finite-difference Jacobian and pivoted or unpivoted LU."""
    import torch
    from paper_2105_12070_amd import chem
    from paper_2105_12070_amd.inputs import make_states

    w = WORKLOADS["c4_adj"]
    mech = w.mechanism()
    nc = args.cells or 2048
    st0_np = make_states(mech, nc, 2104, [(1200.0, 1200.0)])
    p = 13.5 * 101325.0
    dev = torch.device("cuda:0")
    m = chem.Mechanism(mech)
    st0 = torch.tensor(st0_np, device=dev)
    names = ["jac", "formM", "lu", "stage_f", "solves", "total"]
    rows = []
    for atol in (1e-8, 1e-10, 1e-12, 1e-14):
        for jm, lp, label in ((0, 0, "analytic J + pivoted LU"), (1, 0, "FD J + pivoted LU"),
                              (0, 1, "analytic J + unpivoted LU"), (1, 1, "FD J + unpivoted LU")):
            s = st0.clone()
            h = torch.zeros(nc, dtype=torch.float64, device=dev)
            steps = torch.zeros(nc, dtype=torch.int32, device=dev)
            rej = torch.zeros(nc, dtype=torch.int32, device=dev)
            status = torch.zeros(nc, dtype=torch.int32, device=dev)
            pc = torch.zeros((nc, 8), dtype=torch.int64, device=dev)
            opt = chem.Options(phase_cycles=pc, jac_mode=jm, lu_pivot=lp)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            chem.integrate(m, s, h, p, w.dt, 1e-6, atol, options=opt, steps=steps, rejects=rej, status=status)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            c = pc.cpu().numpy().astype(np.float64).sum(axis=0)
            rows.append({"atol": atol, "mode": label, "cells_per_s": nc / el,
                         "steps_mean": float(steps.float().mean()), "rejects_mean": float(rej.float().mean()),
                         "failed_cells": int((status != 0).sum()),
                         "phase_share": {n: float(c[i] / c[5]) for i, n in enumerate(names[:5])}})
            print(f"# atol {atol:g} {label}: {nc / el:.0f} cells/s, steps {rows[-1]['steps_mean']:.0f}, "
                  f"jac share {rows[-1]['phase_share']['jac']:.2f}", file=sys.stderr, flush=True)
    base = [r for r in rows if r["atol"] == 1e-10 and r["mode"].startswith("analytic J + pivoted")][0]
    print(json.dumps({"metric": "ablation: cells/s and phase shares, analytic vs finite-difference Jacobian, "
                                "pivoted vs unpivoted LU", "value": base["cells_per_s"], "unit": "cells/s",
                      "n_gpus": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": f"53 species / 325 reactions, {nc} cells at T = 1200 K, p = 13.5 atm, "
                                             "dt = 1e-6 s, rtol 1e-6, atol swept"},
                      "rows": rows}), flush=True)


def bench_adjoint(args):
    import torch
    from paper_2105_12070_amd import chem
    from paper_2105_12070_amd.inputs import objective_weights

    name = args.config or "c4_adj"
    w = WORKLOADS[name]
    mech = w.mechanism()
    st0_np = w.states(mech)
    if args.cells:
        st0_np = np.ascontiguousarray(st0_np[:, :args.cells])
    nc = st0_np.shape[1]
    dev = torch.device("cuda:0")
    m = chem.Mechanism(mech)
    st0 = torch.tensor(st0_np, device=dev)
    lam = torch.empty_like(st0)
    lam[0] = 1.0
    lam[1:] = torch.tensor(objective_weights(w.n_species), device=dev)[:, None]
    h = torch.zeros(nc, dtype=torch.float64, device=dev)
    ck, max_tape = 8, 8192
    ev = None

    def one_step(evp=None):
        h.zero_()
        if evp:
            evp[0].record()
        r = chem.integrate_adjoint(m, st0, h, w.p_pa, w.dt, w.rtol, w.atol, lam, checkpoint_every=ck,
                                   max_tape=max_tape)
        if evp:
            evp[1].record()
        return r

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = one_step(evs[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    call_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    out, lam0, grad, steps, status = res
    st = status.cpu().numpy()
    sp = steps.cpu().numpy().astype(np.int64)
    if np.any(st != 0):
        print(f"# warning: {np.sum(st != 0)} cells with nonzero status {np.bincount(st)}", file=sys.stderr)
    # forward-only rate on the same cells and the plain one-cell-per-block launch, for context
    s2 = st0.clone()
    h.zero_()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    chem.integrate(m, s2, h, w.p_pa, w.dt, w.rtol, w.atol)
    b.record()
    s2.copy_(st0)
    h.zero_()
    c, d = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c.record()
    chem.integrate(m, s2, h, w.p_pa, w.dt, w.rtol, w.atol, options=chem.Options(persistent=0, waves_per_block=1))
    d.record()
    torch.cuda.synchronize()
    fwd_ms, plain_ms = a.elapsed_time(b), c.elapsed_time(d)
    fm = adjoint_flop_model(mech, name=w.name)
    flops_adj = float(np.sum(sp * (fm["f_replay"] + fm["f_rev"])))
    adj_kernel_ms = max(call_ms - fwd_ms, 1e-6)
    achieved = flops_adj / (adj_kernel_ms * 1e-3) / 1e12
    value = nc * args.steps / elapsed
    outd = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-gradients/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generator: element-balanced Chemkin-form mechanism, random states)",
        "config": {"workload": f"{w.name}: {w.n_species} species / {w.n_reactions} reactions, {nc} cells, "
                               f"p = {w.p_pa:g} Pa, dt = {w.dt:g} s, rtol {w.rtol:g}, atol {w.atol:g}, ROS4; "
                               f"gradient of sum_cells [T + w.Y](dt) w.r.t. lnA, b, theta of all "
                               f"{w.n_reactions} reactions and the initial states; checkpoints every {ck} steps",
                   "n_cells": nc, "N": w.N},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None, "kernel": "k_adjoint",
                     "kernel_ms": adj_kernel_ms, "flops_per_launch": flops_adj,
                     "note": "reverse-sweep FLOPs estimated by adjoint_flop_model; kernel time = call time "
                             "minus the forward integration time"},
        "forward_cells_per_s": nc / (fwd_ms * 1e-3),
        "plain_one_cell_per_block_cells_per_s": nc / (plain_ms * 1e-3),
        "adjoint_over_forward_time": call_ms / fwd_ms,
        "steps_mean": float(sp.mean()),
    }
    print(json.dumps(outd), flush=True)


if __name__ == "__main__":
    main()
