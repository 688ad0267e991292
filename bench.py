#!/usr/bin/env python3
"""Benchmark of the FC-RKPM Poisson hot path on one MI355X.

One step = the whole path on one synthetic input already resident in HBM:
setup (kernel spectra, moment convolutions and per-node moment solves, Alg 1),
load vector (Alg 4), CG on the stiffness operator (Alg 2 inside Alg 5; FP32
FFT matvecs inside FP64 iterative refinement by default) and the field u^h
(Alg 3).  The headline value is CG matvecs per second over the timed steps
(every K product counts: FP32 inner and FP64 outer); DOF/s multiplies by the
free unknowns.

Prints one JSON line.  Usage:
  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5|paper|c3|c4]
                  [--mode f32_refined|f64] [--tol 1e-12] [--no-cpu-baseline]
                  [--no-fp64-compare]

--workload c4 measures the batched path instead: 16 cube problems (boxes
32^3 .. 96^3) and 32 seeded Gaussian right-hand sides on a 96^3 box in one
fcrkpm_solve_batch call per step, a fixed number of CG iterations (--c4-iters)
from a zero start; the value is node-rhs K products per second over the batch,
with CG blocks replayed from captured HIP graphs, beside the same batch with
direct launches.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5", choices=["c5", "c5_256", "paper", "c3", "c4", "c1", "c2"])
    ap.add_argument("--c4-iters", type=int, default=240)
    ap.add_argument("--probe", type=int, default=0,
                    help="counter probe: setup, a refined solve capped at N CG iterations "
                         "(direct launches), then a 256 MiB device copy that calibrates the "
                         "memory counters; prints one line and exits")
    ap.add_argument("--probe-variant", type=int, default=1,
                    help="register-path variant for --probe (layout + 2 (tiles - 1)); the "
                         "default is the one setup's autotuner picks for 128^3 on MI355X")
    ap.add_argument("--mode", default=None, choices=["f32_refined", "f64"],
                    help="default: f64 for c1 and c2 (plain FP64 configurations), else f32_refined")
    ap.add_argument("--tol", type=float, default=1e-12)
    ap.add_argument("--maxit", type=int, default=100000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="skip the short runs of the other configurations in the default c5 line")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--cpu-cg-cap", type=int, default=10,
                    help="iterations of the oracle's CG solve and adjoint on boxes above 64^3")
    ap.add_argument("--table1", action="store_true",
                    help="the paper's timing table instead: setup, K (FP64 and FP32), f^r and u^h "
                         "on the Eq 106 problem (support 1.5h) at boxes 8^3 .. 256^3")
    ap.add_argument("--fixed-iters", type=int, default=0,
                    help="run exactly N CG iterations per step instead of solving to --tol "
                         "(throughput of workloads whose CG converges too slowly, e.g. c3)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: the FC-RKPM path runs on one GPU only (asked for --gpus {a.gpus}); "
              "the single-GPU run is the whole workload", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2403_19854_amd import fcrkpm
    from paper_2403_19854_amd import traffic
    from paper_2403_19854_amd import workloads as W

    fcrkpm.load_library()
    if a.mode is None:
        a.mode = "f64" if a.workload in ("c1", "c2") else "f32_refined"
    if a.table1:
        return bench_table1(a)
    if a.workload == "c4":
        return bench_c4(a)
    wl = {"c5": W.config5, "c5_256": W.config5_256, "paper": W.paper_shape, "c3": W.config3,
          "c1": W.config1, "c2": W.config2}[a.workload]()
    if a.probe:
        return probe(a, wl)
    dev = torch.device("cuda:0")
    chi = torch.from_numpy(wl.chi).to(dev)
    dirm = torch.from_numpy(wl.dirichlet).to(dev)
    vol = torch.from_numpy(wl.vol).to(dev)
    r = torch.from_numpy(wl.r).to(dev)
    torch.cuda.synchronize()

    def step(mode, profile=False):
        pb = fcrkpm.Problem(wl.dims, wl.h, wl.at, wl.degree, chi, dirm, vol, device=dev)
        if profile:
            pb.profile(True)
        if a.fixed_iters:
            d, uh, info = pb.solve(r, mode=mode, tol=1e-300, maxit=a.fixed_iters, want_uh=True,
                                   raise_on_noconv=False)
        else:
            d, uh, info = pb.solve(r, mode=mode, tol=a.tol, maxit=a.maxit, want_uh=True)
        info["layout"] = pb.get_option(fcrkpm.OPT_REGLAYOUT)
        prof = None
        if profile:
            pb.profile(False)
            prof = pb.profile_read()
        pb.close()
        return info, prof, uh, d

    for _ in range(a.warmup):
        step(a.mode)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    prof_acc = {}
    step_ms = []
    for i in range(a.steps):
        ts = time.perf_counter()
        info, prof, uh, d_final = step(a.mode, profile=True)
        step_ms.append(1e3 * (time.perf_counter() - ts))
        infos.append(info)
        for k, (n, ms, by) in prof.items():
            n0, w0, b0 = prof_acc.get(k, (0, 0.0, 0.0))
            prof_acc[k] = (n0 + n, w0 + ms * n, by)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    clocks = gpu_clocks()
    matvecs = sum(i["matvecs_f32"] + i["matvecs_f64"] for i in infos)
    value = matvecs / elapsed
    n_free = wl.n_free
    # the dominant kernel: largest estimated share of device time
    kernels = {k: {"launches": n, "mean_ms": w / n, "bytes_per_launch": by,
                   "est_total_ms": w}
               for k, (n, w, by) in prof_acc.items()}
    dom = max(kernels, key=lambda k: kernels[k]["est_total_ms"])
    dk = kernels[dom]
    achieved = dk["bytes_per_launch"] / (dk["mean_ms"] * 1e-3) / 1e9
    m = wl.chi > 0
    uh_err = float(np.linalg.norm((uh.cpu().numpy() - wl.u_exact)[m]) /
                   np.linalg.norm(wl.u_exact[m])) if wl.u_exact is not None else None

    out = {
        "metric": ("CG matvecs/s at 128^3 (K products of the refined-FP32 solve, FP64 outer residual)"
                   if a.workload == "c5" and a.mode == "f32_refined" else
                   f"CG matvecs/s, {wl.name} ({'refined FP32' if a.mode == 'f32_refined' else 'FP64'})"),
        "value": value,
        "unit": "matvec/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "step_ms_median_iqr": [float(np.median(step_ms))] + [float(v) for v in np.percentile(step_ms, [25, 75])],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if a.mode == "f32_refined" else "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "box": list(wl.dims), "support": wl.at[0],
                   "degree": wl.degree, "free_unknowns": n_free, "mode": a.mode,
                   "tol": None if a.fixed_iters else a.tol,
                   "step": (f"setup + f^r + {a.fixed_iters} CG iterations + u^h" if a.fixed_iters
                            else "setup + f^r + CG to tol + u^h")},
        "dof_per_s": value * n_free,
        "us_per_matvec": 1e6 / value,
        "box_nodes_per_s": value * float(np.prod(wl.dims)),
        "solve": {"iters": infos[-1]["iters"], "outer_iters": infos[-1]["outer_iters"],
                  "matvecs_f32": infos[-1]["matvecs_f32"],
                  "matvecs_f64": infos[-1]["matvecs_f64"],
                  "true_rel_res": infos[-1]["true_rel_res"],
                  "fallback_used": infos[-1]["fallback_used"],
                  "register_variant": infos[-1]["layout"],
                  "uh_rel_l2_vs_exact": uh_err},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic.load(wl.name, dom, infos[-1]["layout"]),
                     "mean_ms": dk["mean_ms"], "bytes_per_launch": dk["bytes_per_launch"]},
        "kernels": kernels,
        "gpu_clocks": clocks,
    }

    if not a.no_fp64_compare and a.mode != "f64":
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        info64, _, uh64, _ = step("f64")
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        e = float(np.linalg.norm((uh.cpu().numpy() - uh64.cpu().numpy())[m]) /
                  np.linalg.norm(uh64.cpu().numpy()[m]))
        out["fp64_path"] = {"ms_per_step": 1e3 * (t3 - t2), "iters": info64["iters"],
                            "matvecs_per_s": info64["matvecs_f64"] / (t3 - t2),
                            "speedup_refined_vs_fp64": (t3 - t2) / (elapsed / a.steps),
                            "uh_rel_l2_refined_vs_fp64": e}

    if not a.no_fp64_compare and a.mode != "f64" and not a.fixed_iters:
        out["time_to_solution"] = time_to_solution(a, wl, chi, dirm, vol, r, dev)
        out["apply_loop"] = apply_loop(wl, chi, dirm, vol, dev)
        if a.workload == "c5":
            out["adjoint"] = adjoint_time(a, wl, chi, dirm, vol, r, dev)
            out["transient"] = transient_time(a, wl, chi, dirm, vol, r, dev)
            out["flux"] = flux_time(a, wl, dev)
            out["nonlinear"] = nonlinear_time(a, wl, chi, dirm, vol, dev)
            out["nonlinear_cg"] = nonlinear_cg_time(a, wl, chi, dirm, vol, dev)
            if not a.no_other_configs:
                out["other_configs"] = other_configs(a, dev)

    if not a.no_cpu_baseline:
        gpu_iters = out.get("fp64_path", {}).get("iters")
        out["cpu_baseline"] = cpu_baseline(a, wl, gpu_iters,
                                           d_final.cpu().numpy() if a.fixed_iters else None)
        if a.fixed_iters:
            out["solve"]["oracle_rel_res"] = out["cpu_baseline"].pop("oracle_rel_res")
    print(json.dumps(out), flush=True)


def cpu_baseline(a, wl, gpu_iters=None, d_fixed=None):
    """The oracle (FP64 neighbour-loop RKPM on the host cores) on the same grid:

    * value: K products per second with all its threads, over about
      --cpu-seconds of products;
    * one_thread: one K product on one thread;
    * fr_s, uh_s: one f^r and one u^h with all its threads;
    * solve / adjoint: its CG solve of the load (Alg 5) and its adjoint solve to
      the bench tolerance; on boxes above 64^3 both are capped at --cpu-cg-cap
      iterations and the time at the GPU's FP64 iteration count is extrapolated
      from the time per iteration (stated as such);
    * with d_fixed (a fixed-iteration GPU run), the relative residual
      |chi_Omega (f^r - K d)| / |chi_Omega f^r| of that d under the oracle's
      operator."""
    import numpy as np

    import oracle
    from paper_2403_19854_amd import workloads as W

    threads = oracle.threads(0)
    t0 = time.perf_counter()
    o = oracle.Oracle(wl.dims, wl.h, wl.at, wl.degree, wl.chi, wl.vol)
    t_setup = time.perf_counter() - t0
    x = np.where(wl.free > 0, np.random.default_rng(0).standard_normal(wl.shape), 0.0)
    n = 0
    tc0 = time.perf_counter()
    while True:
        o.apply_k_free(x, wl.free)
        n += 1
        if time.perf_counter() - tc0 >= a.cpu_seconds:
            break
    tc = time.perf_counter() - tc0
    res = {"value": n / tc, "unit": "matvec/s", "cores": threads, "kind": "oracle",
           "sample": f"{n} oracle K products (neighbour-loop RKPM, FP64) on the same {wl.name} "
                     f"grid, {tc:.1f} s",
           "setup_s": t_setup}
    oracle.threads(1)
    try:
        t0 = time.perf_counter()
        o.apply_k_free(x, wl.free)
        t1 = time.perf_counter() - t0
    finally:
        oracle.threads(threads)
    res["one_thread"] = {"value": 1.0 / t1, "unit": "matvec/s", "cores": 1,
                         "sample": "one oracle K product on one thread"}
    # the load f^r (Alg 4) and the field u^h (Alg 3), once each, all threads
    t0 = time.perf_counter()
    o.apply_fr(wl.r)
    t_fr = time.perf_counter() - t0
    t0 = time.perf_counter()
    o.apply_uh(x)
    res["fr_s"], res["uh_s"] = t_fr, time.perf_counter() - t0
    big = int(np.prod(wl.dims)) > 64 ** 3
    cap = a.cpu_cg_cap if big else a.maxit
    t0 = time.perf_counter()
    _, it, rel = o.solve(wl.free, wl.dirichlet, wl.r, tol=a.tol, maxit=cap)
    ts = time.perf_counter() - t0
    sol = {"tol": a.tol, "iterations": it, "rel_res": rel, "seconds": ts, "cores": threads}
    if rel > a.tol:
        sol["capped_at"] = cap
        sol["s_per_iteration"] = ts / max(it, 1)
        if gpu_iters:
            sol["est_seconds_at_gpu_fp64_iterations"] = ts / max(it, 1) * gpu_iters
            sol["gpu_fp64_iterations"] = gpu_iters
    res["solve"] = sol
    rng = np.random.default_rng(7)
    dl = (W.config5_target(wl) if wl.name.startswith("c5") else
          np.where(wl.chi > 0, rng.standard_normal(wl.shape), 0.0))
    t0 = time.perf_counter()
    _, _, it = o.adjoint(wl.free, dl, tol=a.tol, maxit=cap)
    ta = time.perf_counter() - t0
    adj = {"tol": a.tol, "iterations": it, "seconds": ta, "cores": threads}
    if big:
        adj["capped_at"] = cap
        adj["s_per_iteration"] = ta / max(it, 1)
    res["adjoint"] = adj
    if d_fixed is not None:
        fr = np.where(wl.free > 0, o.apply_fr(wl.r), 0.0)
        rr = np.where(wl.free > 0, fr - o.apply_k(d_fixed), 0.0)
        res["oracle_rel_res"] = float(np.linalg.norm(rr) / np.linalg.norm(fr))
    return res


def time_to_solution(a, wl, chi, dirm, vol, r, dev):
    """Solve-call wall time (setup excluded) of the refined and the plain FP64
    solve on one context, both to the bench tolerance, and how far apart their
    solutions are."""
    import numpy as np
    import torch

    from paper_2403_19854_amd import fcrkpm

    pb = fcrkpm.Problem(wl.dims, wl.h, wl.at, wl.degree, chi, dirm, vol, device=dev)
    res = {"tol": a.tol}
    ds = {}
    for mode in ("f32_refined", "f64"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d, _, info = pb.solve(r, mode=mode, tol=a.tol, maxit=a.maxit, want_uh=False)
        torch.cuda.synchronize()
        res[mode + "_ms"] = 1e3 * (time.perf_counter() - t0)
        res[mode + "_iters"] = info["iters"]
        ds[mode] = d.cpu().numpy()
    pb.close()
    m = wl.free > 0
    res["speedup"] = res["f64_ms"] / res["f32_refined_ms"]
    res["d_rel_l2_refined_vs_f64"] = float(np.linalg.norm((ds["f32_refined"] - ds["f64"])[m]) /
                                           np.linalg.norm(ds["f64"][m]))
    return res


def adjoint_time(a, wl, chi, dirm, vol, r, dev):
    """The gradient of L = 0.5 |u^h - u_t|^2 with respect to r (config 5): the
    forward solve for u^h, then the adjoint (N^T, a solve with K, V o N), both
    refined FP32 to the bench tolerance; wall times of the two calls."""
    import numpy as np
    import torch

    from paper_2403_19854_amd import fcrkpm
    from paper_2403_19854_amd import workloads as W

    pb = fcrkpm.Problem(wl.dims, wl.h, wl.at, wl.degree, chi, dirm, vol, device=dev)
    ut = torch.from_numpy(W.config5_target(wl)).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, uh, info_f = pb.solve(r, mode="f32_refined", tol=a.tol, maxit=a.maxit, want_uh=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g, info_a = pb.adjoint(uh - ut, mode="f32_refined", tol=a.tol, maxit=a.maxit)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    pb.close()
    return {"forward_ms": 1e3 * (t1 - t0), "adjoint_ms": 1e3 * (t2 - t1),
            "adjoint_iters": info_a["iters"],
            "adjoint_matvecs_per_s": (info_a["matvecs_f32"] + info_a["matvecs_f64"]) / (t2 - t1),
            "grad_norm": float(torch.linalg.vector_norm(g).item())}


def transient_time(a, wl, chi, dirm, vol, r, dev, steps=2, explicit_steps=50):
    """Time-dependent diffusion on the same grid (App. C), source r, nu = 1,
    from d = 0: `steps` backward-Euler steps with dt = 4 h^2 (one solve with
    M + dt K each; refined FP32 and FP64, both to the bench tolerance), then
    `explicit_steps` forward-Euler steps with the lumped mass and dt = 0.02 h^2,
    and standalone mass products."""
    import numpy as np
    import torch

    from paper_2403_19854_amd import fcrkpm

    pb = fcrkpm.Problem(wl.dims, wl.h, wl.at, wl.degree, chi, dirm, vol, device=dev)
    h2 = min(wl.h) ** 2
    d0 = torch.zeros(wl.shape, dtype=torch.float64, device=dev)
    res = {"nu": 1.0, "implicit": {"theta": 1.0, "dt": 4.0 * h2, "steps": steps, "tol": a.tol}}
    ds = {}
    pb.transient(d0, 1.0, 4.0 * h2, 0, r=r, tol=a.tol)  # zero steps: builds the rows of M and M + dt K
    for mode in ("f32_refined", "f64"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d, _, info = pb.transient(d0, 1.0, 4.0 * h2, steps, r=r, mode=mode, tol=a.tol, maxit=a.maxit)
        torch.cuda.synchronize()
        res["implicit"][mode + "_ms"] = 1e3 * (time.perf_counter() - t0)
        res["implicit"][mode + "_iters"] = info["iters"]
        ds[mode] = d.cpu().numpy()
    m = wl.free > 0
    res["implicit"]["speedup"] = res["implicit"]["f64_ms"] / res["implicit"]["f32_refined_ms"]
    res["implicit"]["d_rel_l2_refined_vs_f64"] = float(
        np.linalg.norm((ds["f32_refined"] - ds["f64"])[m]) / np.linalg.norm(ds["f64"][m]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pb.transient(d0, 1.0, 0.02 * h2, explicit_steps, r=r, scheme="explicit", mode="f64")
    torch.cuda.synchronize()
    te = time.perf_counter() - t0
    res["explicit"] = {"dt": 0.02 * h2, "steps": explicit_steps, "ms": 1e3 * te,
                       "steps_per_s": explicit_steps / te}
    pb.close()
    res["mass_products"] = apply_loop(wl, chi, dirm, vol, dev, op="M")
    return res


def flux_time(a, wl, dev, reps=20):
    """A flux boundary on the same box (App. A): the cube's x = 1 face carries
    q = du/dx of the manufactured solution (areas h^2), the other faces keep
    u = 0; the refined solve with f^q in its right-hand side, its u^h error,
    and standalone flux loads (median over `reps`, HIP events)."""
    import numpy as np
    import torch

    from paper_2403_19854_amd import fcrkpm
    from paper_2403_19854_amd import workloads as W

    p = W.cube_neumann(wl.dim, wl.dims[0], wl.at[0], wl.degree)
    pb = fcrkpm.Problem.from_workload(p, device=dev)
    pb.set_boundary(torch.from_numpy(p.area))
    r = torch.from_numpy(p.r).to(dev)
    q = torch.from_numpy(p.q).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d, uh, info = pb.solve(r, q=q, mode="f32_refined", tol=a.tol, maxit=a.maxit)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    m = p.chi > 0
    err = float(np.linalg.norm((uh.cpu().numpy() - p.u_exact)[m]) / np.linalg.norm(p.u_exact[m]))
    st = torch.cuda.current_stream()
    res = {"flux_nodes": int((p.area > 0).sum()), "solve_ms": 1e3 * ts, "iters": info["iters"],
           "uh_rel_l2_vs_exact": err}
    for name, qt in (("f32", q.float()), ("f64", q)):
        y = torch.empty_like(qt)
        for _ in range(5):
            pb.apply("FQ", qt, out=y, stream=st)
        tl = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            pb.apply("FQ", qt, out=y, stream=st)
            e1.record(st)
            e1.synchronize()
            tl.append(e0.elapsed_time(e1))
        res["load_" + name + "_median_ms"] = float(np.median(tl))
    pb.close()
    return res


def nonlinear_time(a, wl, chi, dirm, vol, dev, kappa=5.0):
    """-lap u + kappa u^3 = r on the same grid (App. B), r manufactured from
    the workload's u: the refined Newton solve from d = 0 (each step's CG to
    the bench tolerance, Newton to 1e-10), its steps, CG iterations and u^h
    error."""
    import numpy as np
    import torch

    from paper_2403_19854_amd import fcrkpm

    pb = fcrkpm.Problem(wl.dims, wl.h, wl.at, wl.degree, chi, dirm, vol, device=dev)
    r = torch.from_numpy(wl.r + kappa * wl.u_exact ** 3).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d, uh, info = pb.solve_nonlinear(r, kappa, mode="f32_refined", tol=a.tol, newton_tol=1e-10,
                                     maxit=a.maxit)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    pb.close()
    m = wl.chi > 0
    err = float(np.linalg.norm((uh.cpu().numpy() - wl.u_exact)[m]) / np.linalg.norm(wl.u_exact[m]))
    return {"kappa": kappa, "solve_ms": 1e3 * ts, "newton_steps": info["outer_iters"],
            "cg_iters": info["iters"], "residual": info["rel_res"], "uh_rel_l2_vs_exact": err}


def nonlinear_cg_time(a, wl, chi, dirm, vol, dev, kappa=5.0, kappa_grad=0.5, tol=1e-10):
    """Nonlinear CG (Alg B.3, FP64) on the same grid from d = 0, to relative
    residual `tol`: the cubic force with r manufactured from the workload's u
    (-lap u + kappa u^3 = r; u^h error reported), and the gradient force
    (1 + kappa |grad u|^2) grad u with the workload's r."""
    import numpy as np
    import torch

    from paper_2403_19854_amd import fcrkpm

    pb = fcrkpm.Problem(wl.dims, wl.h, wl.at, wl.degree, chi, dirm, vol, device=dev)
    m = wl.chi > 0
    res = {"tol": tol}
    for kind, kap, rr in (("cubic", kappa, wl.r + kappa * wl.u_exact ** 3),
                          ("gradient", kappa_grad, wl.r)):
        r = torch.from_numpy(rr).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d, uh, info = pb.solve_nonlinear_cg(r, kap, kind=kind, tol=tol, maxit=a.maxit,
                                            raise_on_noconv=False)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        e = {"kappa": kap, "solve_ms": 1e3 * ts, "cg_iters": info["iters"],
             "line_search_steps": info["outer_iters"], "rel_res": info["true_rel_res"],
             "status": info["status"]}
        if kind == "cubic":
            e["uh_rel_l2_vs_exact"] = float(np.linalg.norm((uh.cpu().numpy() - wl.u_exact)[m]) /
                                            np.linalg.norm(wl.u_exact[m]))
        res[kind] = e
    pb.close()
    return res


def apply_loop(wl, chi, dirm, vol, dev, reps=20, warm=5, op="K"):
    """Standalone products of operator `op` (K, or M for the consistent mass):
    median over `reps` single launches (HIP events on the launch stream) after
    `warm` warm-ups, FP32 and FP64."""
    import numpy as np
    import torch

    from paper_2403_19854_amd import fcrkpm

    pb = fcrkpm.Problem(wl.dims, wl.h, wl.at, wl.degree, chi, dirm, vol, device=dev)
    x = torch.from_numpy(np.where(wl.free > 0, np.random.default_rng(0).standard_normal(wl.shape),
                                  0.0)).to(dev)
    res = {"reps": reps, "warmup": warm}
    st = torch.cuda.current_stream()
    for name, xt in (("f32", x.float()), ("f64", x)):
        y = torch.empty_like(xt)
        for _ in range(warm):
            pb.apply(op, xt, out=y, stream=st)
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            pb.apply(op, xt, out=y, stream=st)
            e1.record(st)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        med = float(np.median(ts))
        q1, q3 = (float(v) for v in np.percentile(ts, [25, 75]))
        res[name] = {"median_ms": med, "iqr_ms": [q1, q3], "matvecs_per_s": 1e3 / med}
    pb.close()
    return res


def gpu_clocks():
    """The GPU's current clocks as rocm-smi reports them (None where it is not
    available): read right after the timed region."""
    import subprocess
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True,
                           timeout=20)
        d = json.loads(r.stdout)
    except Exception:
        return None
    card = next(iter(d.values()), {}) if isinstance(d, dict) and d else {}
    if not isinstance(card, dict):
        return None
    clk = {k.rstrip(":").strip(): v for k, v in card.items() if "clk" in k.lower() or "clock" in k.lower()}
    return clk or None


def probe(a, wl):
    """A short run for counter collection (see paper_2403_19854_amd/traffic.py)."""
    import torch

    from paper_2403_19854_amd import fcrkpm

    dev = torch.device("cuda:0")
    pb = fcrkpm.Problem.from_workload(wl, device=dev)
    pb.set_graphs(False)
    # counter collection distorts setup's variant timing: measure the variant
    # an ordinary run picks (--probe-variant), where the box has it
    try:
        pb.set_option(fcrkpm.OPT_REGLAYOUT, a.probe_variant)
    except fcrkpm.FcrkpmError:
        pass
    layout = pb.get_option(fcrkpm.OPT_REGLAYOUT)
    r = torch.from_numpy(wl.r).to(dev)
    _, _, info = pb.solve(r, mode=a.mode, tol=1e-300, maxit=a.probe, want_uh=False,
                          raise_on_noconv=False)
    torch.cuda.synchronize()
    src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"probe": wl.name, "cg_iterations": info["iters"], "layout": layout,
                      "calibration_copy_bytes": 4 * src.numel()}), flush=True)
    pb.close()


def bench_table1(a, sizes=(8, 16, 32, 64, 128, 256), reps=20):
    """Per-operation times on the paper's timing problem (Eq 106 on [-1,1]^3,
    support 1.5h, linear basis) at the box sizes of its timing table: setup
    (moment convolutions, moment solves, the register path's records and the
    autotuner, wall time of the call), and medians over `reps` launches (HIP
    events) of K in FP64 and FP32, f^r and u^h in FP64."""
    import numpy as np
    import torch

    from paper_2403_19854_amd import fcrkpm
    from paper_2403_19854_amd import workloads as W

    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream()
    rows = []
    for n in sizes:
        wl = W.paper_shape(n)
        chi = torch.from_numpy(wl.chi).to(dev)
        dirm = torch.from_numpy(wl.dirichlet).to(dev)
        vol = torch.from_numpy(wl.vol).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pb = fcrkpm.Problem(wl.dims, wl.h, wl.at, wl.degree, chi, dirm, vol, device=dev)
        torch.cuda.synchronize()
        row = {"box": n, "omega_nodes": int(wl.chi.sum()), "setup_ms": 1e3 * (time.perf_counter() - t0)}
        x = torch.from_numpy(np.where(wl.chi > 0, np.random.default_rng(0).standard_normal(wl.shape),
                                      0.0)).to(dev)
        for name, op, xt in (("k_f64", "K_FULL", x), ("k_f32", "K_FULL", x.float()),
                             ("fr_f64", "FR", x), ("uh_f64", "UH", x)):
            y = torch.empty_like(xt)
            for _ in range(3):
                pb.apply(op, xt, out=y, stream=st)
            ts = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(st)
                pb.apply(op, xt, out=y, stream=st)
                e1.record(st)
                e1.synchronize()
                ts.append(e0.elapsed_time(e1))
            row[name + "_ms"] = float(np.median(ts))
        pb.close()
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    out = {"metric": "per-operation time vs box size, Eq 106 problem, support 1.5h (the paper's timing table)",
           "value": rows[-1]["k_f64_ms"], "unit": "ms (FP64 K at the largest box)", "n_gpus": 1,
           "higher_is_better": False, "data": "synthetic",
           "config": {"workload": "paper_eq106_table", "boxes": list(sizes), "reps": reps}, "rows": rows}
    print(json.dumps(out), flush=True)


def other_configs(a, dev):
    """Short runs of the other configurations beside the c5 line (each from its
    own setup, times of the solve calls): config 1 and 2 (FP64 CG to the bench
    tolerance), the paper's Eq 106 problem at 128^3 (refined), config 3 (500
    refined CG iterations, with the oracle's residual of the iterate), the
    config-4 batch (one step of 240 iterations, graphs) and config 5's problem
    on a 256^3 box (refined, to 1e-10)."""
    import numpy as np
    import torch

    import oracle
    from paper_2403_19854_amd import fcrkpm
    from paper_2403_19854_amd import workloads as W

    res = {}

    def solve(wl, mode, tol, maxit, fixed=False):
        pb = fcrkpm.Problem.from_workload(wl, device=dev)
        r = torch.from_numpy(wl.r).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d, uh, info = pb.solve(r, mode=mode, tol=1e-300 if fixed else tol, maxit=maxit,
                               raise_on_noconv=not fixed)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        pb.close()
        mv = info["matvecs_f32"] + info["matvecs_f64"]
        e = {"mode": mode, "solve_ms": 1e3 * ts, "iters": info["iters"], "matvecs_per_s": mv / ts,
             "true_rel_res": info["true_rel_res"]}
        if wl.u_exact is not None:
            m = wl.chi > 0
            e["uh_rel_l2_vs_exact"] = float(np.linalg.norm((uh.cpu().numpy() - wl.u_exact)[m]) /
                                            np.linalg.norm(wl.u_exact[m]))
        return e, d

    for name, wl, mode, tol in (("c1", W.config1(), "f64", a.tol), ("c2", W.config2(), "f64", a.tol),
                                ("paper_eq106_128", W.paper_shape(128), "f32_refined", a.tol)):
        res[name], _ = solve(wl, mode, tol, a.maxit)
    wl = W.config3()
    e, d = solve(wl, "f32_refined", a.tol, 500, fixed=True)
    o = oracle.Oracle(wl.dims, wl.h, wl.at, wl.degree, wl.chi, wl.vol)
    fr = np.where(wl.free > 0, o.apply_fr(wl.r), 0.0)
    e["oracle_rel_res"] = float(np.linalg.norm(np.where(wl.free > 0, fr - o.apply_k(d.cpu().numpy()), 0.0)) /
                                np.linalg.norm(fr))
    res["c3_500_iterations"] = e
    del o
    c4 = run_c4(a, dev, steps=1, warmup=1, direct=False)
    res["c4"] = {"node_matvecs_per_s": c4["value"], "ms_per_step": c4["ms_per_step"],
                 "cg_iterations": a.c4_iters}
    res["c5_256"], _ = solve(W.config5_256(), "f32_refined", 1e-10, a.maxit)
    return res


def run_c4(a, dev, steps, warmup, direct=True):
    """The config-4 batch: node-rhs K products/s with graphs (and with direct
    launches), and the ms per batched step."""
    import numpy as np
    import torch

    from paper_2403_19854_amd import fcrkpm
    from paper_2403_19854_amd import workloads as W

    probs = W.config4() + [W.config4_rhs_problem()]
    rs = [torch.from_numpy(p.r[None]).to(dev) for p in probs[:-1]]
    rs.append(torch.from_numpy(np.stack(W.config4_rhs(probs[-1]))).to(dev))
    libs = [fcrkpm.Problem.from_workload(p, device=dev) for p in probs]
    nrhs = [int(r.shape[0]) for r in rs]
    torch.cuda.synchronize()

    def run(graphs, steps):
        for g in libs:
            g.set_graphs(graphs)
        node_mv = 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out, st = fcrkpm.solve_batch(libs, rs, mode=a.mode, tol=a.tol, maxit=a.c4_iters,
                                         want_uh=False, raise_on_noconv=False)
            for p, k, (_, _, info) in zip(probs, nrhs, out):
                node_mv += sum(q["matvecs_f32"] + q["matvecs_f64"] for q in info["per_rhs"]) \
                    * float(np.prod(p.dims))
        torch.cuda.synchronize()
        return node_mv / (time.perf_counter() - t0), (time.perf_counter() - t0) / steps

    if warmup > 0:
        run(True, warmup)
    v_graph, t_graph = run(True, steps)
    res = {"value": v_graph, "ms_per_step": 1e3 * t_graph, "problems": len(probs),
           "boxes": [p.dims[0] for p in probs], "rhs": nrhs,
           "box_nodes_total": int(sum(np.prod(p.dims) * k for p, k in zip(probs, nrhs)))}
    if direct:
        v_direct, t_direct = run(False, steps)
        res["direct"] = (v_direct, t_direct)
    for g in libs:
        g.close()
    return res


def bench_c4(a):
    """Ragged batch: aggregate node-rhs matvecs/s of one batched solve."""
    import torch

    c = run_c4(a, torch.device("cuda:0"), a.steps, a.warmup)
    v_graph, t_graph = c["value"], c["ms_per_step"] / 1e3
    v_direct, t_direct = c["direct"]
    out = {
        "metric": "node-rhs K products/s of a ragged batched CG solve (C4)",
        "value": v_graph,
        "unit": "node-matvec/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * t_graph,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if a.mode == "f32_refined" else "f64",
        "data": "synthetic",
        "config": {"workload": "c4_ragged_batch", "problems": c["problems"],
                   "boxes": c["boxes"], "rhs": c["rhs"], "box_nodes_total": c["box_nodes_total"],
                   "cg_iterations": a.c4_iters, "mode": a.mode,
                   "step": "fcrkpm_solve_batch from zero: f^r, CG blocks, residuals (no setup)"},
        "direct_launches": {"value": v_direct, "ms_per_step": 1e3 * t_direct,
                            "graph_speedup": v_graph / v_direct},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
