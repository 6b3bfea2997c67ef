#!/usr/bin/env python3
"""Benchmark of the PEIFE-linear hot path on one MI355X.

One step = one complete Parareal solve (paper Algorithm 1) of the 2D FP64
workload: 255 x 255 interior Q1 nodes on the unit square, D = 0.1, T = 2,
forcing = 8 separable sine modes with random wavenumbers, N(0,1) amplitudes
and cos(omega t) time factors (omega ~ U(1, 20)), u0 = 0, N = 64 slices,
J = 32 fine steps per slice, 3-stage ETD-RK with random nodes, stopping at a
1e-8 relative jump.  A step builds both phi tables, the coarse forcing and
sweep, and runs every fine pass (quadrature + per-axis DST on the matrix
cores + fused diagonal update) and correction sweep until the jump test
holds; inputs are resident in HBM before the timed region.

Reported value: fine DOF*stage updates per second over whole steps,
(fine passes per step) * DOF * N * J * q / seconds per step.

The second half of the metric, Parareal wall time to the 1e-8 jump with the
learned vs the plain coarse propagator, is measured on the 2D learned
workload (511 x 511 nodes, D = 0.01, T = 4, 12 sine modes with
omega ~ U(5, 50), N = 256, J = 32, 4-stage ETD-RK): the per-mode network is
first trained on the GPU by the library's own kernels (4096 seeded forcings
of that family on a 63 x 63 grid), then both solvers run to the jump
tolerance with F recomputed in every iteration.  Training is outside the
timed solves and reported separately.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fine DOF·stage updates/s + Parareal wall time to 1e-8 jump, learned vs plain G"
PEAK_FP64_TFLOPS = 78.6       # MI355X dense FP64 matrix peak
PEAK_HBM_GBS = 8000.0         # MI355X HBM3E


def workload_name(p):
    return (f"2D Q1 {p.n[0]}x{p.n[1]} interior nodes, D={p.D}, T={p.T}, "
            f"{len(p.forcing)} sine modes, N={p.N} slices x J={p.J} fine steps, "
            f"{p.q}-stage ETD-RK (random nodes), FP64, Parareal to {p.tol:g} relative jump")


# sources that define each timed kernel class (the counters are only valid
# for the code they were taken from)
KERNEL_SOURCES = {
    "dst_last": ("dst_f64.hip", "pe_internal.h"),
    "dst_mid": ("dst_f64.hip", "pe_internal.h"),
    "load": ("fine.hip", "pe_internal.h"),
    "update": ("fine.hip", "pe_internal.h"),
    "sweep": ("coarse.hip", "pe_internal.h"),
    "mid_update": ("fused_update.hip", "pe_internal.h"),
    # FFT transform kernels (the fft_transform comparison solve)
    "fft_gen": ("dst_fft.hip", "pe_internal.h"),
    "fft_final": ("dst_fft.hip", "pe_internal.h"),
}


def source_digest(kernel_class=None) -> str:
    """sha256 over the HIP sources of one kernel class (all sources when
    kernel_class is None) and the compiler flags."""
    import glob
    import hashlib
    from paper_2412_01138_amd import build_lib
    csrc = os.path.join(ROOT, "paper_2412_01138_amd", "csrc")
    if kernel_class is None:
        files = sorted(glob.glob(os.path.join(csrc, "*")))
    else:
        files = [os.path.join(csrc, f) for f in KERNEL_SOURCES[kernel_class]]
    h = hashlib.sha256()
    h.update(" ".join(f for f in build_lib.FLAGS if not os.path.isabs(f)).encode())
    for path in files:
        h.update(os.path.basename(path).encode())
        h.update(open(path, "rb").read())
    return h.hexdigest()


def measured_traffic(kernel_class):
    """HBM bytes per launch of a kernel class from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, scaled by the copy-kernel calibration;
    None when the summary is missing or the kernel's sources changed."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_2d255.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kernel_class)
    if not k or k.get("source_sha256") != source_digest(kernel_class):
        return None
    return k["bytes_per_launch"]


def cpu_baseline(prob, slices: int):
    """The FP64 oracle (as it stands) on the first `slices` slices of the same
    workload: both phi tables, the coarse sweep and every fine pass of
    Algorithm 1 until the same jump test holds."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle.eife import Discretization
    from oracle.parareal import parareal

    sub = prob.with_(N=slices, T=prob.dT * slices)
    t0 = time.perf_counter()
    d = Discretization(sub)
    tF = d.tables(sub.dt, sub.c_fine)
    tG = d.tables(sub.dT, sub.c_coarse)
    r = parareal(d, d.initial(), sub.t0, sub.N, sub.J, tF, tG, K_max=sub.K_max, tol=sub.tol)
    sec = time.perf_counter() - t0
    updates = r.iterations * sub.dof * sub.N * sub.J * sub.q
    threads = max([x.get("num_threads", 1) for x in threadpool_info()] or [1])
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": updates / sec, "unit": "fine DOF·stage updates/s", "cores": int(threads),
            "kind": "oracle",
            "sample": (f"oracle Parareal (phi tables, coarse sweep, {r.iterations} fine passes) on "
                       f"the first {slices} of {prob.N} slices, {sec:.1f} s, BLAS threads "
                       f"{threads}, host {cpu}, os.cpu_count()={os.cpu_count()}"),
            "seconds": sec}


def learned_vs_plain(forcings: int, steps: int, repeats: int = 3):
    """Train the coarse correction for the learned workload and time plain-G
    and learned-G Parareal solves to its tolerance."""
    import torch
    import workloads as wl
    from paper_2412_01138_amd import learned_g as lg

    prob = wl.config(4)
    t0 = time.perf_counter()
    X, T, S = lg.training_rows(prob, [10000 + i for i in range(forcings)], (63,) * prob.dim)
    W = lg.row_weights(X, S, prob.N, 0.0)
    torch.cuda.synchronize()
    t_rows = time.perf_counter() - t0
    t0 = time.perf_counter()
    mlp, _ = lg.train(X, T, steps, batch=16384, lr=2e-3, weights=W)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    res = lg.compare(prob, mlp, prob.tol, repeats=repeats)
    pl, le = res["plain"], res["learned"]
    return {
        "workload": (f"2D Q1 {prob.n[0]}x{prob.n[1]}, D={prob.D}, T={prob.T}, "
                     f"{len(prob.forcing)} sine modes omega~U(5,50), N={prob.N}, J={prob.J}, "
                     f"{prob.q}-stage ETD-RK, FP64 state and transforms, tol {prob.tol:g}"),
        "plain_G": pl, "learned_G": le,
        "wall_ms_to_tol_plain_G": pl["wall_ms"], "wall_ms_to_tol_learned_G": le["wall_ms"],
        "speedup": pl["wall_ms"] / le["wall_ms"],
        "answer_rel_diff": res["answer_rel_diff"],
        "training": {"forcings": forcings, "grid": [63] * prob.dim, "rows": int(X.shape[0]),
                     "steps": steps, "batch": 16384, "seconds_rows": t_rows,
                     "seconds_train": t_train,
                     "network": "12-64-64-64-1 GELU, bf16 weights, fp32 accumulation"},
    }


def split_workloads(repeats: int = 2):
    """Plain-G Parareal solves of the two 3D split-bf16 workloads (FP32 state,
    split-bf16 transforms, tol 1e-5): wall time, iterations, fine DOF*stage
    updates/s (whole solve), and the per-kernel HIP-event time."""
    import torch
    import workloads as wl
    from paper_2412_01138_amd import peifem

    out = {}
    for cfg in (3, 5):
        prob = wl.config(cfg)
        g = peifem.Grid.from_problem(prob)
        P = g.solve_params(prob.t0, prob.T, prob.N, prob.J, prob.c_coarse, prob.c_fine,
                           prob.K_max, prob.tol)
        work = g.workspace(g.solve_workspace_bytes(P))
        U = g.empty_states(prob.N + 1)
        g.parareal_solve(P, U=U, work=work)
        torch.cuda.synchronize()
        g.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(repeats):
            _, rep = g.parareal_solve(P, U=U, work=work)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / repeats
        stats = g.get_timing()
        g.set_timing(False)
        upd = rep.iterations * prob.dof * prob.N * prob.J * prob.q
        out[prob.name] = {
            "grid": list(prob.n), "N": prob.N, "J": prob.J, "q": prob.q, "tol": prob.tol,
            "iterations": rep.iterations, "jumps": [rep.jumps[i] for i in range(rep.iterations)],
            "ms_per_solve": ms, "fine_updates_per_s": upd / (ms / 1e3),
            "kernels_ms_per_launch": {k: v["ms"] / v["launches"] for k, v in stats.items()
                                      if v["launches"]},
            "kernels_GB_s": {k: v["bytes"] / v["ms"] / 1e6 for k, v in stats.items()
                             if v["launches"] and v["ms"] > 0},
        }
        del work, U, g
        torch.cuda.empty_cache()
    return out


def fft_transform(prob, U_dense, repeats: int):
    """The same solve with the FFT sine transform (pe_set_transform): wall time
    per solve, fine-pass rate, per-kernel HIP-event time, and the answer's
    distance from the dense-transform answer."""
    import torch
    from paper_2412_01138_amd import peifem

    g = peifem.Grid.from_problem(prob, transform="fft")
    P = g.solve_params(prob.t0, prob.T, prob.N, prob.J, prob.c_coarse, prob.c_fine,
                       prob.K_max, prob.tol)
    work = g.workspace(g.solve_workspace_bytes(P))
    U = g.empty_states(prob.N + 1)
    g.parareal_solve(P, U=U, work=work)
    torch.cuda.synchronize()
    g.set_timing(True)
    reports = []
    t0 = time.perf_counter()
    for _ in range(repeats):
        _, rep = g.parareal_solve(P, U=U, work=work)
        reports.append(rep)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / repeats
    stats = g.get_timing()
    g.set_timing(False)
    iters = reports[-1].iterations
    fine_updates = prob.dof * prob.N * prob.J * prob.q
    fine_ms = sum(r.ms_fine for r in reports) / len(reports) / max(iters, 1)
    diff = float(torch.linalg.vector_norm(U - U_dense) / torch.linalg.vector_norm(U_dense))
    out = {"ms_per_solve": ms, "iterations": iters,
           "fine_updates_per_s": iters * fine_updates / (ms / 1e3),
           "ms_fine_per_pass": fine_ms,
           "fine_pass_updates_per_s": fine_updates / (fine_ms / 1e3),
           "kernels_ms_per_launch": {k: v["ms"] / v["launches"] for k, v in stats.items()
                                     if v["launches"]},
           "kernels_TFLOP_s": {k: v["flops"] / v["ms"] / 1e9 for k, v in stats.items()
                               if v["launches"] and v["ms"] > 0},
           "kernels_GB_s": {k: v["bytes"] / v["ms"] / 1e6 for k, v in stats.items()
                            if v["launches"] and v["ms"] > 0},
           "answer_rel_diff_vs_dense": diff}
    del work, U, g
    torch.cuda.empty_cache()
    return out


def dirichlet_data(prob, repeats: int):
    """The bench solve with non-homogeneous Dirichlet data (two time-dependent
    separable data terms, pe_set_boundary): wall time per solve and fine-pass
    rate, beside the homogeneous solve."""
    import torch
    import workloads as wl
    from paper_2412_01138_amd import peifem

    P = wl.poly_factor
    data = [wl.Term(0.7, wl.TimeFactor(omega=2.0, phase=0.3),
                    (P(1.0, 0.5, -0.2), wl.SpaceFactor(kappa=1.3, phase=0.4))),
            wl.Term(-0.4, wl.TimeFactor(alpha=-0.5, poly=(1.0, 0.3, 0.0, 0.0)),
                    (wl.SpaceFactor(kappa=2.1, phase=0.2), P(0.3, 1.0)))]
    pb = prob.with_(boundary=data)
    g = peifem.Grid.from_problem(pb)
    U0 = g.project_state(pb.u0, pb.t0)
    P_ = g.solve_params(pb.t0, pb.T, pb.N, pb.J, pb.c_coarse, pb.c_fine, pb.K_max, pb.tol)
    work = g.workspace(g.solve_workspace_bytes(P_))
    U = g.empty_states(pb.N + 1)
    g.parareal_solve(P_, U0=U0, U=U, work=work)
    torch.cuda.synchronize()
    reports = []
    t0 = time.perf_counter()
    for _ in range(repeats):
        _, rep = g.parareal_solve(P_, U0=U0, U=U, work=work)
        reports.append(rep)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / repeats
    iters = reports[-1].iterations
    fine_updates = pb.dof * pb.N * pb.J * pb.q
    fine_ms = sum(r.ms_fine for r in reports) / len(reports) / max(iters, 1)
    out = {"data_terms": len(data), "forcing_terms_total": len(pb.forcing) + len(data) * 6,
           "ms_per_solve": ms, "iterations": iters, "converged": bool(reports[-1].converged),
           "fine_updates_per_s": iters * fine_updates / (ms / 1e3), "ms_fine_per_pass": fine_ms}
    del work, U, g
    torch.cuda.empty_cache()
    return out


def periodic_solve(prob, repeats: int):
    """Workload 2's forcing and slicing on a 256 x 256 grid periodic in both
    axes (pe_init_grid_periodic; FFT transform, separate update): wall time
    per solve and fine-pass rate."""
    import torch
    from paper_2412_01138_amd import peifem

    pb = prob.with_(n=(256, 256), periodic=(True, True))
    g = peifem.Grid.from_problem(pb)
    P = g.solve_params(pb.t0, pb.T, pb.N, pb.J, pb.c_coarse, pb.c_fine, pb.K_max, pb.tol)
    work = g.workspace(g.solve_workspace_bytes(P))
    U = g.empty_states(pb.N + 1)
    g.parareal_solve(P, U=U, work=work)
    torch.cuda.synchronize()
    g.set_timing(True)
    reports = []
    t0 = time.perf_counter()
    for _ in range(repeats):
        _, rep = g.parareal_solve(P, U=U, work=work)
        reports.append(rep)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / repeats
    stats = g.get_timing()
    g.set_timing(False)
    iters = reports[-1].iterations
    fine_updates = pb.dof * pb.N * pb.J * pb.q
    fine_ms = sum(r.ms_fine for r in reports) / len(reports) / max(iters, 1)
    out = {"grid": list(pb.n), "periodic": list(pb.periodic), "ms_per_solve": ms,
           "iterations": iters, "converged": bool(reports[-1].converged),
           "fine_updates_per_s": iters * fine_updates / (ms / 1e3), "ms_fine_per_pass": fine_ms,
           "kernels_ms_per_launch": {k: v["ms"] / v["launches"] for k, v in stats.items()
                                     if v["launches"]}}
    del work, U, g
    torch.cuda.empty_cache()
    return out


def example_5_4_runs(repeats: int = 3):
    """The paper's Example 5.4 (1D oscillating hat source, N_x = 1024, N x M =
    4 x 16, 4 Parareal iterations) for its three settings: wall time per solve
    (median of `repeats`) and the final jump."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2412_01138_amd import peifem

    out = {}
    for alpha, freq, sc, sf in ((0.01, 1.0, 2, 2), (0.01, 10.0, 2, 3), (0.1, 10.0, 3, 3)):
        prob = wl.example_5_4(alpha, freq, s_fine=sf, s_coarse=sc)
        g = peifem.Grid.from_problem(prob)
        U0 = g.project(prob.u0)
        P = g.solve_params(prob.t0, prob.T, prob.N, prob.J, prob.c_coarse, prob.c_fine, 4, 0.0)
        work = g.workspace(g.solve_workspace_bytes(P))
        U = g.empty_states(prob.N + 1)
        g.parareal_solve(P, U0=U0, U=U, work=work)
        times = []
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, rep = g.parareal_solve(P, U0=U0, U=U, work=work)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        out[f"PEIFE-linear{sc}{sf}, alpha={alpha:g}, f={freq:g}"] = {
            "ms_per_solve": float(np.median(times)), "iterations": rep.iterations,
            "jumps": [rep.jumps[i] for i in range(rep.iterations)]}
        del work, U, g
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slices", type=int, default=8)
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-vs-plain G comparison")
    ap.add_argument("--no-3d", action="store_true",
                    help="skip the 3D split-bf16 workloads")
    ap.add_argument("--no-fft", action="store_true",
                    help="skip the FFT-transform comparison solve")
    ap.add_argument("--only-3d", action="store_true",
                    help="run only the 3D split-bf16 workloads (profiling)")
    ap.add_argument("--learned-forcings", type=int, default=4096)
    ap.add_argument("--learned-steps", type=int, default=60000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the method shards by time slice; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as wl
    from paper_2412_01138_amd import peifem

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.only_3d:
        print(json.dumps({"split_bf16_workloads": split_workloads()}))
        return
    prob = wl.config(2)
    g = peifem.Grid.from_problem(prob)
    P = g.solve_params(prob.t0, prob.T, prob.N, prob.J, prob.c_coarse, prob.c_fine,
                       prob.K_max, prob.tol)
    nwork = g.solve_workspace_bytes(P)
    work = g.workspace(nwork)
    U = g.empty_states(prob.N + 1)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        g.parareal_solve(P, U=U, work=work)
    torch.cuda.synchronize()

    g.set_timing(True)
    reports = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, rep = g.parareal_solve(P, U=U, work=work)
        reports.append(rep)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    stats = g.get_timing()
    g.set_timing(False)

    ms_per_step = sec * 1e3 / args.steps
    iters = reports[-1].iterations
    fine_updates = prob.dof * prob.N * prob.J * prob.q
    value = iters * fine_updates / (ms_per_step / 1e3)
    fine_ms = sum(r.ms_fine for r in reports) / len(reports)

    # dominant kernel: the class with the largest total event time
    KERNEL_NAMES = {"dst_last": "k_pass_last2 (last-axis DST-I pass, two fold levels, "
                                "fused load quadrature)",
                    "dst_mid": "k_pass_mid2 (axis-0 DST-I pass, two fold levels)",
                    "mid_update": "k_final_update (axis-0 DST-I pass fused with the diagonal "
                                  "update)",
                    "load": "k_load_fields", "update": "k_update", "sweep": "k_sweep"}
    dom = max((k for k in stats if stats[k]["launches"]), key=lambda k: stats[k]["ms"])
    tr = stats[dom]
    avg_ms = tr["ms"] / max(tr["launches"], 1)
    flops_per_launch = tr["flops"] / max(tr["launches"], 1)
    bytes_per_launch = tr["bytes"] / max(tr["launches"], 1)
    kernels = {}
    for name, st in stats.items():
        if st["launches"] == 0:
            continue
        a_ms = st["ms"] / st["launches"]
        kernels[name] = {"launches": st["launches"], "avg_ms": a_ms,
                         "flops_per_launch": st["flops"] / st["launches"],
                         "bytes_per_launch": st["bytes"] / st["launches"],
                         "TFLOP/s": st["flops"] / st["launches"] / (a_ms / 1e3) / 1e12,
                         "GB/s": st["bytes"] / st["launches"] / (a_ms / 1e3) / 1e9}
    # the binding roof: matrix cores when the kernel's algorithmic intensity is
    # above the FP64 ridge (peak flops / peak bandwidth), HBM below it
    ridge = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
    intensity = flops_per_launch / bytes_per_launch if bytes_per_launch > 0 else float("inf")
    if tr["flops"] > 0 and intensity >= ridge:
        achieved = flops_per_launch / (avg_ms / 1e3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS}
    else:
        achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS}
    roof["intensity_flop_per_byte"] = intensity
    roof["ridge_flop_per_byte"] = ridge
    roof["achieved_TFLOP/s"] = flops_per_launch / (avg_ms / 1e3) / 1e12
    roof["traffic"] = measured_traffic(dom)
    roof.update({"kernel": KERNEL_NAMES[dom], "avg_launch_ms": avg_ms,
                 "flops_per_launch": flops_per_launch, "bytes_per_launch": bytes_per_launch,
                 "launches": tr["launches"]})

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "fine DOF·stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload_name(prob), "dof": prob.dof, "N": prob.N, "J": prob.J,
                   "q": prob.q, "tol": prob.tol, "seed": prob.seed},
        "parareal": {"iterations": iters, "converged": bool(reports[-1].converged),
                     "jumps": [reports[-1].jumps[i] for i in range(iters)],
                     "ms_tables": sum(r.ms_tables for r in reports) / len(reports),
                     "ms_coarse": sum(r.ms_coarse for r in reports) / len(reports),
                     "ms_fine_per_pass": fine_ms / max(iters, 1),
                     "ms_sweep": sum(r.ms_sweep for r in reports) / len(reports),
                     "fine_pass_updates_per_s": fine_updates / (fine_ms / max(iters, 1) / 1e3)},
        "roofline": roof,
        "kernels": kernels,
        "cpu_baseline": None,
        "source_sha256": source_digest(),
        "host": platform.node(),
    }
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    if not args.no_fft:
        out["fft_transform"] = fft_transform(prob, U, max(args.steps, 3))
    if not args.no_fft:
        out["dirichlet_data"] = dirichlet_data(prob, max(args.steps, 3))
        out["example_5_4"] = example_5_4_runs()
        out["periodic"] = periodic_solve(prob, max(args.steps, 3))
    if not args.no_learned:
        out["learned_vs_plain_G"] = learned_vs_plain(args.learned_forcings, args.learned_steps)
    if not args.no_3d:
        out["split_bf16_workloads"] = split_workloads()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_slices)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
