#!/usr/bin/env python3
"""Benchmark of the PEIFE-linear hot path on one MI355X.

One step = one complete Parareal solve (paper Algorithm 1) with the plain
coarse propagator of the 2D learned-G workload, the configuration the metric
is quoted on: 511 x 511 interior Q1 nodes on the unit square, D = 0.01,
T = 4, forcing = 12 separable sine modes with random wavenumbers, N(0,1)
amplitudes and cos(omega t) time factors (omega ~ U(5, 50)), u0 = 0,
N = 256 slices, J = 32 fine steps per slice, 4-stage ETD-RK with random
nodes, FP64 state and transforms, stopping at a 1e-8 relative jump.  A step
builds both phi tables, the coarse forcing and sweep, and runs every fine
pass (quadrature + per-axis DST on the matrix cores + fused diagonal
update) and correction sweep until the jump test holds; inputs are resident
in HBM before the timed region.

Reported value: fine DOF*stage updates per second over whole steps,
(fine passes per step) * DOF * N * J * q / seconds per step.

The second half of the metric, Parareal wall time to the 1e-8 jump with the
learned vs the plain coarse propagator, on the same workload: the per-mode
network is first trained on the GPU by the library's own kernels (4096
seeded forcings of that family on a 63 x 63 grid), then both solvers run to
the jump tolerance with F recomputed in every iteration (training outside
the timed solves, reported separately), and the learned solve is repeated
on 16 unseen forcings of the family.

Every solve's answer is compared with the FP64 oracle's sequential fine
solution (the answer Parareal converges to) on every forced mode plus 32
seeded random modes at every slice end; those oracle values are stored in
tests/golden/fullsize_modal_reference.json, written by a script that runs
only the oracle.  The oracle itself runs only in the cpu_baseline leg.
"""
import argparse
import glob
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fine DOF·stage updates/s + Parareal wall time to 1e-8 jump, learned vs plain G"
UNIT = "fine DOF·stage updates/s"
PEAK_FP64_TFLOPS = 78.6       # MI355X dense FP64 matrix peak
PEAK_BF16_TFLOPS = 2500.0     # MI355X dense bf16 matrix peak (split-bf16 products)
PEAK_HBM_GBS = 8000.0         # MI355X HBM3E

KERNEL_NAMES = {
    "dst_last": "last-axis DST-I pass with the fused load quadrature (generating pass; 3D "
                "split grids: fused with the middle-axis pass)",
    "dst_mid": "DST-I pass along another axis",
    "mid_update": "axis-0 DST-I pass fused with the diagonal update",
    "load": "separate load quadrature", "update": "separate diagonal update",
    "sweep": "coarse / correction sweep with the FP64 norms",
    "coarse_forcing": "coarse forcing r_n (all its kernels)",
}
# sources that define each timed kernel class (counters are only valid for
# the code they were taken from)
KERNEL_SOURCES = {
    "dst_last": ("dst_f64.hip", "dst_split.hip", "pe_internal.h"),
    "dst_mid": ("dst_f64.hip", "dst_split.hip", "pe_internal.h"),
    "load": ("fine.hip", "pe_internal.h"),
    "update": ("fine.hip", "pe_internal.h"),
    "sweep": ("coarse.hip", "pe_internal.h"),
    "mid_update": ("fused_update.hip", "pe_internal.h"),
    "coarse_forcing": ("dst_f64.hip", "dst_split.hip", "fused_update.hip", "fine.hip",
                       "pe_internal.h"),
}


def workload_name(p):
    return (f"{p.dim}D Q1 {'x'.join(map(str, p.n))} interior nodes, D={p.D}, T={p.T}, "
            f"{len(p.forcing)} sine modes, N={p.N} slices x J={p.J} fine steps, "
            f"{p.q}-stage ETD-RK (random nodes), "
            f"{'FP64' if p.precision == 'fp64' else 'split-bf16 transforms, FP32 state'}, "
            f"plain-G Parareal to {p.tol:g} relative jump")


def source_digest(kernel_class=None) -> str:
    """sha256 over the HIP sources of one kernel class (all sources when
    kernel_class is None) and the compiler flags."""
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


def measured_counters(tag, kernel_class):
    """Per-launch counter figures of a kernel class from the committed
    rocprofv3 summary profiles/counters_<tag>.json (HBM bytes from
    FETCH_SIZE / WRITE_SIZE scaled by the copy-kernel calibration, matrix-core
    figures from SQ_ counters); None when the summary is missing or the
    kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"counters_{tag}.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kernel_class)
    if not k or k.get("source_sha256") != source_digest(kernel_class):
        return None
    return k


# --------------------------------------------------------------------------
# error against the oracle (stored values)
# --------------------------------------------------------------------------

_REF = None


def oracle_error(cfg, U):
    """Relative L2 error of a solve's iterates U [N+1][...] against the
    oracle's sequential fine solution on the stored modes (all slice ends),
    and the norm outside the forced modes relative to the norm inside."""
    import numpy as np
    import torch
    global _REF
    if _REF is None:
        path = os.path.join(ROOT, "tests", "golden", "fullsize_modal_reference.json")
        _REF = json.load(open(path))["workloads"]
    rec = _REF[str(cfg)]
    flat = U.reshape(U.shape[0], -1)
    idx = torch.as_tensor(rec["flat_index"], device=U.device)
    got = flat[:, idx].double().cpu().numpy()
    ref = np.array([[float.fromhex(v) for v in row] for row in rec["W"]])
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    forced = torch.as_tensor(rec["forced_flat_index"], device=U.device)
    inside = float(torch.linalg.vector_norm(flat[:, forced].double()))
    rest = flat.double().clone()
    rest[:, forced] = 0
    outside = float(torch.linalg.vector_norm(rest))
    return {"rel_l2_vs_oracle": err, "sampled_modes": len(rec["flat_index"]),
            "slice_ends": len(rec["W"]), "outside_forced_rel": outside / max(inside, 1e-300)}


# --------------------------------------------------------------------------
# solves
# --------------------------------------------------------------------------

def timed_solves(g, P, steps, warmup, U0=None, timing=False):
    """`warmup` untimed then `steps` timed solves (synchronised around the
    timed region): (seconds, reports, kernel stats or None, final iterates)."""
    import torch
    work = g.workspace(g.solve_workspace_bytes(P))
    U = g.empty_states(P.N + 1)
    for _ in range(warmup):
        g.parareal_solve(P, U0=U0, U=U, work=work)
    torch.cuda.synchronize()
    if timing:
        g.set_timing(True)
    reports = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, rep = g.parareal_solve(P, U0=U0, U=U, work=work)
        reports.append(rep)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    stats = None
    if timing:
        stats = g.get_timing()
        g.set_timing(False)
    del work
    return sec, reports, stats, U


def report_summary(rep):
    k = rep.iterations
    return {"iterations": k, "converged": bool(rep.converged),
            "jumps": [rep.jumps[i] for i in range(k)],
            "residuals": [rep.residuals[i] for i in range(k)],
            "ms_tables": rep.ms_tables, "ms_coarse": rep.ms_coarse,
            "ms_fine_per_pass": rep.ms_fine / max(k, 1), "ms_sweep": rep.ms_sweep,
            "ms_learned": rep.ms_learned, "fallback": rep.fallback}


def kernel_table(stats):
    out = {}
    for name, st in stats.items():
        if st["launches"] == 0:
            continue
        a_ms = st["ms"] / st["launches"]
        out[name] = {"launches": st["launches"], "avg_ms": a_ms, "total_ms": st["ms"],
                     "flops_per_launch": st["flops"] / st["launches"],
                     "bytes_per_launch": st["bytes"] / st["launches"],
                     "TFLOP/s": st["flops"] / st["launches"] / (a_ms / 1e3) / 1e12,
                     "GB/s": st["bytes"] / st["launches"] / (a_ms / 1e3) / 1e9}
    return out


def roofline(stats, tag, peak_tflops=PEAK_FP64_TFLOPS):
    """The kernel class with the largest total event time, against the roof
    its algorithmic intensity puts it under."""
    dom = max((k for k in stats if stats[k]["launches"]), key=lambda k: stats[k]["ms"])
    tr = stats[dom]
    avg_ms = tr["ms"] / tr["launches"]
    flops = tr["flops"] / tr["launches"]
    nbytes = tr["bytes"] / tr["launches"]
    ridge = peak_tflops * 1e12 / (PEAK_HBM_GBS * 1e9)
    intensity = flops / nbytes if nbytes > 0 else float("inf")
    if flops > 0 and intensity >= ridge:
        achieved = flops / (avg_ms / 1e3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak_tflops, "unit": "TFLOP/s",
                "frac": achieved / peak_tflops}
    else:
        achieved = nbytes / (avg_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS}
    cnt = measured_counters(tag, dom)
    roof["traffic"] = cnt["bytes_per_launch"] if cnt else None
    roof.update({"kernel_class": dom, "kernel": (cnt or {}).get("kernel", KERNEL_NAMES[dom]),
                 "avg_launch_ms": avg_ms, "launches": tr["launches"],
                 "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": nbytes,
                 "intensity_flop_per_byte": intensity, "ridge_flop_per_byte": ridge,
                 "achieved_TFLOP/s": flops / (avg_ms / 1e3) / 1e12,
                 "achieved_GB/s": nbytes / (avg_ms / 1e3) / 1e9})
    if cnt and "mfma" in cnt:
        roof["mfma_counters"] = cnt["mfma"]
    return roof


def solve_entry(prob, cfg, steps, warmup, tag=None, mlp=None, fusion=True):
    """Timed plain- (or learned-) G solves of a workload with the kernel
    table and the error against the oracle (fusion=False: the generating
    and middle-axis passes of 3D split grids as two kernels)."""
    from paper_2412_01138_amd import peifem
    g = peifem.Grid.from_problem(prob)
    g.set_fusion(fusion)
    P = g.solve_params(prob.t0, prob.T, prob.N, prob.J, prob.c_coarse, prob.c_fine,
                       prob.K_max, prob.tol, None, mlp)
    sec, reports, stats, U = timed_solves(g, P, steps, warmup, timing=True)
    ms = sec * 1e3 / steps
    rep = reports[-1]
    upd = rep.iterations * prob.dof * prob.N * prob.J * prob.q
    out = {"workload": workload_name(prob), "ms_per_solve": ms,
           "fine_updates_per_s": upd / (ms / 1e3), **report_summary(rep),
           "kernels": kernel_table(stats), **oracle_error(cfg, U)}
    if tag:
        peak = PEAK_FP64_TFLOPS if prob.precision == "fp64" else PEAK_BF16_TFLOPS
        out["roofline"] = roofline(stats, tag, peak)
    del U, g
    return out


def learned_vs_plain(forcings, train_steps, repeats=3, validation=16):
    """Workload 4: train the coarse correction, time plain-G and learned-G
    solves to the tolerance, state both answers' error against the oracle,
    and repeat the learned solve on `validation` unseen forcings."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2412_01138_amd import learned_g as lg, peifem

    prob = wl.config(4)
    t0 = time.perf_counter()
    X, T, S = lg.training_rows(prob, [10000 + i for i in range(forcings)], (63,) * prob.dim)
    W = lg.row_weights(X, S, prob.N, 0.0)
    torch.cuda.synchronize()
    t_rows = time.perf_counter() - t0
    t0 = time.perf_counter()
    mlp, _ = lg.train(X, T, train_steps, batch=16384, lr=2e-3, weights=W)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    g = peifem.Grid.from_problem(prob)
    out = {"workload": workload_name(prob).replace("plain-G ", "")}
    for label, net in (("plain_G", None), ("learned_G", mlp)):
        P = g.solve_params(prob.t0, prob.T, prob.N, prob.J, prob.c_coarse, prob.c_fine,
                           prob.K_max, prob.tol, None, net)
        work = g.workspace(g.solve_workspace_bytes(P))
        U = g.empty_states(prob.N + 1)
        g.parareal_solve(P, U=U, work=work)
        times = []
        for _ in range(repeats):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, rep = g.parareal_solve(P, U=U, work=work)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t1) * 1e3)
        out[label] = {"wall_ms": float(np.median(times)), "wall_ms_all": times,
                      **report_summary(rep), **oracle_error(4, U)}
        out[label + "_U"] = U[-1].clone()
        del work, U
    u_plain, u_learn = out.pop("plain_G_U"), out.pop("learned_G_U")
    out["wall_ms_to_tol_plain_G"] = out["plain_G"]["wall_ms"]
    out["wall_ms_to_tol_learned_G"] = out["learned_G"]["wall_ms"]
    out["speedup"] = out["plain_G"]["wall_ms"] / out["learned_G"]["wall_ms"]
    # the two answers at T: the same converged solution up to rounding
    out["answer_rel_diff"] = float(torch.linalg.vector_norm(u_plain - u_learn) /
                                   torch.linalg.vector_norm(u_plain))
    out["training"] = {"forcings": forcings, "grid": [63] * prob.dim, "rows": int(X.shape[0]),
                       "steps": train_steps, "batch": 16384, "seconds_rows": t_rows,
                       "seconds_train": t_train,
                       "network": "12-64-64-64-1 GELU, bf16 weights, fp32 accumulation"}
    # unseen forcings of the family (seeds 20000 + i): one fine pass each
    fam = lg.WORKLOAD_FAMILY[4]
    j_learn, j_plain = [], []
    box = list(zip(prob.lo, prob.hi))
    for i in range(validation):
        g.set_forcing(wl.random_forcing(20000 + i, prob.dim, fam[0], box, fam[1], fam[2],
                                        kmax=fam[3]))
        for net, acc in ((mlp, j_learn), (None, j_plain)):
            P = g.solve_params(prob.t0, prob.T, prob.N, prob.J, prob.c_coarse, prob.c_fine, 1,
                               prob.tol, None, net)
            _, rep = g.parareal_solve(P)
            acc.append(rep.jumps[0])
    jl = np.array(j_learn)
    out["validation"] = {"forcings": validation, "seeds": f"20000..{20000 + validation - 1}",
                         "converged_in_one_pass": int(np.sum(jl <= prob.tol)),
                         "median_jump1_learned": float(np.median(jl)),
                         "max_jump1_learned": float(np.max(jl)),
                         "median_jump1_plain": float(np.median(j_plain)),
                         "jump1_learned": j_learn, "jump1_plain": j_plain}
    del g
    torch.cuda.empty_cache()
    return out


def split_workloads(steps, learned_forcings, learned_steps):
    """The two 3D split-bf16 workloads (FP32 state, split-bf16 transforms,
    tol 1e-5): plain-G solves, and learned vs plain G on the 255^3 one."""
    import torch
    import workloads as wl
    from paper_2412_01138_amd import learned_g as lg

    out = {}
    for cfg in (3, 5):
        prob = wl.config(cfg)
        out[prob.name] = solve_entry(prob, cfg, steps, 1, tag=f"w{cfg}")
        torch.cuda.empty_cache()
    # the same 255^3 solve with the generating and middle-axis passes as two
    # kernels (the axis-2 results through HBM)
    prob = wl.config(5)
    out[prob.name + " two-pass"] = solve_entry(prob, 5, steps, 1, fusion=False)
    torch.cuda.empty_cache()
    if learned_forcings > 0:
        prob = wl.config(5)
        t0 = time.perf_counter()
        X, T, S = lg.training_rows(prob, [10000 + i for i in range(learned_forcings)],
                                   (63,) * prob.dim)
        W = lg.row_weights(X, S, prob.N, 0.0)
        torch.cuda.synchronize()
        t_rows = time.perf_counter() - t0
        t0 = time.perf_counter()
        mlp, _ = lg.train(X, T, learned_steps, batch=16384, lr=2e-3, weights=W)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        del X, T, S, W
        le = solve_entry(prob, 5, steps, 1, mlp=mlp)
        le["training"] = {"forcings": learned_forcings, "grid": [63] * 3,
                          "steps": learned_steps, "seconds_rows": t_rows,
                          "seconds_train": t_train}
        out[prob.name + " learned_G"] = le
        pl = out[prob.name]
        out[prob.name + " learned_vs_plain"] = {
            "wall_ms_plain_G": pl["ms_per_solve"], "wall_ms_learned_G": le["ms_per_solve"],
            "iterations_plain_G": pl["iterations"], "iterations_learned_G": le["iterations"],
            "speedup": pl["ms_per_solve"] / le["ms_per_solve"]}
        torch.cuda.empty_cache()
    return out


def fft_transform(prob, repeats):
    """Workload 2 with the FFT sine transform (pe_set_transform)."""
    import torch
    from paper_2412_01138_amd import peifem
    g = peifem.Grid.from_problem(prob, transform="fft")
    P = g.solve_params(prob.t0, prob.T, prob.N, prob.J, prob.c_coarse, prob.c_fine,
                       prob.K_max, prob.tol)
    sec, reports, stats, U = timed_solves(g, P, repeats, 1, timing=True)
    ms = sec * 1e3 / repeats
    rep = reports[-1]
    out = {"ms_per_solve": ms, **report_summary(rep),
           "fine_updates_per_s": rep.iterations * prob.dof * prob.N * prob.J * prob.q / (ms / 1e3),
           "kernels": kernel_table(stats), **oracle_error(2, U)}
    del U, g
    torch.cuda.empty_cache()
    return out


def dirichlet_data(prob, repeats):
    """Workload 2 with non-homogeneous Dirichlet data (two time-dependent
    separable data terms, pe_set_boundary)."""
    import torch
    import workloads as wl
    from paper_2412_01138_amd import peifem
    P_ = wl.poly_factor
    data = [wl.Term(0.7, wl.TimeFactor(omega=2.0, phase=0.3),
                    (P_(1.0, 0.5, -0.2), wl.SpaceFactor(kappa=1.3, phase=0.4))),
            wl.Term(-0.4, wl.TimeFactor(alpha=-0.5, poly=(1.0, 0.3, 0.0, 0.0)),
                    (wl.SpaceFactor(kappa=2.1, phase=0.2), P_(0.3, 1.0)))]
    pb = prob.with_(boundary=data)
    g = peifem.Grid.from_problem(pb)
    U0 = g.project_state(pb.u0, pb.t0)
    P = g.solve_params(pb.t0, pb.T, pb.N, pb.J, pb.c_coarse, pb.c_fine, pb.K_max, pb.tol)
    sec, reports, _, U = timed_solves(g, P, repeats, 1, U0=U0)
    ms = sec * 1e3 / repeats
    rep = reports[-1]
    out = {"data_terms": len(data), "forcing_terms_total": len(pb.forcing) + len(data) * 6,
           "ms_per_solve": ms, **report_summary(rep),
           "fine_updates_per_s": rep.iterations * pb.dof * pb.N * pb.J * pb.q / (ms / 1e3),
           "error_vs_oracle": "tests/test_gpu_boundary.py (full size, slices 1-2: 1.1e-12)"}
    del U, g
    torch.cuda.empty_cache()
    return out


def periodic_solve(prob, repeats):
    """Workload 2's forcing and slicing on a 256 x 256 grid periodic in both
    axes (pe_init_grid_periodic; FFT transform)."""
    import torch
    from paper_2412_01138_amd import peifem
    pb = prob.with_(n=(256, 256), periodic=(True, True))
    g = peifem.Grid.from_problem(pb)
    P = g.solve_params(pb.t0, pb.T, pb.N, pb.J, pb.c_coarse, pb.c_fine, pb.K_max, pb.tol)
    sec, reports, stats, U = timed_solves(g, P, repeats, 1, timing=True)
    ms = sec * 1e3 / repeats
    rep = reports[-1]
    out = {"grid": list(pb.n), "periodic": list(pb.periodic), "ms_per_solve": ms,
           **report_summary(rep),
           "fine_updates_per_s": rep.iterations * pb.dof * pb.N * pb.J * pb.q / (ms / 1e3),
           "kernels": kernel_table(stats),
           "error_vs_oracle": "tests/test_gpu_periodic.py (full size, slices 1-2: 2.2e-13)"}
    del U, g
    torch.cuda.empty_cache()
    return out


def example_5_4_runs(repeats=3):
    """The paper's Example 5.4 (1D oscillating hat source, N_x = 1024,
    N x M = 4 x 16, 4 Parareal iterations) for its three settings."""
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
            "ms_per_solve": float(np.median(times)), **report_summary(rep),
            "error_vs_oracle": "tests/test_gpu_moving.py (iterates 1 and 4: 2.4-4.0e-12)"}
        del work, U, g
    return out


def cpu_baseline(prob, slices):
    """The FP64 oracle as it stands, on the host cores: its fine propagator
    F^J (J steps of eq. (2.6): load quadrature, dense LAPACK-basis mode
    products, diagonal update) on the first `slices` slices of the workload.
    The oracle's fine phi table (mpmath, one value per distinct z) is built
    first and timed separately: it is a one-off cost of a solve."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle.eife import Discretization
    from oracle.parareal import fine_prop

    t0 = time.perf_counter()
    d = Discretization(prob)
    tF = d.tables(prob.dt, prob.c_fine)
    t_tab = time.perf_counter() - t0
    W = np.zeros(prob.n)
    t0 = time.perf_counter()
    for n in range(slices):
        fine_prop(d, W, prob.t0 + n * prob.dT, tF, prob.J)
    sec = time.perf_counter() - t0
    updates = slices * prob.dof * prob.J * prob.q
    threads = max([x.get("num_threads", 1) for x in threadpool_info()] or [1])
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": updates / sec, "unit": UNIT, "cores": int(threads), "kind": "oracle",
            "sample": (f"oracle fine propagator F^J (J={prob.J} steps x {prob.q} stages) on the "
                       f"first {slices} of {prob.N} slices of the {prob.n[0]}x{prob.n[1]} "
                       f"workload, {sec:.1f} s; its fine phi table ({np.unique(d.lam).size} "
                       f"distinct z, mpmath) took {t_tab:.1f} s before the timed region; BLAS "
                       f"threads {threads}, host {cpu}, os.cpu_count()={os.cpu_count()}"),
            "seconds": sec, "seconds_phi_table": t_tab}


def progress(msg):
    """One line per finished leg, on stderr (stdout carries the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--only-headline", action="store_true",
                    help="time the headline solve only (profiling)")
    ap.add_argument("--only-3d", action="store_true",
                    help="run only the 3D split-bf16 plain-G solves (profiling)")
    ap.add_argument("--only-2d255", action="store_true",
                    help="run only the 255 x 255 FP64 solve (profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slices", type=int, default=4)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FFT, Dirichlet, periodic and Example 5.4 solves")
    ap.add_argument("--learned-forcings", type=int, default=4096)
    ap.add_argument("--learned-steps", type=int, default=300000)
    ap.add_argument("--learned3d-forcings", type=int, default=1024)
    ap.add_argument("--learned3d-steps", type=int, default=40000)
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
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.only_3d:
        print(json.dumps(split_workloads(max(args.steps, 1), 0, 0)))
        return
    if args.only_2d255:
        print(json.dumps(solve_entry(wl.config(2), 2, args.steps, args.warmup, tag="w2")))
        return

    prob = wl.config(4)
    g = peifem.Grid.from_problem(prob)
    P = g.solve_params(prob.t0, prob.T, prob.N, prob.J, prob.c_coarse, prob.c_fine,
                       prob.K_max, prob.tol)
    sec, reports, stats, U = timed_solves(g, P, args.steps, args.warmup, timing=True)
    ms_per_step = sec * 1e3 / args.steps
    rep = reports[-1]
    fine_updates = prob.dof * prob.N * prob.J * prob.q
    value = rep.iterations * fine_updates / (ms_per_step / 1e3)
    err = oracle_error(4, U)
    del U, g
    torch.cuda.empty_cache()
    progress(f"headline: {ms_per_step:.2f} ms per solve, {rep.iterations} fine passes, "
             f"error vs oracle {err['rel_l2_vs_oracle']:.2e}")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload_name(prob), "dof": prob.dof, "N": prob.N,
                   "J": prob.J, "q": prob.q, "tol": prob.tol, "seed": prob.seed},
        "parareal": {**report_summary(rep),
                     "fine_pass_updates_per_s": fine_updates /
                     (sum(r.ms_fine for r in reports) / len(reports) / rep.iterations / 1e3)},
        "error_vs_oracle": err,
        "roofline": roofline(stats, "w4"),
        "kernels": kernel_table(stats),
        "cpu_baseline": None,
        "source_sha256": source_digest(),
        "host": platform.node(),
    }
    if not args.only_headline:
        if not args.no_learned:
            out["learned_vs_plain_G"] = learned_vs_plain(args.learned_forcings,
                                                         args.learned_steps)
            lv = out["learned_vs_plain_G"]
            progress(f"learned vs plain G: {lv['wall_ms_to_tol_plain_G']:.1f} -> "
                     f"{lv['wall_ms_to_tol_learned_G']:.1f} ms, validation "
                     f"{lv['validation']['converged_in_one_pass']}/{lv['validation']['forcings']}")
        out["fp64_255x255"] = solve_entry(wl.config(2), 2, max(args.steps, 5), 2, tag="w2")
        progress(f"255x255: {out['fp64_255x255']['ms_per_solve']:.2f} ms per solve")
        if not args.no_extras:
            p2 = wl.config(2)
            out["fft_transform_255x255"] = fft_transform(p2, max(args.steps, 3))
            out["dirichlet_data_255x255"] = dirichlet_data(p2, max(args.steps, 3))
            out["periodic_256x256"] = periodic_solve(p2, max(args.steps, 3))
            out["example_5_4"] = example_5_4_runs()
            progress("FFT, Dirichlet, periodic and Example 5.4 solves done")
        if not args.no_3d:
            out["split_bf16_workloads"] = split_workloads(
                2, 0 if args.no_learned else args.learned3d_forcings, args.learned3d_steps)
            progress("3D split-bf16 workloads done")
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(prob, args.cpu_slices)
            progress(f"cpu baseline: {out['cpu_baseline']['value']:.3e} updates/s")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
