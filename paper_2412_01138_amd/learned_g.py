"""Training and evaluation driver of the learned coarse correction.

Everything numerical runs in the library (libpeifem): the fine and coarse
forcing responses F^J(0), G(0), the training rows (network inputs from the
forcing's term spectra and time factors), the BF16-MFMA training steps and
the corrected Parareal solve.  This module only
sequences those calls.

Training data: for each seeded forcing of the workload's family, on a grid of
the same box, D, slicing and stage nodes (possibly coarser than the target
grid: the per-mode map depends only on z = D lambda dT and the slice's time
signal, and forced wavenumbers up to 32 are resolved by 63 nodes per axis),
the rows (x, (R - r) / (s dT)) of every forced (slice, mode), s the size of
the forcing samples' part of degree >= 4.

    python -m paper_2412_01138_amd.learned_g --workload 4 --forcings 512 --out w.npy
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from typing import Optional, Sequence

import numpy as np

from . import peifem

WORKLOAD_FAMILY = {
    # workload: (modes, omega_lo, omega_hi, largest wavenumber)
    4: (12, 5.0, 50.0, 32),
    5: (24, 2.0, 40.0, 32),
    2: (8, 1.0, 20.0, 32),
    3: (16, 1.0, 20.0, 32),
}


def init_params(seed: int) -> np.ndarray:
    """Scaled-normal initial weights (zero biases), W[in][out] layout."""
    rng = np.random.default_rng(seed)
    shapes = [(12, 64), (64,), (64, 64), (64,), (64, 64), (64,), (64,), (1,)]
    parts = []
    for shp in shapes:
        if len(shp) == 2:
            parts.append(rng.normal(size=shp) / math.sqrt(shp[0]))
        elif shp == (64,) and len(parts) == 6:
            parts.append(rng.normal(size=shp) / 8.0)      # output weights w4
        else:
            parts.append(np.zeros(shp))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def training_rows(template, seeds: Sequence[int], grid_n: Optional[Sequence[int]] = None,
                  rel_thresh: float = 1e-9, log=None, family=None, precision: str = "fp64"):
    """Rows (x, target, s) on `template`'s box/slicing for each forcing seed;
    family = (modes, omega_lo, omega_hi, largest wavenumber) of the seeded
    sine-mode forcings (default: the workload's own).  The responses are
    computed at `precision` (FP64 by default: the targets are differences of
    two responses, which an FP32 state would resolve only coarsely)."""
    import torch
    import workloads as wl
    if family is None:
        family = WORKLOAD_FAMILY.get(_workload_id(template), (12, 5.0, 50.0, 32))
    modes, wlo, whi, kmax = family
    prob = template.with_(precision=precision)
    if grid_n is not None:
        prob = prob.with_(n=tuple(grid_n))
    g = peifem.Grid(prob.n, prob.lo, prob.hi, prob.D, prob.precision)
    EF, BF = g.phi_tables(prob.dt, prob.c_fine)
    EG, BG = g.phi_tables(prob.dT, prob.c_coarse)
    zero = g.empty_states(prob.N).zero_()
    fwork = g.workspace(g.fine_workspace_bytes(prob.N * prob.J * prob.q))
    R = g.empty_states(prob.N)
    r = g.empty_states(prob.N)
    U = g.empty_states(prob.N + 1).zero_()
    cwork = g.workspace(g.L.pe_coarse_workspace_bytes(g.h, prob.N, prob.p))
    xs, ts, ss = [], [], []
    t0 = time.perf_counter()
    for i, seed in enumerate(seeds):
        terms = wl.random_forcing(seed, prob.dim, modes, list(zip(prob.lo, prob.hi)), wlo, whi,
                                  kmax=kmax)
        g.set_forcing(terms)
        g.fine_propagate(zero, prob.t0, prob.dT, prob.J, prob.c_fine, EF, BF, Uout=R, work=fwork)
        g.coarse_sweep(U, prob.t0, prob.dT, prob.c_coarse, EG, BG, r, work=cwork)
        x, t, sc, _ = g.learned_rows(R, r, prob.t0, prob.dT, rel_thresh=rel_thresh,
                                     max_rows=prob.N * modes * 2, want_scale=True)
        xs.append(x.clone())
        ts.append(t.clone())
        ss.append(sc.clone())
        if log and (i + 1) % max(1, len(seeds) // 16) == 0:
            log(f"  rows: {i + 1}/{len(seeds)} forcings, {sum(len(q) for q in ts)} rows, "
                f"{time.perf_counter() - t0:.1f} s")
    return torch.cat(xs), torch.cat(ts), torch.cat(ss)


def row_weights(X, S, n_slices: int, power: float = 1.0):
    """Importance of a row for the coarse error: the size s of its correction
    times the number of slices over which a coarse error of that mode
    persists, min(N, 1 / (1 - e^{-z})) (z = exp(8 x_0)), to the given power
    for the gain."""
    import torch
    z = torch.exp(8.0 * X[:, 0].double())
    persist = torch.clamp(1.0 / (-torch.expm1(-z)), max=float(n_slices))
    return (S.double() * persist ** power) ** 2


def _wrms(y, t, w):
    d = (y.double() - t.double()) ** 2
    return float(((w * d).sum() / (w * t.double() ** 2).sum().clamp_min(1e-300)).sqrt())


def _workload_id(prob) -> int:
    name = getattr(prob, "name", "")
    return int(name[3]) if name.startswith("cfg") and name[3].isdigit() else 4


def train(X, T, steps: int, batch: int = 16384, lr: float = 2e-3, seed: int = 0, log=None,
          X_val=None, T_val=None, weights=None, W_val=None):
    """Adam on mini-batches with a cosine learning-rate schedule.  Batches are
    drawn with probability proportional to `weights` when given (the loss is
    then the weighted mean squared error), else by reshuffled passes."""
    import torch
    m = peifem.Mlp(init_params(seed))
    n = X.shape[0]
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    cdf = None
    if weights is not None:
        cdf = torch.cumsum(weights.double(), 0)
        cdf = (cdf / cdf[-1]).float()
    perm = torch.randperm(n, device=X.device, generator=gen)
    pos = 0
    hist = []
    Xe = X_val if X_val is not None else X[:65536]
    Te = T_val if T_val is not None else T[:65536]
    We = W_val if W_val is not None else (weights[:65536] if weights is not None else None)
    for step in range(steps):
        if cdf is not None:
            u = torch.rand(batch, device=X.device, generator=gen)
            idx = torch.clamp(torch.searchsorted(cdf, u), max=n - 1)
        else:
            if pos + batch > n:
                perm = torch.randperm(n, device=X.device, generator=gen)
                pos = 0
            idx = perm[pos:pos + batch]
            pos += batch
        rate = lr * 0.5 * (1.0 + math.cos(math.pi * step / steps))
        m.train_step(X[idx].contiguous(), T[idx].contiguous(), lr=rate)
        if log and (step + 1) % max(1, steps // 10) == 0:
            y = m.forward(Xe)
            rms = _wrms(y, Te, torch.ones_like(Te, dtype=torch.float64))
            wrms = _wrms(y, Te, We) if We is not None else rms
            hist.append((step + 1, rms, wrms))
            log(f"  step {step + 1}/{steps}: relative rms {rms:.3e}, weighted {wrms:.3e}")
    return m, hist


def compare(prob, mlp, tol: float, K_max: int = 8, repeats: int = 3):
    """Plain-G vs learned-G Parareal on `prob`: iterations, jumps and wall time
    (median of `repeats` full solves each, after one warm-up)."""
    import torch
    g = peifem.Grid.from_problem(prob)
    U0 = g.project(prob.u0) if prob.u0 else None
    out = {}
    for label, net in (("plain", None), ("learned", mlp)):
        P = g.solve_params(prob.t0, prob.T, prob.N, prob.J, prob.c_coarse, prob.c_fine, K_max, tol,
                           None, net)
        work = g.workspace(g.solve_workspace_bytes(P))
        U = g.empty_states(prob.N + 1)
        g.parareal_solve(P, U0=U0, U=U, work=work)
        times, rep = [], None
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, rep = g.parareal_solve(P, U0=U0, U=U, work=work)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        out[label] = {"iterations": rep.iterations, "converged": bool(rep.converged),
                      "jumps": [rep.jumps[i] for i in range(rep.iterations)],
                      "wall_ms": float(np.median(times)), "ms_learned": rep.ms_learned,
                      "fallback": rep.fallback, "U_last": U[-1].double().cpu().numpy()}
        del work
    d = out["plain"]["U_last"] - out["learned"]["U_last"]
    out["answer_rel_diff"] = float(np.linalg.norm(d) / max(np.linalg.norm(out["plain"]["U_last"]), 1e-300))
    for k in ("plain", "learned"):
        del out[k]["U_last"]
    return out


def main(argv=None):
    import torch
    import workloads as wl
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", type=int, default=4)
    ap.add_argument("--forcings", type=int, default=512)
    ap.add_argument("--grid", type=int, default=63, help="training grid nodes per axis")
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--weight-power", type=float, default=1.0,
                    help="persistence exponent of the row weights; negative: uniform rows")
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--eval-n", type=int, default=None, help="evaluation grid (default: full)")
    ap.add_argument("--out", type=str, default=None)
    ap.add_argument("--json", type=str, default=None)
    args = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    prob = wl.config(args.workload)
    tol = prob.tol if args.tol is None else args.tol
    train_seeds = [10000 + i for i in range(args.forcings)]
    val_seeds = [20000 + i for i in range(max(8, args.forcings // 16))]
    log(f"training rows on {args.grid}^{prob.dim} for {len(train_seeds)} forcings")
    t0 = time.perf_counter()
    X, T, S = training_rows(prob, train_seeds, (args.grid,) * prob.dim, log=log)
    Xv, Tv, Sv = training_rows(prob, val_seeds, (args.grid,) * prob.dim)
    W = Wv = None
    if args.weight_power >= 0:
        W = row_weights(X, S, prob.N, args.weight_power)
        Wv = row_weights(Xv, Sv, prob.N, args.weight_power)
    t_rows = time.perf_counter() - t0
    log(f"{X.shape[0]} training rows, {Xv.shape[0]} validation rows, {t_rows:.1f} s")
    t0 = time.perf_counter()
    mlp, hist = train(X, T, args.steps, args.batch, args.lr, log=log, X_val=Xv, T_val=Tv,
                      weights=W, W_val=Wv)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    if args.out:
        np.save(args.out, mlp.get_params())
    eval_prob = prob if args.eval_n is None else prob.with_(n=(args.eval_n,) * prob.dim)
    res = compare(eval_prob, mlp, tol)
    res.update({"workload": args.workload, "train_grid": args.grid, "forcings": args.forcings,
                "rows": int(X.shape[0]), "steps": args.steps, "seconds_rows": t_rows,
                "seconds_train": t_train, "history": hist, "tol": tol,
                "weight_power": args.weight_power,
                "eval_grid": list(eval_prob.n)})
    log(json.dumps(res))
    if args.json:
        json.dump(res, open(args.json, "w"), indent=1)


if __name__ == "__main__":
    main()
