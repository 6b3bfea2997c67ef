"""Moving hat sources (pe_set_moving_sources; the oscillating source of the
paper's Example 5.4, not separable in t and x) on the GPU against the FP64
oracle, through the C ABI.

Bars as for separable forcing: single propagations 1e-12 relative L2,
Parareal iterates 1e-11 (FP64), 2e-5 on the split-bf16 path.  Example 5.4
runs at the paper's size (N_x = 1024 elements, N x M = 4 x 16, 4
iterations) for its three (alpha, f, scheme) settings; the paper shows only
figures for it, so the oracle is the only reference.
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle.eife import Discretization
from oracle.parareal import fine_prop, parareal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pe():
    from paper_2412_01138_amd import peifem
    return peifem


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _hats(prob, axis):
    lo, hi = prob.lo[axis], prob.hi[axis]
    L = hi - lo
    others = tuple(wl.SpaceFactor(kappa=1.7 + a, phase=0.3) for a in range(prob.dim))
    return [wl.MovingHat(4.0, axis, 0.08 * L, lo + 0.5 * L, 0.4 * L, omega=2 * math.pi * 3.0,
                         phase=0.2, time=wl.TimeFactor(), space=others),
            wl.MovingHat(-1.5, axis, 0.15 * L, lo + 0.3 * L, 0.1 * L, omega=5.0,
                         time=wl.TimeFactor(alpha=-0.4), space=others)]


@pytest.mark.parametrize("dim,n,axis,transform,precision", [
    (1, (127,), 0, "dense", "fp64"),
    (1, (127,), 0, "fft", "fp64"),
    (2, (63, 100), 1, "dense", "fp64"),
    (3, (9, 20, 17), 0, "dense", "fp64"),
    (2, (37, 40), 0, "dense", "split_bf16"),
])
def test_moving_fine_propagate(dim, n, axis, transform, precision):
    pe = _pe()
    print(f"moving fine propagate dim {dim} n {n} axis {axis} {transform} {precision}", flush=True)
    prob = wl.tiny_problem(dim, n, seed=8, N=2, J=3, s=3, T=0.9, precision=precision)
    prob = prob.with_(moving=_hats(prob, axis))
    d = Discretization(prob)
    rng = np.random.default_rng(9)
    Uin = rng.normal(size=(prob.N,) + prob.n)
    g = pe.Grid.from_problem(prob, transform=transform)
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    dt = torch.float64 if precision == "fp64" else torch.float32
    U = torch.as_tensor(Uin, dtype=dt, device="cuda:0")
    out = g.fine_propagate(U, prob.t0, prob.dT, prob.J, prob.c_fine, E, B)
    tab = d.tables(prob.dt, prob.c_fine)
    ref = np.stack([fine_prop(d, Uin[k], prob.t0 + k * prob.dT, tab, prob.J)
                    for k in range(prob.N)])
    assert rel(out.double().cpu().numpy(), ref) <= (1e-12 if precision == "fp64" else 2e-5)


def test_moving_only_source():
    """Moving sources and no separable forcing (no pure-decay shortcut)."""
    pe = _pe()
    prob = wl.tiny_problem(2, (31, 20), seed=10, N=3, J=2, s=2, u0_modes=1)
    prob = prob.with_(forcing=[], moving=_hats(prob, 0))
    g, U, rep = pe.solve_problem(prob, K_max=3, tol=1e-10)
    d = Discretization(prob)
    r = parareal(d, d.initial(), prob.t0, prob.N, prob.J, d.tables(prob.dt, prob.c_fine),
                 d.tables(prob.dT, prob.c_coarse), K_max=3, tol=1e-10)
    assert rep.iterations == r.iterations
    assert rel(U.cpu().numpy(), r.iterates[-1]) <= 1e-11


@pytest.mark.parametrize("alpha,freq,sc,sf", [(0.01, 1.0, 2, 2), (0.01, 10.0, 2, 3),
                                              (0.1, 10.0, 3, 3)])
def test_example_5_4_full_size(alpha, freq, sc, sf):
    """Example 5.4 at the paper's size, PEIFE-linear{sc}{sf}, 4 iterations:
    every iterate's end state against the oracle's."""
    pe = _pe()
    prob = wl.example_5_4(alpha, freq, s_fine=sf, s_coarse=sc)
    print(f"example 5.4 alpha {alpha} f {freq} scheme {sc}{sf}, n {prob.n}", flush=True)
    d = Discretization(prob)
    r = parareal(d, d.initial(), prob.t0, prob.N, prob.J, d.tables(prob.dt, prob.c_fine),
                 d.tables(prob.dT, prob.c_coarse), K_max=4, tol=0.0)
    for K in (1, 4):
        g, U, rep = pe.solve_problem(prob, K_max=K, tol=0.0)
        assert rep.iterations == K
        err = rel(U.cpu().numpy(), r.iterates[K])
        print(f"  K = {K}: relative L2 error {err:.3e}")
        assert err <= 1e-11


def test_moving_source_arguments():
    pe = _pe()
    prob = wl.tiny_problem(2, (15, 12), seed=11)
    g = pe.Grid.from_problem(prob)
    good = _hats(prob, 0)
    for bad in (good[0].__class__(**{**good[0].__dict__, "axis": 2}),
                good[0].__class__(**{**good[0].__dict__, "width": 0.0})):
        with pytest.raises(pe.PeifemError):
            g.set_moving_sources([bad])
    with pytest.raises(pe.PeifemError):
        g.set_moving_sources(good * 9)          # 18 > PE_MAX_MOVING
    g.set_moving_sources(good)
    with pytest.raises(pe.PeifemError):
        g.learned_samples(prob.N, prob.t0, prob.dT)
