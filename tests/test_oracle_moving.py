"""Pins of the oracle's moving hat source (the oscillating source of the
paper's Example 5.4; oracle/forcing.py hat_load_1d, load_moving):

* when the hat's kinks sit on nodes the hat is a Q1 function, so its exact
  Galerkin load is the full-grid mass matrix times its nodal values, and the
  q-point Gauss rule (exact for the piecewise quadratic integrand) must
  reproduce that, at two times of the oscillation;
* with kinks inside elements the rule converges to the exact integral
  (computed here piece by piece between the kinks) as q grows;
* a hat that does not move, with a constant amplitude, is a constant
  forcing: the ETD-RK solution equals the exact semi-discrete solution from
  scipy's expm of a system assembled in this test;
* in 2D the load of a hat along one axis times a factor on the other is the
  outer product of the two 1D loads (a literal 2D element loop checks it).
"""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg

import workloads as wl
from oracle.eife import Discretization, sequential
from oracle.fem import gauss_legendre_01
from oracle.forcing import hat_load_1d, load_moving, space_factor


def _full_mass(n, lo, hi):
    h = (hi - lo) / (n + 1)
    m = n + 2
    M = np.diag(np.full(m, 4.0 * h / 6.0)) + np.diag(np.full(m - 1, h / 6.0), 1) \
        + np.diag(np.full(m - 1, h / 6.0), -1)
    M[0, 0] = M[-1, -1] = 2.0 * h / 6.0
    return M


def _hat_nodal(c, w, xs):
    return np.maximum(1.0 - np.abs(xs - c) / w, 0.0)


def test_aligned_hat_load_is_mass_times_nodal_values():
    n, lo, hi = 39, 0.0, 2.0                     # h = 0.05
    h = (hi - lo) / (n + 1)
    hat = wl.MovingHat(3.0, 0, 2 * h, 1.0, 6 * h, omega=2.5, phase=0.0)
    xs = lo + h * np.arange(n + 2)
    M = _full_mass(n, lo, hi)
    for t in (0.0, (math.pi / 2) / 2.5):         # centre on node 20, then node 26
        c = hat.c0 + hat.c1 * math.sin(hat.omega * t)
        exact = (M @ _hat_nodal(c, hat.width, xs))[1:-1]
        got = hat_load_1d(hat, t, n, lo, hi, 3)
        assert np.max(np.abs(got - exact)) <= 1e-15
        assert abs(got.sum() - hat.width) <= 1e-14   # area of the unit hat


def _exact_hat_load(c, w, n, lo, hi):
    """int hat(x) phi_j(x) dx exactly: both factors are linear between the
    breakpoints (nodes and kinks), so a 2-point rule per piece is exact."""
    h = (hi - lo) / (n + 1)
    xs = lo + h * np.arange(n + 2)
    xg, wg = gauss_legendre_01(2)
    C = np.zeros(n)
    for j in range(1, n + 1):
        for a, b in ((xs[j - 1], xs[j]), (xs[j], xs[j + 1])):
            cuts = sorted({a, b, *[k for k in (c - w, c, c + w) if a < k < b]})
            for p, r in zip(cuts[:-1], cuts[1:]):
                x = p + (r - p) * xg
                phi = np.maximum(1.0 - np.abs(x - xs[j]) / h, 0.0)
                C[j - 1] += (r - p) * np.sum(wg * _hat_nodal(c, w, x) * phi)
    return C


def test_unaligned_hat_load_converges_to_the_exact_integral():
    n, lo, hi = 30, 0.0, 1.0
    hat = wl.MovingHat(1.0, 0, 0.05, 0.5, 0.45, omega=2 * math.pi * 10)
    t = 0.0123
    c = hat.c0 + hat.c1 * math.sin(hat.omega * t)
    exact = _exact_hat_load(c, hat.width, n, lo, hi)
    errs = [np.max(np.abs(hat_load_1d(hat, t, n, lo, hi, q) - exact)) for q in (3, 8, 20)]
    scale = np.max(np.abs(exact))
    assert errs[0] > 1e-6 * scale            # the kinks make q = 3 inexact ...
    assert errs[2] < errs[1] < errs[0]       # ... and a finer rule closes in
    assert errs[2] <= 1e-3 * scale


def test_standing_hat_matches_matrix_exponential():
    n, lo, hi = 9, 0.0, 1.0
    h = (hi - lo) / (n + 1)
    hat = wl.MovingHat(2.0, 0, 2 * h, 0.4, 0.0)          # kinks on nodes, at rest
    prob = wl.Problem("standing-hat", 1, (n,), (lo,), (hi,), 0.3, 0.0, 0.8, [], [], 1, 6,
                      (0.0, 0.6), (0.0, 0.6), moving=[hat])
    d = Discretization(prob)
    W = sequential(d, d.initial(), 0.0, d.tables(prob.dt, prob.c_fine), prob.J)
    U = d.grid.to_nodal(W)
    Mf = _full_mass(n, lo, hi)
    M = Mf[1:-1, 1:-1]
    A = (np.diag(np.full(n, 2.0)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)) / h
    F = hat.amp * (Mf @ _hat_nodal(hat.c0, hat.width, lo + h * np.arange(n + 2)))[1:-1]
    Uinf = np.linalg.solve(prob.D * A, F)
    Ut = Uinf + scipy.linalg.expm(-prob.T * prob.D * np.linalg.solve(M, A)) @ (0 - Uinf)
    assert np.max(np.abs(U - Ut)) <= 1e-12 * np.max(np.abs(Ut))


def test_2d_hat_load_is_the_element_loop():
    prob = wl.tiny_problem(2, (6, 7), seed=2, u0_modes=0)
    hat = wl.MovingHat(1.7, 1, 0.3, 0.6, 0.2, omega=3.0, phase=0.4, time=wl.TimeFactor(omega=1.5),
                       space=(wl.SpaceFactor(kappa=2.0, phase=0.1),))
    d = Discretization(prob)
    t, q = 0.37, 3
    F = load_moving(d.grid, [hat], t, q)
    # literal element loop over the 2D elements and their tensor Gauss points
    xg, wg = gauss_legendre_01(q)
    ax = d.grid.axes
    c = hat.c0 + hat.c1 * math.sin(hat.omega * t + hat.phase)
    amp = hat.amp * math.cos(1.5 * t)
    ref = np.zeros(prob.n)
    for e0, e1 in itertools.product(range(ax[0].n + 1), range(ax[1].n + 1)):
        for g0, g1 in itertools.product(range(q), repeat=2):
            x0 = ax[0].lo + ax[0].h * (e0 + xg[g0])
            x1 = ax[1].lo + ax[1].h * (e1 + xg[g1])
            val = amp * float(space_factor(hat.space[0], np.array(x0))) * max(1 - abs(x1 - c) / hat.width, 0)
            wgt = wg[g0] * wg[g1] * ax[0].h * ax[1].h
            for k0, k1 in itertools.product((0, 1), repeat=2):
                j0, j1 = e0 + k0 - 1, e1 + k1 - 1
                if 0 <= j0 < ax[0].n and 0 <= j1 < ax[1].n:
                    b0 = xg[g0] if k0 else 1 - xg[g0]
                    b1 = xg[g1] if k1 else 1 - xg[g1]
                    ref[j0, j1] += wgt * val * b0 * b1
    assert np.max(np.abs(F - ref)) <= 1e-14 * np.max(np.abs(ref))
