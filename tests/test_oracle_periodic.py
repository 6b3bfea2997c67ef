"""Pins of the oracle's periodic axes (oracle/fem.py periodic_axis_matrices,
axis_basis(periodic=True); oracle/forcing.py load_1d(periodic=True)).

The paper carries the method over to periodic boundary conditions (Section 1;
closing remark of Section 2).  On a periodic axis with n nodes the Q1
matrices are circulant, so:

* the eigenvalues are lambda(k) = (6/h^2)(1 - cos t)/(2 + cos t),
  t = 2 pi k / n, k = 0..n-1 (a zero mode, and double eigenvalues);
* the projection of a Fourier mode cos(2 pi k x / L) is a discrete
  eigenvector, so with f = 0 it decays exactly like exp(-D lambda_k t);
* A 1 = 0, so with f = c constant the integral of u_h grows exactly by
  c |Omega| t (an ETD-RK step integrates constant forcing exactly);
* the factorised load equals a literal element loop with wrapped nodes;
* a manufactured solution (periodic in x, Dirichlet in y) converges in L2
  like h^2.
"""
import itertools
import math

import numpy as np
import pytest

import workloads as wl
from oracle.eife import Discretization, sequential
from oracle.fem import axis_basis, gauss_legendre_01
from oracle.forcing import load_field, space_factor

PI = math.pi


@pytest.mark.parametrize("n", [8, 32, 128])
def test_periodic_eigenvalues_closed_form(n):
    lo, hi = 0.25, 1.75
    ax = axis_basis(n, lo, hi, True)
    h = (hi - lo) / n
    t = 2 * PI * np.arange(n) / n
    lam = (6 / h ** 2) * (1 - np.cos(t)) / (2 + np.cos(t))
    mu = (h / 3) * (2 + np.cos(t))
    assert np.max(np.abs(np.sort(ax.lam) - np.sort(lam))) <= 1e-11 * lam.max()
    assert np.max(np.abs(np.sort(ax.mu) - np.sort(mu))) <= 1e-14
    assert np.allclose(ax.Q.T @ ax.M @ ax.Q, np.eye(n), atol=1e-12)


def _periodic_prob(n, forcing, u0, D=0.3, N=2, J=4, s=3, T=0.5, lo=(0.0,), hi=(1.0,), per=(True,)):
    return wl.Problem("periodic", len(n), tuple(n), tuple(lo), tuple(hi), D, 0.0, T, forcing, u0, N, J,
                      (0.0, 0.45, 0.9)[:s], (0.0, 0.45, 0.9)[:s], periodic=per)


def test_fourier_mode_decays_exactly():
    n, L = 32, 1.0
    k = 3
    u0 = [wl.Term(1.0, wl.TimeFactor(), (wl.SpaceFactor(kappa=2 * PI * k / L, phase=PI / 2),))]
    prob = _periodic_prob((n,), [], u0, D=0.2, T=0.7)
    d = Discretization(prob)
    W0 = d.initial()
    W = sequential(d, W0, 0.0, d.tables(prob.dt, prob.c_fine), prob.N * prob.J)
    h = L / n
    th = 2 * PI * k / n
    lam = (6 / h ** 2) * (1 - math.cos(th)) / (2 + math.cos(th))
    U0, U = d.grid.to_nodal(W0), d.grid.to_nodal(W)
    assert np.max(np.abs(U - math.exp(-prob.D * lam * prob.T) * U0)) <= 1e-13 * np.max(np.abs(U0))
    # the projection of the mode is the mode at the grid's nodes, scaled
    mode = np.cos(2 * PI * k * d.grid.nodes(0) / L)
    scale = float(U0 @ mode / (mode @ mode))
    assert np.max(np.abs(U0 - scale * mode)) <= 1e-13


def test_mean_follows_constant_forcing():
    n = (16, 12)
    f = [wl.Term(0.7, wl.TimeFactor(), (wl.poly_factor(1.0), wl.poly_factor(1.0)))]
    u0 = [wl.Term(1.0, wl.TimeFactor(), (wl.SpaceFactor(kappa=2 * PI, phase=0.3), wl.poly_factor(1.0, 0.5)))]
    prob = _periodic_prob(n, f, u0, lo=(0.0, 0.0), hi=(1.0, 2.0), per=(True, True))
    d = Discretization(prob)
    W0 = d.initial()
    W = sequential(d, W0, 0.0, d.tables(prob.dt, prob.c_fine), prob.N * prob.J)
    ones = np.ones(n)
    integral = lambda W: float(np.sum(d.grid.mass_apply(ones) * d.grid.to_nodal(W)))
    assert abs(integral(W) - (integral(W0) + 0.7 * 2.0 * prob.T)) <= 1e-12


def test_periodic_load_is_the_element_loop():
    n = (6, 5)
    lo, hi = (0.5, 0.0), (2.0, 1.0)
    terms = [wl.Term(1.3, wl.TimeFactor(omega=2.0), (wl.poly_factor(0.2, 1.0, -0.3),
                                                     wl.SpaceFactor(kappa=1.1, phase=0.4)))]
    prob = _periodic_prob(n, terms, [], lo=lo, hi=hi, per=(True, False))
    d = Discretization(prob)
    t, q = 0.3, 3
    F = load_field(d.grid, terms, t, q)
    xg, wg = gauss_legendre_01(q)
    h = [(hi[0] - lo[0]) / n[0], (hi[1] - lo[1]) / (n[1] + 1)]
    ref = np.zeros(n)
    amp = 1.3 * math.cos(2.0 * t)
    for e0, e1 in itertools.product(range(n[0]), range(n[1] + 1)):
        for g0, g1 in itertools.product(range(q), repeat=2):
            x0 = lo[0] + h[0] * (e0 + xg[g0])
            x1 = lo[1] + h[1] * (e1 + xg[g1])
            val = amp * float(space_factor(terms[0].space[0], np.array(x0))) * \
                float(space_factor(terms[0].space[1], np.array(x1)))
            w = wg[g0] * wg[g1] * h[0] * h[1]
            for k0, k1 in itertools.product((0, 1), repeat=2):
                j0 = (e0 + k0) % n[0]                 # periodic: node n is node 0
                j1 = e1 + k1 - 1                      # Dirichlet: interior 1..n
                if 0 <= j1 < n[1]:
                    b0 = xg[g0] if k0 else 1 - xg[g0]
                    b1 = xg[g1] if k1 else 1 - xg[g1]
                    ref[j0, j1] += w * val * b0 * b1
    assert np.max(np.abs(F - ref)) <= 1e-14 * np.max(np.abs(ref))


def _eval_matrix(n, q, periodic):
    xg, _ = gauss_legendre_01(q)
    ne = n if periodic else n + 1
    B = np.zeros((ne * q, n))
    for e in range(ne):
        for g in range(q):
            r = e * q + g
            if periodic:
                B[r, e] += 1 - xg[g]
                B[r, (e + 1) % n] += xg[g]
            else:
                if e - 1 >= 0:
                    B[r, e - 1] = 1 - xg[g]
                if e < n:
                    B[r, e] = xg[g]
    return B


def test_manufactured_solution_converges_like_h2():
    """u = e^{-t} (cos 2 pi x + 0.3 sin 4 pi x) sin(pi y), periodic in x,
    Dirichlet in y, D = 0.05."""
    D = 0.05
    dec = wl.TimeFactor(alpha=-1.0)
    cx = wl.SpaceFactor(kappa=2 * PI, phase=PI / 2)
    sx = wl.SpaceFactor(kappa=4 * PI, phase=0.0)
    sy = wl.SpaceFactor(kappa=PI, phase=0.0)
    u = [wl.Term(1.0, dec, (cx, sy)), wl.Term(0.3, dec, (sx, sy))]
    f = [wl.Term(-1.0 + D * (4 * PI ** 2 + PI ** 2), dec, (cx, sy)),
         wl.Term(0.3 * (-1.0 + D * (16 * PI ** 2 + PI ** 2)), dec, (sx, sy))]
    errs = []
    q = 5
    xg, wg = gauss_legendre_01(q)
    for m in (16, 32, 64):
        prob = _periodic_prob((m, m - 1), f, u, D=D, N=2, J=8, T=0.4, lo=(0.0, 0.0), hi=(1.0, 1.0),
                              per=(True, False))
        d = Discretization(prob)
        W = sequential(d, d.initial(), 0.0, d.tables(prob.dt, prob.c_fine), prob.N * prob.J)
        U = d.grid.to_nodal(W)
        B0, B1 = _eval_matrix(m, q, True), _eval_matrix(m - 1, q, False)
        uh = B0 @ U @ B1.T
        h0, h1 = 1.0 / m, 1.0 / m
        x0 = (h0 * (np.arange(m)[:, None] + xg[None, :])).ravel()
        x1 = (h1 * (np.arange(m)[:, None] + xg[None, :])).ravel()
        ex = sum(t.amp * math.exp(-prob.T) * np.outer(space_factor(t.space[0], x0),
                                                       space_factor(t.space[1], x1)) for t in u)
        w = np.outer(np.tile(wg * h0, m), np.tile(wg * h1, m))
        errs.append(math.sqrt(np.sum(w * (uh - ex) ** 2)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.85 <= r <= 2.15 for r in rates), (errs, rates)
