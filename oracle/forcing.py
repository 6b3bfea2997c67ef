"""Separable functions and Galerkin load vectors.

The EIFE step (paper, eq. (2.6)) needs P_h f at the stage times; in the nodal
basis P_h f = M^{-1} F with the load vector F_j(t) = int f(t, x) Phi_j(x) dx,
and the initial value u_h(t0) = P_h u0 (eq. (2.2)) likewise comes from the
load vector of u0.  The paper does not state how these integrals are
evaluated; the reading used here (and by the HIP library) is the consistent
Galerkin load evaluated element by element with a q-point tensor
Gauss-Legendre rule (q = 3 by default; a 20-point rule stands in for the exact
integral when reproducing the paper's tables).

For a separable term amp * tau(t) * prod_a X_a(x_a) a tensor Gauss rule on a
box element factorises exactly into the product of the 1D rules, so the d-D
load of one term is the outer product of 1D loads (``load_field``).
``load_field_elementwise`` does the d-D element loop literally (used to check
that factorisation on small grids).
"""
from __future__ import annotations

import itertools
import math
from functools import lru_cache
from typing import Sequence

import numpy as np

from .fem import Grid, gauss_legendre_01

EXACT_Q = 20   # Gauss points per element standing in for exact integrals


def time_factor(tf, t):
    p = tf.poly
    return (math.exp(tf.alpha * t) * math.cos(tf.omega * t + tf.phase)
            * (p[0] + t * (p[1] + t * (p[2] + t * p[3]))))


def space_factor(sf, x):
    q = sf.poly
    return (q[0] + x * (q[1] + x * q[2])) * np.sin(sf.kappa * x + sf.phase)


def eval_terms(terms, t, grid_points: Sequence[np.ndarray], use_time=True) -> np.ndarray:
    """Value of sum_m amp tau(t) prod X_a on the tensor grid of 1D point sets."""
    shape = tuple(len(p) for p in grid_points)
    out = np.zeros(shape)
    for term in terms:
        v = term.amp * (time_factor(term.time, t) if use_time else 1.0)
        prod = np.ones(())
        for a, (sf, xs) in enumerate(zip(term.space, grid_points)):
            prod = np.multiply.outer(prod, space_factor(sf, xs))
        out = out + v * prod
    return out


@lru_cache(maxsize=4096)
def load_1d(sf, n: int, lo: float, hi: float, q: int, periodic: bool = False) -> np.ndarray:
    """C_j = int X(x) phi_j(x) dx over the two elements touching node j.

    Element e = [x_e, x_{e+1}] (e = 0..n) carries the local hats 1 - xi (node
    e) and xi (node e + 1); interior node j (1..n) collects the right half of
    element j - 1 and the left half of element j.  The elements are looped
    over as one vectorised array.  Periodic axis (n nodes per period, node j
    at lo + j h, element e = [x_e, x_{e+1}], e = 0..n-1, node n = node 0):
    node j collects the right half of element j - 1 (mod n) and the left half
    of element j."""
    if periodic:
        h = (hi - lo) / n
        xg, wg = gauss_legendre_01(q)
        e = np.arange(n)[:, None]
        X = space_factor(sf, lo + h * (e + xg[None, :]))
        left = h * np.sum(wg * X * (1.0 - xg), axis=1)        # to node e
        right = h * np.sum(wg * X * xg, axis=1)               # to node e + 1
        C = left + np.roll(right, 1)
        C.setflags(write=False)
        return C
    h = (hi - lo) / (n + 1)
    xg, wg = gauss_legendre_01(q)
    e = np.arange(n + 1)[:, None]
    X = space_factor(sf, lo + h * (e + xg[None, :]))          # [n+1, q]
    left = h * np.sum(wg * X * (1.0 - xg), axis=1)            # to node e
    right = h * np.sum(wg * X * xg, axis=1)                   # to node e + 1
    C = np.zeros(n)
    C += left[1:]          # node j = e for e = 1..n  -> index e - 1
    C += right[:-1]        # node j = e + 1 for e = 0..n-1 -> index e
    C.setflags(write=False)
    return C


def hat_center(hat, t: float) -> float:
    return hat.c0 + hat.c1 * math.sin(hat.omega * t + hat.phase)


def hat_load_1d(hat, t: float, n: int, lo: float, hi: float, q: int) -> np.ndarray:
    """C_j = int max(1 - |x - c(t)| / w, 0) phi_j(x) dx by the q-point Gauss
    rule on the two elements touching node j (the rule of every other load,
    reading R2; the hat's kinks fall inside elements and are not treated
    specially)."""
    h = (hi - lo) / (n + 1)
    xg, wg = gauss_legendre_01(q)
    c = hat_center(hat, t)
    e = np.arange(n + 1)[:, None]
    x = lo + h * (e + xg[None, :])
    X = np.maximum(1.0 - np.abs(x - c) / hat.width, 0.0)
    left = h * np.sum(wg * X * (1.0 - xg), axis=1)
    right = h * np.sum(wg * X * xg, axis=1)
    C = np.zeros(n)
    C += left[1:]
    C += right[:-1]
    return C


def load_moving(grid: Grid, hats, t: float, q: int = 3) -> np.ndarray:
    """Nodal load of moving hat sources: per source, the hat's 1D load along
    its axis times the other axes' factor loads, times amp tau(t)."""
    F = np.zeros(grid.n)
    for hat in hats:
        v = hat.amp * time_factor(hat.time, t)
        prod = np.ones(())
        for a, ax in enumerate(grid.axes):
            if a == hat.axis:
                vec = hat_load_1d(hat, t, ax.n, ax.lo, ax.hi, q)
            else:
                vec = load_1d(hat.space[a], ax.n, ax.lo, ax.hi, q)
            prod = np.multiply.outer(prod, vec)
        F = F + v * prod
    return F


def load_field(grid: Grid, terms, t: float, q: int = 3, use_time: bool = True) -> np.ndarray:
    """Nodal load vector F(t) of a separable function, shape grid.n."""
    F = np.zeros(grid.n)
    for term in terms:
        v = term.amp * (time_factor(term.time, t) if use_time else 1.0)
        prod = np.ones(())
        for a, sf in enumerate(term.space):
            ax = grid.axes[a]
            prod = np.multiply.outer(prod, load_1d(sf, ax.n, ax.lo, ax.hi, q, ax.periodic))
        F = F + v * prod
    return F


def load_field_elementwise(grid: Grid, terms, t: float, q: int = 3, use_time: bool = True) -> np.ndarray:
    """The same load vector by a literal d-D element loop (small grids only):
    for every box element, for every tensor Gauss point, add
    w * f(t, x) * Phi_j(x) to the 2^d vertices j of the element."""
    xg, wg = gauss_legendre_01(q)
    d = grid.dim
    hs = [ax.h for ax in grid.axes]
    F = np.zeros(grid.n)
    for elem in itertools.product(*[range(ax.n + 1) for ax in grid.axes]):
        for gidx in itertools.product(range(q), repeat=d):
            x = [grid.axes[a].lo + hs[a] * (elem[a] + xg[gidx[a]]) for a in range(d)]
            w = float(np.prod([wg[g] for g in gidx]) * np.prod(hs))
            fval = 0.0
            for term in terms:
                v = term.amp * (time_factor(term.time, t) if use_time else 1.0)
                for a, sf in enumerate(term.space):
                    v *= float(space_factor(sf, np.array(x[a])))
                fval += v
            for corner in itertools.product((0, 1), repeat=d):
                idx = []
                basis = 1.0
                for a in range(d):
                    node = elem[a] + corner[a]
                    basis *= xg[gidx[a]] if corner[a] else (1.0 - xg[gidx[a]])
                    idx.append(node - 1)
                if all(0 <= idx[a] < grid.axes[a].n for a in range(d)):
                    F[tuple(idx)] += w * fval * basis
    return F
