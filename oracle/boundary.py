"""Non-homogeneous Dirichlet data for the FP64 oracle (test infrastructure).

The paper states its method for homogeneous Dirichlet data (Section 2,
eq. (2.1)) and notes at the start of Sections 3 and 4 that the extension to
non-homogeneous data is straightforward, without giving it.  Reading used
here (and by the HIP library): the discrete solution is
    u_h(t) = sum_{interior j} U_j(t) phi_j + g_h(t),
    g_h(t) = sum_{boundary b} g(t, x_b) phi_b,
the Q1 interpolant of the boundary data on the boundary nodes.  Testing the
Galerkin form with the interior hats gives, for the interior unknowns,
    M_II U' + D A_II U = F_I(t) - M_IB G_B'(t) - D A_IB G_B(t),
so the method of eq. (2.6) runs unchanged on the load vector
F_I - M_IB G_B' - D A_IB G_B, and the initial interior values are the L2
projection of u0 with the boundary part fixed:
    M_II U(t0) = (u0, phi_I) - M_IB G_B(t0).

Everything here is assembled literally on the full grid, boundary nodes
included: 1D element matrices over all n + 2 nodes, their Kronecker
products, and the nodal boundary field G_B (the data g at boundary nodes,
zero inside).  The time derivative of the data's time factors is taken by a
complex step (exact to rounding for these analytic factors), not by a
formula, so it does not share the library's derivative.
"""
from __future__ import annotations

import cmath
import math

import numpy as np

from .fem import gauss_legendre_01
from .forcing import eval_terms, space_factor


def full_axis_matrices(n: int, lo: float, hi: float):
    """Mass and stiffness of all n + 2 hats of an axis (boundary nodes
    included), assembled element by element."""
    h = (hi - lo) / (n + 1)
    xg, wg = gauss_legendre_01(2)
    shape = [1.0 - xg, xg]
    dshape = [-1.0 / h, 1.0 / h]
    M = np.zeros((n + 2, n + 2))
    A = np.zeros((n + 2, n + 2))
    for e in range(n + 1):
        nodes = (e, e + 1)
        for a in range(2):
            for b in range(2):
                M[nodes[a], nodes[b]] += h * float(np.sum(wg * shape[a] * shape[b]))
                A[nodes[a], nodes[b]] += h * dshape[a] * dshape[b]
    return M, A


def _time_factor_c(tf, t: complex) -> complex:
    p = tf.poly
    return (cmath.exp(tf.alpha * t) * cmath.cos(tf.omega * t + tf.phase)
            * (p[0] + t * (p[1] + t * (p[2] + t * p[3]))))


def time_factor_derivative(tf, t: float) -> float:
    """d tau / dt by a complex step: Im tau(t + i eps) / eps."""
    eps = 1e-30
    return (_time_factor_c(tf, complex(t, eps))).imag / eps


def full_nodes(prob, a: int) -> np.ndarray:
    n, lo, hi = prob.n[a], prob.lo[a], prob.hi[a]
    h = (hi - lo) / (n + 1)
    return lo + h * np.arange(n + 2)


def boundary_field(prob, t: float, derivative: bool = False) -> np.ndarray:
    """G_B(t) (or G_B'(t)) on the full (n_a + 2)-node grid: the data at the
    boundary nodes, zero at interior nodes."""
    pts = [full_nodes(prob, a) for a in range(prob.dim)]
    shape = tuple(len(p) for p in pts)
    G = np.zeros(shape)
    for term in prob.boundary:
        tau = time_factor_derivative(term.time, t) if derivative else _time_factor_c(term.time, t).real
        prod = np.ones(())
        for sf, xs in zip(term.space, pts):
            prod = np.multiply.outer(prod, space_factor(sf, xs))
        G = G + term.amp * tau * prod
    interior = tuple(slice(1, -1) for _ in range(prob.dim))
    G[interior] = 0.0
    return G


def _apply(mats, X):
    for a, Ma in enumerate(mats):
        X = np.moveaxis(np.tensordot(Ma, X, axes=([1], [a])), 0, a)
    return X


class FullGrid:
    """Full-grid matrices of one problem (boundary nodes included)."""

    def __init__(self, prob):
        self.prob = prob
        self.mats = [full_axis_matrices(prob.n[a], prob.lo[a], prob.hi[a]) for a in range(prob.dim)]

    def mass(self, X: np.ndarray) -> np.ndarray:
        return _apply([M for M, _ in self.mats], X)

    def stiffness(self, X: np.ndarray) -> np.ndarray:
        out = np.zeros_like(X)
        for a in range(self.prob.dim):
            out = out + _apply([A if b == a else M for b, (M, A) in enumerate(self.mats)], X)
        return out

    def interior(self, X: np.ndarray) -> np.ndarray:
        return X[tuple(slice(1, -1) for _ in range(self.prob.dim))]

    def load_correction(self, t: float) -> np.ndarray:
        """-(M_IB G_B'(t) + D A_IB G_B(t)) on the interior nodes."""
        G = boundary_field(self.prob, t)
        Gd = boundary_field(self.prob, t, derivative=True)
        return -self.interior(self.mass(Gd) + self.prob.D * self.stiffness(G))

    def initial_correction(self, t: float) -> np.ndarray:
        """-M_IB G_B(t) on the interior nodes."""
        return -self.interior(self.mass(boundary_field(self.prob, t)))


def full_nodal(prob, U_interior: np.ndarray, t: float) -> np.ndarray:
    """Nodal values of u_h on the full grid: interior unknowns plus g."""
    G = boundary_field(prob, t)
    G[tuple(slice(1, -1) for _ in range(prob.dim))] = U_interior
    return G


def l2_error_full(prob, U_interior: np.ndarray, exact_terms, t: float, q: int = 5) -> float:
    """|| u_h - u(t) ||_L2 with u_h from the full nodal values (boundary
    included), by a q-point tensor Gauss rule per element."""
    Uf = full_nodal(prob, U_interior, t)
    pts, wts, mats = [], [], []
    xg, wg = gauss_legendre_01(q)
    for a in range(prob.dim):
        n, lo, hi = prob.n[a], prob.lo[a], prob.hi[a]
        h = (hi - lo) / (n + 1)
        e = np.arange(n + 1)[:, None]
        pts.append((lo + h * (e + xg[None, :])).ravel())
        wts.append(np.tile(wg * h, n + 1))
        B = np.zeros(((n + 1) * q, n + 2))
        for el in range(n + 1):
            for g in range(q):
                B[el * q + g, el] = 1.0 - xg[g]
                B[el * q + g, el + 1] = xg[g]
        mats.append(B)
    uh = _apply(mats, Uf)
    u = eval_terms(exact_terms, t, pts)
    w = np.ones(())
    for wa in wts:
        w = np.multiply.outer(w, wa)
    return float(math.sqrt(np.sum(w * (uh - u) ** 2)))
