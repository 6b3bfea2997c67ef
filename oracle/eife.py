"""The EIFE-linear method in the M-orthonormal eigenbasis.

Paper, eq. (2.6):  u^{n+1} = e^{-h L_h} u^n + h sum_i b_i(-h L_h) P_h f(t_n + c_i h).

With U = Q W (Q = kron_a Q_a, Q^T M Q = I, Q^T A Q = diag(lambda)) the
semi-discrete system M U' + D A U = F(t) becomes W' + D diag(lambda) W = Q^T F,
so L_h acts as D*lambda_k on coefficient k and P_h f has coefficients Q^T F.
The L2 norm of u_h is the Euclidean norm of W.  u_h(t0) = P_h u0 has
coefficients Q^T F_{u0}, F_{u0} the load vector of u0 (eq. (2.2)).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import phi
from .boundary import FullGrid
from .fem import Grid, gauss_legendre_01
from .forcing import load_field, load_moving, eval_terms, space_factor, time_factor


@dataclass
class StepTables:
    h: float
    c: tuple
    E: np.ndarray      # exp(-h D lambda)
    b: np.ndarray      # [s, *grid.n], b_i(h D lambda)


class Discretization:
    """Grid + diffusion coefficient + forcing of one problem."""

    def __init__(self, prob, q: int = 3):
        self.prob = prob
        self.grid = Grid(prob.n, prob.lo, prob.hi, getattr(prob, "periodic", None))
        if any(self.grid.periodic):
            assert not getattr(prob, "boundary", None) and not getattr(prob, "moving", None), \
                "Dirichlet data and moving sources are for non-periodic axes"
        self.D = float(prob.D)
        self.q = q
        self.lam = self.grid.eigenvalues()
        # non-homogeneous Dirichlet data: the interior system's load gains
        # -(M_IB G_B' + D A_IB G_B) (oracle/boundary.py)
        self.full = FullGrid(prob) if getattr(prob, "boundary", None) else None

    def tables(self, h: float, c: Sequence[float]) -> StepTables:
        z = h * self.D * self.lam
        E, b = phi.tables(z, c)
        return StepTables(h, tuple(c), E, b)

    def spectral_forcing(self, t: float) -> np.ndarray:
        """Coefficients of P_h f(t): Q^T F(t) (with the boundary coupling)."""
        F = load_field(self.grid, self.prob.forcing, t, self.q)
        if getattr(self.prob, "moving", None):
            F = F + load_moving(self.grid, self.prob.moving, t, self.q)
        if self.full is not None:
            F = F + self.full.load_correction(t)
        return self.grid.to_spectral(F)

    def initial(self) -> np.ndarray:
        """Coefficients of P_h u0 (with boundary data: the interior part of
        the L2 projection whose boundary values are g(t0))."""
        F = np.zeros(self.grid.n)
        if self.prob.u0:
            F = load_field(self.grid, self.prob.u0, 0.0, self.q, use_time=False)
        if self.full is not None:
            F = F + self.full.initial_correction(self.prob.t0)
        return self.grid.to_spectral(F)


def eife_step(disc: Discretization, W: np.ndarray, t: float, tab: StepTables) -> np.ndarray:
    """One step of eq. (2.6) from t to t + h."""
    out = tab.E * W
    for i, ci in enumerate(tab.c):
        out = out + tab.h * tab.b[i] * disc.spectral_forcing(t + ci * tab.h)
    return out


def sequential(disc: Discretization, W0: np.ndarray, t0: float, tab: StepTables, nsteps: int,
               keep_every: Optional[int] = None):
    """nsteps steps of eq. (2.6); returns the final W (and the states every
    ``keep_every`` steps, including the start, when asked)."""
    W = W0
    kept = [W0] if keep_every else None
    for j in range(nsteps):
        W = eife_step(disc, W, t0 + j * tab.h, tab)
        if keep_every and (j + 1) % keep_every == 0:
            kept.append(W)
    return (W, kept) if keep_every else W


# ---------------------------------------------------------------------------
# errors against an exact solution
# ---------------------------------------------------------------------------

def _hat_eval_matrix(ax, xs_elem, q):
    """B[(e, g), j] = phi_j(x_{e,g}) for the q Gauss points of each element."""
    n = ax.n
    xg, _ = gauss_legendre_01(q)
    B = np.zeros(((n + 1) * q, n))
    for e in range(n + 1):
        for g in range(q):
            r = e * q + g
            if e - 1 >= 0:
                B[r, e - 1] = 1.0 - xg[g]
            if e < n:
                B[r, e] = xg[g]
    return B


def l2_error(disc: Discretization, W: np.ndarray, exact_terms, t: float, q: int = 5) -> float:
    """|| u_h - u(t) ||_{L2(Omega)} by a q-point tensor Gauss rule per element."""
    grid = disc.grid
    U = grid.to_nodal(W)
    pts, wts, mats = [], [], []
    for ax in grid.axes:
        xg, wg = gauss_legendre_01(q)
        e = np.arange(ax.n + 1)[:, None]
        pts.append((ax.lo + ax.h * (e + xg[None, :])).ravel())
        wts.append(np.tile(wg * ax.h, ax.n + 1))
        mats.append(_hat_eval_matrix(ax, None, q))
    uh = U
    for a, Ba in enumerate(mats):
        uh = np.moveaxis(np.tensordot(Ba, uh, axes=([1], [a])), 0, a)
    u = eval_terms(exact_terms, t, pts)
    w = np.ones(())
    for wa in wts:
        w = np.multiply.outer(w, wa)
    return float(np.sqrt(np.sum(w * (uh - u) ** 2)))


def nodal_max_error(disc: Discretization, W: np.ndarray, exact_terms, t: float) -> float:
    """max_j |U_j - u(t, x_j)| over the interior nodes."""
    grid = disc.grid
    U = grid.to_nodal(W)
    u = eval_terms(exact_terms, t, [grid.nodes(a) for a in range(grid.dim)])
    return float(np.max(np.abs(U - u)))
