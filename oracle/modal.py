"""Selected-mode FP64 oracle of the fine solution (test infrastructure).

In the M-orthonormal eigenbasis every coefficient evolves on its own: the
EIFE step, eq. (2.6), acts on coefficient k as

    w <- e^{-z_k} w + h sum_i b_i(z_k) ghat_k(t + c_i h),   z_k = h D lambda_k,

with b_i from eq. (2.7).  For a separable forcing
f = sum_m amp_m tau_m(t) prod_a X_{m,a}(x_a) the tensor Gauss rule factorises,
so the nodal load is F(t) = sum_m amp_m tau_m(t) kron_a C_{m,a} (C_{m,a} the 1D
loads), and by the Kronecker identity (kron_a Q_a)^T (kron_a C_a) =
kron_a (Q_a^T C_a) its coefficient k is

    ghat_k(t) = sum_m amp_m tau_m(t) prod_a (Q_a^T C_{m,a})[k_a].

The sequential fine solution (the answer Parareal converges to: every iterate
k >= 1 equals it, Theorem 4.4 and its strong form) of any chosen set of modes
therefore needs only per-axis eigenvectors and 1D loads, at any grid size.
The per-axis pieces come from the same dense LAPACK basis and element loads
as the full-field oracle (``fem``, ``forcing``); the tests pin this module
against the full-field oracle on small grids.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from . import phi
from .fem import axis_basis
from .forcing import load_1d, time_factor


def axis_spectra(prob, terms=None, q: int = 3):
    """spec[a][m] = Q_a^T C_{m,a}: the spectral 1D load of term m on axis a."""
    terms = prob.forcing if terms is None else terms
    out = []
    for a in range(prob.dim):
        ax = axis_basis(prob.n[a], prob.lo[a], prob.hi[a])
        out.append([ax.Q.T @ load_1d(term.space[a], ax.n, ax.lo, ax.hi, q) for term in terms])
    return out


def forced_modes(prob, rel: float = 1e-10, q: int = 3) -> np.ndarray:
    """Multi-indices [count, d] of the modes some forcing term reaches: per
    term, the product of the per-axis indices whose spectral load exceeds
    rel times that axis' largest."""
    spec = axis_spectra(prob, q=q)
    found = set()
    for m in range(len(prob.forcing)):
        per_axis = []
        for a in range(prob.dim):
            v = np.abs(spec[a][m])
            per_axis.append(np.nonzero(v > rel * v.max())[0] if v.max() > 0 else [])
        grids = np.meshgrid(*per_axis, indexing="ij")
        for idx in zip(*[g.ravel() for g in grids]):
            found.add(tuple(int(i) for i in idx))
    return np.array(sorted(found), dtype=np.int64).reshape(-1, prob.dim)


def mode_lambdas(prob, modes: np.ndarray) -> np.ndarray:
    lam = np.zeros(len(modes))
    for a in range(prob.dim):
        ax = axis_basis(prob.n[a], prob.lo[a], prob.hi[a])
        lam += ax.lam[modes[:, a]]
    return lam


class ModalForcing:
    """ghat on a fixed set of modes: [terms, modes] factor matrix times the
    per-term time factors."""

    def __init__(self, prob, modes: np.ndarray, terms=None, q: int = 3):
        terms = prob.forcing if terms is None else terms
        spec = axis_spectra(prob, terms, q)
        self.terms = terms
        self.G = np.ones((len(terms), len(modes)))
        for m in range(len(terms)):
            for a in range(prob.dim):
                self.G[m] *= spec[a][m][modes[:, a]]

    def at(self, t: float) -> np.ndarray:
        coef = np.array([term.amp * time_factor(term.time, t) for term in self.terms])
        return coef @ self.G

    def static(self) -> np.ndarray:
        """Coefficients of a time-independent separable function (P_h u0)."""
        return np.array([term.amp for term in self.terms]) @ self.G


class ModalFine:
    """The fine propagator F^J (J steps of eq. (2.6) with step dt = dT/J and
    the fine nodes) restricted to a set of modes."""

    def __init__(self, prob, modes: np.ndarray, q: int = 3):
        self.modes = np.asarray(modes, dtype=np.int64).reshape(-1, prob.dim)
        self.dT = (prob.T - prob.t0) / prob.N
        self.dt = self.dT / prob.J
        self.J = prob.J
        self.c = tuple(prob.c_fine)
        lam = mode_lambdas(prob, self.modes)
        self.E, self.B = phi.tables(self.dt * prob.D * lam, self.c)
        self.forcing = ModalForcing(prob, self.modes, q=q)

    def propagate(self, W: np.ndarray, Tn: float) -> np.ndarray:
        """F^J(W) over the slice starting at Tn."""
        for j in range(self.J):
            t = Tn + j * self.dt
            acc = self.E * W
            for i, ci in enumerate(self.c):
                acc = acc + self.dt * self.B[i] * self.forcing.at(t + ci * self.dt)
            W = acc
        return W


def sequential_fine_modes(prob, modes: np.ndarray, q: int = 3,
                          steps: Optional[int] = None) -> np.ndarray:
    """W[n, i] at T_n = t0 + n dT (n = 0..N) of mode modes[i] under N*J fine
    steps of eq. (2.6) with the fine nodes; W[0] = P_h u0 on those modes."""
    fine = ModalFine(prob, modes, q)
    W = (ModalForcing(prob, fine.modes, terms=prob.u0, q=q).static() if prob.u0
         else np.zeros(len(fine.modes)))
    out = [W]
    for n in range(prob.N if steps is None else steps):
        W = fine.propagate(W, prob.t0 + n * fine.dT)
        out.append(W)
    return np.stack(out)


def sample_modes(prob, n_random: int, seed: int) -> np.ndarray:
    """The forced modes plus n_random other modes drawn from the seed."""
    forced = forced_modes(prob)
    rng = np.random.default_rng(seed)
    extra = np.stack([rng.integers(0, prob.n[a], n_random) for a in range(prob.dim)], axis=1)
    allm = np.concatenate([forced, extra]) if len(forced) else extra
    return np.unique(allm, axis=0)


def flat_index(prob, modes: np.ndarray) -> np.ndarray:
    """C-order flat index of each multi-index (last axis fastest)."""
    return np.ravel_multi_index(tuple(modes[:, a] for a in range(prob.dim)), prob.n)
