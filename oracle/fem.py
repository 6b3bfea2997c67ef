"""1D Q1 finite element matrices and their dense LAPACK diagonalisation.

Paper, Section 2.1: the space V_h is the tensor product of 1D piecewise-linear
hat spaces on a uniform mesh of each axis (eq. (2.2)); the Galerkin form
(u_t, v) + a(u, v) = (f, v) with a(w, v) = int D grad w . grad v (eq. (2.3)).
In the nodal basis this is  M U' + D A U = F(t)  with M = kron_a M_a and
A = sum_a M_1 x .. x A_a x .. x M_d.  Section 2.3 (closing paragraph) states
that M and A are diagonalised simultaneously by one orthogonal matrix; here
that basis is *computed* by dense LAPACK (scipy.linalg.eigh of A_a) rather
than written down, so that the closed-form sine basis used by the HIP library
is checked by something independent of it.

Reading of the paper's grid (it calls N_i the number of subdomains but indexes
basis functions 1..N_i): an axis with n interior nodes has n + 1 elements of
width h = (hi - lo)/(n + 1); homogeneous Dirichlet data removes the two end
nodes.  This reading reproduces Table 1 of the paper digit for digit.
"""
from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache

import numpy as np
import scipy.linalg


def gauss_legendre_01(q: int):
    """q-point Gauss-Legendre nodes and weights on [0, 1] (weights sum to 1)."""
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def axis_matrices(n: int, lo: float, hi: float):
    """Dense 1D mass M_ij = int phi_i phi_j and stiffness A_ij = int phi_i' phi_j'
    over interior hats, assembled element by element (2-point Gauss is exact
    for the products of two linear functions)."""
    h = (hi - lo) / (n + 1)
    xg, wg = gauss_legendre_01(2)
    shape = [1.0 - xg, xg]            # local hats on the reference element
    dshape = [-1.0 / h, 1.0 / h]      # their derivatives in x
    M = np.zeros((n, n))
    A = np.zeros((n, n))
    for e in range(n + 1):            # element e = [x_e, x_{e+1}], nodes e, e+1
        gl = (e, e + 1)
        for a in range(2):
            I = gl[a] - 1             # interior index of global node gl[a]
            if I < 0 or I >= n:
                continue
            for b in range(2):
                J = gl[b] - 1
                if J < 0 or J >= n:
                    continue
                M[I, J] += h * float(np.sum(wg * shape[a] * shape[b]))
                A[I, J] += h * dshape[a] * dshape[b]
    return M, A


def periodic_axis_matrices(n: int, lo: float, hi: float):
    """Mass and stiffness of the n hats of a periodic axis (node j at
    lo + j h, h = (hi - lo)/n; element e joins nodes e and e + 1 mod n),
    assembled element by element."""
    h = (hi - lo) / n
    xg, wg = gauss_legendre_01(2)
    shape = [1.0 - xg, xg]
    dshape = [-1.0 / h, 1.0 / h]
    M = np.zeros((n, n))
    A = np.zeros((n, n))
    for e in range(n):
        gl = (e, (e + 1) % n)
        for a in range(2):
            for b in range(2):
                M[gl[a], gl[b]] += h * float(np.sum(wg * shape[a] * shape[b]))
                A[gl[a], gl[b]] += h * dshape[a] * dshape[b]
    return M, A


@dataclass
class AxisBasis:
    n: int
    lo: float
    hi: float
    h: float
    M: np.ndarray
    A: np.ndarray
    Q: np.ndarray       # M-orthonormal eigenvectors (columns), Q^T M Q = I
    lam: np.ndarray     # generalized eigenvalues: A q = lam M q
    mu: np.ndarray      # mass eigenvalues of the orthonormal eigenvectors
    periodic: bool = False


@lru_cache(maxsize=16)
def axis_basis(n: int, lo: float, hi: float, periodic: bool = False) -> AxisBasis:
    """Diagonalise the commuting pair (M_a, A_a) with dense LAPACK.

    eigh(A) gives orthonormal eigenvectors V (A has distinct eigenvalues, so V
    is unique up to signs).  M commutes with A, hence V^T M V is diagonal too:
    mu = diag(V^T M V), lam = diag(V^T A V) / mu (Rayleigh quotients), and
    Q = V diag(mu)^(-1/2) satisfies Q^T M Q = I, Q^T A Q = diag(lam).
    Signs are fixed so that the first component of each column is positive.
    (The generalized solver eigh(A, M) is avoided: it is markedly less
    accurate for the smallest eigenvalue at n ~ 500.)
    """
    if periodic:
        # circulant pair: A has double eigenvalues (the cos/sin pairs), where
        # any orthonormal basis of the eigenspace serves (M is a polynomial
        # in A, so it is diagonal there too); results are compared through
        # basis-free quantities (nodal values, norms)
        M, A = periodic_axis_matrices(n, lo, hi)
        _, V = scipy.linalg.eigh(A)
        V = V * np.sign(V[np.argmax(np.abs(V), axis=0), np.arange(n)])
        h = (hi - lo) / n
    else:
        M, A = axis_matrices(n, lo, hi)
        _, V = scipy.linalg.eigh(A)
        V = V * np.sign(V[0, :])
        h = (hi - lo) / (n + 1)
    mu = np.sum(V * (M @ V), axis=0)
    lam = np.sum(V * (A @ V), axis=0) / mu
    Q = V / np.sqrt(mu)
    return AxisBasis(n, lo, hi, h, M, A, Q, lam, mu, periodic)


class Grid:
    """Tensor-product Q1 grid on a box: per axis homogeneous Dirichlet data
    (default) or periodicity (n nodes per period)."""

    def __init__(self, n, lo, hi, periodic=None):
        self.n = tuple(int(v) for v in n)
        self.lo = tuple(float(v) for v in lo)
        self.hi = tuple(float(v) for v in hi)
        self.dim = len(self.n)
        per = tuple(bool(p) for p in periodic) if periodic else (False,) * self.dim
        self.periodic = per + (False,) * (self.dim - len(per))
        self.axes = [axis_basis(a, l, r, p) for a, l, r, p in
                     zip(self.n, self.lo, self.hi, self.periodic)]

    @property
    def shape(self):
        return self.n

    def eigenvalues(self) -> np.ndarray:
        """lambda_k = sum_a lam_a(k_a) on the tensor eigenbasis, C order."""
        lam = np.zeros(self.n)
        for a, ax in enumerate(self.axes):
            sh = [1] * self.dim
            sh[a] = ax.n
            lam = lam + ax.lam.reshape(sh)
        return lam

    def nodes(self, a: int) -> np.ndarray:
        ax = self.axes[a]
        if ax.periodic:
            return ax.lo + ax.h * np.arange(ax.n)
        return ax.lo + ax.h * np.arange(1, ax.n + 1)

    # mode products ------------------------------------------------------
    def _mode_product(self, X: np.ndarray, mats) -> np.ndarray:
        """Apply mats[a] along spatial axis a of X (trailing dim axes)."""
        off = X.ndim - self.dim
        for a, Ma in enumerate(mats):
            X = np.moveaxis(np.tensordot(Ma, X, axes=([1], [off + a])), 0, off + a)
        return X

    def to_spectral(self, F: np.ndarray) -> np.ndarray:
        """W = (kron_a Q_a)^T F : load vector -> M-orthonormal coefficients."""
        return self._mode_product(F, [ax.Q.T for ax in self.axes])

    def to_nodal(self, W: np.ndarray) -> np.ndarray:
        """U = (kron_a Q_a) W : coefficients -> nodal values of u_h."""
        return self._mode_product(W, [ax.Q for ax in self.axes])

    def mass_apply(self, U: np.ndarray) -> np.ndarray:
        return self._mode_product(U, [ax.M for ax in self.axes])

    def dense_mass(self) -> np.ndarray:
        out = np.ones((1, 1))
        for ax in self.axes:
            out = np.kron(out, ax.M)
        return out

    def dense_stiffness(self) -> np.ndarray:
        N = int(np.prod(self.n))
        out = np.zeros((N, N))
        for a in range(self.dim):
            term = np.ones((1, 1))
            for b, ax in enumerate(self.axes):
                term = np.kron(term, ax.A if b == a else ax.M)
            out += term
        return out
