"""phi_j functions and exponential Runge-Kutta weights, in mpmath.

Paper, eq. (2.7): b_i(-h L) = int_0^1 exp(-h(1 - theta) L) l_i(theta) dtheta
with the Lagrange basis l_i of the stage nodes c_1..c_s.  In the proof of
Theorem 3.1 the functions phi_j(-h L) = int_0^1 exp(-h(1-theta)L)
theta^(j-1)/(j-1)! dtheta appear.  On the eigenbasis L acts as the scalar
D*lambda_k, so with z = h D lambda_k every weight is a scalar function of z:

    write l_i(theta) = sum_j a_ij theta^(j-1); then
    b_i(z) = sum_j a_ij (j-1)! phi_j(-z).

phi_j is evaluated by the plain recurrence phi_0(x) = e^x,
phi_j(x) = (phi_{j-1}(x) - 1/(j-1)!) / x at a working precision high enough
that its cancellation for small z is irrelevant (>= 40 digits after the loss).
"""
from __future__ import annotations

import math
from typing import Sequence

import mpmath as mp
import numpy as np


def _dps_for(z: float, s: int) -> int:
    loss = 0 if z >= 1.0 else int(math.ceil(-math.log10(max(z, 1e-300))))
    return 40 + (s + 1) * loss


def phi_mp(j: int, x):
    """phi_j(x) by the recurrence, in the current mpmath precision."""
    x = mp.mpf(x)
    if x == 0:
        return mp.mpf(1) / mp.factorial(j)
    val = mp.exp(x)
    for i in range(1, j + 1):
        val = (val - mp.mpf(1) / mp.factorial(i - 1)) / x
    return val


def lagrange_coeffs(c: Sequence[float]):
    """a[i][j] (mpmath) with l_i(theta) = sum_j a[i][j] theta^j, j = 0..s-1."""
    s = len(c)
    cm = [mp.mpf(v) for v in c]
    out = []
    for i in range(s):
        poly = [mp.mpf(1)]                      # coefficients, ascending powers
        denom = mp.mpf(1)
        for m in range(s):
            if m == i:
                continue
            # multiply by (theta - c_m)
            new = [mp.mpf(0)] * (len(poly) + 1)
            for p, coef in enumerate(poly):
                new[p + 1] += coef
                new[p] -= cm[m] * coef
            poly = new
            denom *= (cm[i] - cm[m])
        out.append([coef / denom for coef in poly])
    return out


def weights_scalar(z: float, c: Sequence[float]):
    """(E, [b_1..b_s]) at one z >= 0, as float64 (rounded from mpmath)."""
    s = len(c)
    with mp.workdps(_dps_for(z, s)):
        a = lagrange_coeffs(c)
        x = -mp.mpf(z)
        phis = [phi_mp(j, x) for j in range(1, s + 1)]
        b = []
        for i in range(s):
            acc = mp.mpf(0)
            for j in range(1, s + 1):
                acc += a[i][j - 1] * mp.factorial(j - 1) * phis[j - 1]
            b.append(float(acc))
        return float(mp.exp(x)), b


def tables(z: np.ndarray, c: Sequence[float]):
    """E[k] = exp(-z_k) and b[i, k] = b_i(z_k) for an array of z >= 0.

    Distinct z values are evaluated once (tensor grids repeat eigenvalue
    sums along their diagonals)."""
    z = np.asarray(z, dtype=np.float64)
    uz, inv = np.unique(z.ravel(), return_inverse=True)
    s = len(c)
    E = np.empty(len(uz))
    B = np.empty((s, len(uz)))
    for k, zk in enumerate(uz):
        e, b = weights_scalar(float(zk), c)
        E[k] = e
        B[:, k] = b
    return E[inv].reshape(z.shape), B[:, inv].reshape((s,) + z.shape)

