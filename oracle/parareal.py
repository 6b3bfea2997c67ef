"""Algorithm 1 of the paper (PEIFE-linear), literally.

Coarse propagator G: one EIFE step of size dT with p nodes; fine propagator F:
J steps of size dt = dT/J with q nodes (Section 2.3).  Algorithm 1:

    U^{0,(0)} = P_h u0
    U^{n+1,(0)} = G(U^{n,(0)})                                   (sequential)
    repeat:
        Fbar^{n+1} = F^J(U^{n,(k)})              for all n       (parallel)
        U^{n+1,(k+1)} = G(U^{n,(k+1)}) + Fbar^{n+1} - G(U^{n,(k)}),
        U^{0,(k+1)} = U^0                                        (eq. (2.8))

The stopping rule is left open by the paper.  Reading used here: after each
iteration the relative jump ||U^{(k+1)} - U^{(k)}||_2 / ||U^{(k+1)}||_2 over
all slice ends n = 1..N and all coefficients is recorded; the loop stops when
it is <= tol or after K_max iterations.  The Euclidean norm of coefficients
is the L2 norm of u_h (M-orthonormal basis).

The second quantity the loop can watch is the residual of an iterate, how
far it is from a fine trajectory:

    res^{(k)} = ||U^{n+1,(k)} - F^J(U^{n,(k)})||_2 / ||U^{(k)}||_2,

norms over n = 0..N-1 (slice ends 1..N) and all coefficients.  F^J(U^{(k)})
is what the fine pass of iteration k + 1 computes, so the residual of
iterate k becomes known during that pass: after K passes the residuals of
iterates 0..K-1 are recorded.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from .eife import Discretization, StepTables, eife_step


@dataclass
class PararealResult:
    iterates: List[np.ndarray]          # iterates[k] has shape [N+1, *grid]
    jumps: List[float]                  # jumps[k-1] = rel. jump of iterate k vs k-1
    residuals: List[float]              # residuals[k-1] = rel. residual of iterate k-1
    iterations: int                     # number of fine passes performed
    converged: bool
    fine_outputs: List[np.ndarray] = field(default_factory=list)


def coarse_step(disc: Discretization, v: np.ndarray, Tn: float, tabG: StepTables,
                correction: Optional[np.ndarray] = None) -> np.ndarray:
    out = eife_step(disc, v, Tn, tabG)
    if correction is not None:
        out = out + correction
    return out


def fine_prop(disc: Discretization, v: np.ndarray, Tn: float, tabF: StepTables, J: int) -> np.ndarray:
    W = v
    for j in range(J):
        W = eife_step(disc, W, Tn + j * tabF.h, tabF)
    return W


def parareal(disc: Discretization, W0: np.ndarray, t0: float, N: int, J: int,
             tabF: StepTables, tabG: StepTables, K_max: int, tol: float = 0.0,
             corrections: Optional[List[np.ndarray]] = None,
             keep_fine: bool = False) -> PararealResult:
    """Run Algorithm 1.  ``corrections[n]`` (optional) is a state-independent
    additive correction of G on slice n (a learned coarse correction)."""
    dT = tabG.h
    corr = corrections if corrections is not None else [None] * N

    def G(v, n):
        return coarse_step(disc, v, t0 + n * dT, tabG, corr[n])

    U = [W0]
    for n in range(N):
        U.append(G(U[n], n))
    iterates = [np.stack(U)]
    jumps: List[float] = []
    residuals: List[float] = []
    fines = []
    converged = False
    k = 0
    while k < K_max:
        Fbar = [fine_prop(disc, U[n], t0 + n * dT, tabF, J) for n in range(N)]
        if keep_fine:
            fines.append(np.stack(Fbar))
        # residual of the iterate the fine pass started from
        cur = iterates[-1]
        res = np.stack([cur[n + 1] - Fbar[n] for n in range(N)])
        residuals.append(float(np.linalg.norm(res.ravel()) /
                               max(np.linalg.norm(cur[1:].ravel()), 1e-300)))
        Unew = [W0]
        for n in range(N):
            Unew.append(G(Unew[n], n) + Fbar[n] - G(U[n], n))
        new = np.stack(Unew)
        old = iterates[-1]
        jump = float(np.linalg.norm((new[1:] - old[1:]).ravel()) /
                     max(np.linalg.norm(new[1:].ravel()), 1e-300))
        jumps.append(jump)
        iterates.append(new)
        U = Unew
        k += 1
        if jump <= tol:
            converged = True
            break
    return PararealResult(iterates, jumps, residuals, k, converged, fines)


def sequential_fine(disc: Discretization, W0: np.ndarray, t0: float, N: int, J: int,
                    tabF: StepTables) -> np.ndarray:
    """U_seq[n] at T_n by N*J fine steps in sequence: shape [N+1, *grid]."""
    out = [W0]
    W = W0
    for n in range(N):
        W = fine_prop(disc, W, t0 + n * tabF.h * J, tabF, J)
        out.append(W)
    return np.stack(out)


def sequential_coarse(disc: Discretization, W0: np.ndarray, t0: float, N: int,
                      tabG: StepTables) -> np.ndarray:
    out = [W0]
    W = W0
    for n in range(N):
        W = eife_step(disc, W, t0 + n * tabG.h, tabG)
        out.append(W)
    return np.stack(out)
