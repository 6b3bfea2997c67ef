"""Pins of the oracle's non-homogeneous Dirichlet data (oracle/boundary.py)
against what the mathematics fixes, independently of the oracle's own
formula for the boundary coupling:

* a bilinear (harmonic, Q1-representable) u with f = 0 and g = u is a steady
  state: the projected initial value is u at the interior nodes and stays so;
* u = tau(t) l(x), l bilinear, f = tau' l, g = u is the exact semi-discrete
  solution, and a 3-stage ETD-RK step is exact for a quadratic tau (the
  forcing is then a polynomial of degree < s in t, paper Section 2.2);
* time-independent non-harmonic data with f = 0 on a tiny grid: the exact
  semi-discrete solution U(t) = U_inf + exp(-t D M^-1 A)(U0 - U_inf), built
  here from matrices assembled in the test and scipy's expm (ETD-RK
  integrates constant forcing exactly);
* data that vanishes on the boundary gives the homogeneous answer;
* a manufactured solution with time-dependent boundary values converges in
  L2 like h^2 (Lemma 3.1 / Theorem 4.5 of the paper, extended to the
  non-homogeneous data).
"""
import math

import numpy as np
import pytest
import scipy.linalg

import workloads as wl
from oracle import boundary as ob
from oracle.eife import Discretization, sequential

pytestmark = pytest.mark.filterwarnings("ignore")

P = wl.poly_factor
ONE = wl.TimeFactor()


def _bilinear(dim):
    """l(x) = 1 + 0.5 x0 - 0.3 x1 + 0.7 x0 x1 (+ 0.2 x2 - 0.4 x0 x2 in 3D)."""
    terms = [wl.Term(1.0, ONE, tuple(P(1.0) for _ in range(dim))),
             wl.Term(0.5, ONE, (P(0.0, 1.0),) + tuple(P(1.0) for _ in range(dim - 1)))]
    if dim >= 2:
        terms += [wl.Term(-0.3, ONE, (P(1.0), P(0.0, 1.0)) + tuple(P(1.0) for _ in range(dim - 2))),
                  wl.Term(0.7, ONE, (P(0.0, 1.0), P(0.0, 1.0)) + tuple(P(1.0) for _ in range(dim - 2)))]
    if dim == 3:
        terms += [wl.Term(0.2, ONE, (P(1.0), P(1.0), P(0.0, 1.0))),
                  wl.Term(-0.4, ONE, (P(0.0, 1.0), P(1.0), P(0.0, 1.0)))]
    return terms


def _with_time(terms, tf):
    return [wl.Term(t.amp, tf, t.space) for t in terms]


def _prob(dim, n, D=0.37, N=2, J=3, s=3, T=0.4, **kw):
    base = wl.tiny_problem(dim, n, seed=3, s=s, N=N, J=J, D=D, T=T, u0_modes=0)
    return base.with_(**kw)


def _interior_values(prob, terms, t):
    pts = [ob.full_nodes(prob, a)[1:-1] for a in range(prob.dim)]
    from oracle.forcing import eval_terms
    return eval_terms(terms, t, pts)


@pytest.mark.parametrize("dim,n", [(1, (9,)), (2, (7, 6)), (3, (5, 4, 6))])
def test_bilinear_data_is_a_steady_state(dim, n):
    l = _bilinear(dim)
    prob = _prob(dim, n, forcing=[], u0=l, boundary=l)
    d = Discretization(prob)
    W0 = d.initial()
    U0 = d.grid.to_nodal(W0)
    assert np.max(np.abs(U0 - _interior_values(prob, l, 0.0))) <= 1e-13
    tab = d.tables(prob.dt, prob.c_fine)
    W = sequential(d, W0, prob.t0, tab, 6)
    assert np.linalg.norm(W - W0) <= 1e-13 * np.linalg.norm(W0)


@pytest.mark.parametrize("dim,n", [(1, (11,)), (2, (7, 9))])
def test_moving_harmonic_lift_is_exact(dim, n):
    tau = wl.TimeFactor(poly=(1.0, 0.5, 0.2, 0.0))
    dtau = wl.TimeFactor(poly=(0.5, 0.4, 0.0, 0.0))
    l = _bilinear(dim)
    prob = _prob(dim, n, forcing=_with_time(l, dtau), u0=l, boundary=_with_time(l, tau),
                 c_fine=(0.0, 0.4, 0.9))
    d = Discretization(prob)
    tab = d.tables(prob.dt, prob.c_fine)
    W = sequential(d, d.initial(), prob.t0, tab, 7)
    t = prob.t0 + 7 * prob.dt
    ref = (1.0 + 0.5 * t + 0.2 * t * t) * _interior_values(prob, l, 0.0)
    assert np.max(np.abs(d.grid.to_nodal(W) - ref)) <= 1e-12


def _full_1d(n, lo, hi):
    """Closed-form full-grid Q1 matrices (n + 2 nodes)."""
    h = (hi - lo) / (n + 1)
    m = n + 2
    M = np.diag(np.full(m, 4.0 * h / 6.0)) + np.diag(np.full(m - 1, h / 6.0), 1) \
        + np.diag(np.full(m - 1, h / 6.0), -1)
    A = np.diag(np.full(m, 2.0 / h)) - np.diag(np.full(m - 1, 1.0 / h), 1) \
        - np.diag(np.full(m - 1, 1.0 / h), -1)
    M[0, 0] = M[-1, -1] = 2.0 * h / 6.0
    A[0, 0] = A[-1, -1] = 1.0 / h
    return M, A


def test_constant_data_matches_matrix_exponential():
    g = [wl.Term(0.8, ONE, (wl.SpaceFactor(kappa=2.0, phase=0.3), P(1.0, 0.0, 1.0))),
         wl.Term(0.3, ONE, (P(1.0), P(1.0)))]
    prob = _prob(2, (4, 3), D=0.6, N=1, J=5, s=2, T=0.7, forcing=[], u0=[], boundary=g)
    d = Discretization(prob)
    tab = d.tables(prob.dt, prob.c_fine)
    U = d.grid.to_nodal(sequential(d, d.initial(), prob.t0, tab, prob.J))
    # the whole system from closed-form full-grid matrices
    (M0, A0), (M1, A1) = [_full_1d(prob.n[a], prob.lo[a], prob.hi[a]) for a in range(2)]
    M = np.kron(M0, M1)
    A = np.kron(A0, M1) + np.kron(M0, A1)
    pts = [prob.lo[a] + (prob.hi[a] - prob.lo[a]) / (prob.n[a] + 1) * np.arange(prob.n[a] + 2)
           for a in range(2)]
    from oracle.forcing import eval_terms
    Gf = eval_terms(g, 0.0, pts)
    inner = np.zeros_like(Gf, dtype=bool)
    inner[1:-1, 1:-1] = True
    I, B = inner.ravel(), ~inner.ravel()
    GB = Gf.ravel()[B]
    MII, MIB, AII, AIB = M[np.ix_(I, I)], M[np.ix_(I, B)], A[np.ix_(I, I)], A[np.ix_(I, B)]
    U0 = np.linalg.solve(MII, -MIB @ GB)
    Uinf = np.linalg.solve(AII, -AIB @ GB)
    L = prob.D * np.linalg.solve(MII, AII)
    Ut = Uinf + scipy.linalg.expm(-prob.T * L) @ (U0 - Uinf)
    assert np.max(np.abs(U.ravel() - Ut)) <= 1e-12 * np.max(np.abs(Ut))


def test_data_vanishing_on_the_boundary_is_homogeneous():
    base = wl.tiny_problem(2, (9, 7), seed=5, N=2, J=3, s=3, u0_modes=1)
    sine = [wl.Term(1.3, wl.TimeFactor(omega=3.0),
                    (wl.sine_factor(2, base.lo[0], base.hi[0]), wl.sine_factor(1, base.lo[1], base.hi[1])))]
    with_b = base.with_(boundary=sine)
    d0, d1 = Discretization(base), Discretization(with_b)
    tab = d0.tables(base.dt, base.c_fine)
    W0 = sequential(d0, d0.initial(), base.t0, tab, 4)
    W1 = sequential(d1, d1.initial(), base.t0, tab, 4)
    # sin(k pi) at the far boundary node is ~1e-16, not 0: the coupling it
    # leaves is rounding-sized
    assert np.linalg.norm(W1 - W0) <= 1e-12 * np.linalg.norm(W0)


def test_manufactured_solution_converges_like_h2():
    """u = e^{-t} (1 + x)(1 + y^2) on (0,1)^2: f = u_t - D lap u =
    -e^{-t}(1 + x)(1 + y^2) - 2 D e^{-t}(1 + x), g = u on the boundary."""
    D = 0.5
    decay = wl.TimeFactor(alpha=-1.0)
    u = [wl.Term(1.0, decay, (P(1.0, 1.0), P(1.0, 0.0, 1.0)))]
    f = [wl.Term(-1.0, decay, (P(1.0, 1.0), P(1.0, 0.0, 1.0))),
         wl.Term(-2.0 * D, decay, (P(1.0, 1.0), P(1.0)))]
    errs = []
    for n in (7, 15, 31):
        prob = wl.Problem("manufactured", 2, (n, n), (0.0, 0.0), (1.0, 1.0), D, 0.0, 0.5, f, u,
                          2, 16, (0.0, 0.5, 1.0), (0.0, 0.5, 1.0), boundary=u)
        d = Discretization(prob)
        tab = d.tables(prob.dt, prob.c_fine)
        W = sequential(d, d.initial(), prob.t0, tab, prob.N * prob.J)
        errs.append(ob.l2_error_full(prob, d.grid.to_nodal(W), u, prob.T))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.85 <= r <= 2.15 for r in rates), (errs, rates)
