"""The FP64 oracle pinned to things other than itself.

Each check ties the oracle to a fact the paper or the mathematics fixes:
printed table values of the paper's worked examples, closed-form eigenpairs,
closed-form loads, brute-force matrix exponentials on tiny grids, exactness
for polynomial forcing, convergence rates, and the Parareal identities.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

import workloads as wl
from conftest import load_golden
from oracle import phi
from oracle import modal
from oracle.eife import Discretization, eife_step, l2_error, nodal_max_error, sequential
from oracle.fem import axis_basis, axis_matrices, Grid, gauss_legendre_01
from oracle.forcing import load_1d, load_field, load_field_elementwise, EXACT_Q
from oracle.parareal import parareal, sequential_coarse, sequential_fine


# --------------------------------------------------------------------------
# P1: 1D matrices, eigenpairs and the transform
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 7])
def test_axis_matrices_closed_form(n):
    lo, hi = 0.3, 1.7
    h = (hi - lo) / (n + 1)
    M, A = axis_matrices(n, lo, hi)
    T = np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)
    np.testing.assert_allclose(M, h / 6 * (4 * np.eye(n) + T), rtol=0, atol=1e-15)
    np.testing.assert_allclose(A, (2 * np.eye(n) - T) / h, rtol=1e-15, atol=1e-13)


@pytest.mark.parametrize("n,tol", [(7, 1e-13), (63, 2e-13), (255, 1e-12), (511, 3e-12)])
def test_axis_eigenpairs_closed_form(n, tol):
    lo, hi = 0.0, 1.0 + 0.5 * (n % 3)
    ax = axis_basis(n, lo, hi)
    h = (hi - lo) / (n + 1)
    k = np.arange(1, n + 1)
    th = k * np.pi / (n + 1)
    lam = 6.0 / h ** 2 * (1 - np.cos(th)) / (2 + np.cos(th))
    mu = h / 3 * (2 + np.cos(th))
    np.testing.assert_allclose(ax.lam, lam, rtol=tol)
    np.testing.assert_allclose(ax.mu, mu, rtol=1e-13)
    # M-orthonormal sine vectors
    j = np.arange(1, n + 1)[:, None]
    S = np.sqrt(2.0 / (n + 1)) * np.sin(j * k[None, :] * np.pi / (n + 1))
    np.testing.assert_allclose(ax.Q, S / np.sqrt(mu), atol=1e-9 * np.max(np.abs(ax.Q)))
    I = ax.Q.T @ ax.M @ ax.Q
    np.testing.assert_allclose(I, np.eye(n), atol=1e-12)
    L = ax.Q.T @ ax.A @ ax.Q
    np.testing.assert_allclose(np.diag(L), lam, rtol=tol)
    assert np.max(np.abs(L - np.diag(np.diag(L)))) <= 1e-10 * np.max(lam)


def test_spectral_norm_is_l2_norm():
    """||W||_2 equals the L2 norm of u_h (M-orthonormal coordinates)."""
    p = wl.tiny_problem(2, (9, 6), seed=3)
    d = Discretization(p)
    rng = np.random.default_rng(0)
    W = rng.normal(size=p.n)
    assert abs(l2_error(d, W, [], 0.0, q=3) - np.linalg.norm(W)) <= 1e-13 * np.linalg.norm(W)


def test_transform_roundtrip_3d():
    g = Grid((5, 7, 4), (0, 0, 0), (1, 2, 1.5))
    X = np.random.default_rng(1).normal(size=g.n)
    # U = Q W and W = Q^T M U
    np.testing.assert_allclose(g.to_spectral(g.mass_apply(g.to_nodal(X))), X, atol=1e-12)


# --------------------------------------------------------------------------
# P7: loads of sine modes (closed form) and the tensor factorisation
# --------------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 5, 20])
def test_sine_load_closed_form(k):
    n, lo, hi = 31, 0.25, 1.25
    sf = wl.sine_factor(k, lo, hi)
    h = (hi - lo) / (n + 1)
    kap = sf.kappa
    x = lo + h * np.arange(1, n + 1)
    exact = h * (np.sin(kap * h / 2) / (kap * h / 2)) ** 2 * np.sin(kap * (x - lo))
    np.testing.assert_allclose(load_1d(sf, n, lo, hi, EXACT_Q), exact, atol=1e-15)
    # q-point Gauss: C_q = 2h sum_g w_g xi_g cos(kappa h (1 - xi_g))
    xg, wg = gauss_legendre_01(3)
    cq = 2 * h * np.sum(wg * xg * np.cos(kap * h * (1 - xg)))
    np.testing.assert_allclose(load_1d(sf, n, lo, hi, 3), cq * np.sin(kap * (x - lo)), atol=1e-15)
    # 1-sparse spectral load with the closed-form coefficient
    g = Grid((n,), (lo,), (hi,))
    W = g.to_spectral(load_1d(sf, n, lo, hi, 3))
    th = k * np.pi / (n + 1)
    mu = h / 3 * (2 + np.cos(th))
    expect = cq * np.sqrt((n + 1) / 2) / np.sqrt(mu)
    assert abs(W[k - 1] - expect) <= 1e-12 * abs(expect)
    W[k - 1] = 0
    assert np.max(np.abs(W)) <= 1e-12 * abs(expect)


def test_polynomial_load_exact():
    """3-point Gauss integrates a quadratic times a hat exactly."""
    n, lo, hi = 9, 0.0, 2.0
    sf = wl.poly_factor(0.5, -1.0, 3.0)
    np.testing.assert_allclose(load_1d(sf, n, lo, hi, 3), load_1d(sf, n, lo, hi, EXACT_Q), rtol=1e-13)


@pytest.mark.parametrize("dim,n", [(2, (4, 3)), (3, (3, 2, 3))])
def test_elementwise_load_matches_factorised(dim, n):
    p = wl.tiny_problem(dim, n, seed=11, n_modes=2)
    p.forcing.append(wl.Term(0.7, wl.TimeFactor(alpha=0.3, poly=(1.0, 2.0, 0.0, 0.0)),
                             tuple(wl.poly_factor(1.0, 0.5, -0.25) for _ in range(dim))))
    g = Grid(p.n, p.lo, p.hi)
    a = load_field(g, p.forcing, 0.37, q=3)
    b = load_field_elementwise(g, p.forcing, 0.37, q=3)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-15)


# --------------------------------------------------------------------------
# P5: phi functions and b_i weights against their defining integrals
# --------------------------------------------------------------------------

def _lagrange(c, i, th):
    v = 1.0
    for m, cm in enumerate(c):
        if m != i:
            v *= (th - cm) / (c[i] - cm)
    return v


@pytest.mark.parametrize("c", [(0.0, 0.5), (0.0, 1 / 3, 2 / 3), (0.12, 0.4, 0.55, 0.93)])
@pytest.mark.parametrize("z", [1e-6, 3e-3, 0.4, 1.0, 7.5, 300.0])
def test_b_weights_vs_definition(c, z):
    E, b = phi.weights_scalar(z, c)
    assert abs(E - math.exp(-z)) <= 1e-16
    with mp.workdps(40):
        for i in range(len(c)):
            ref = mp.quad(lambda th: mp.exp(-z * (1 - th)) * _lagrange([mp.mpf(x) for x in c], i, th),
                          [0, 1 - min(1.0, 30.0 / z) if z > 30 else 0, 1])
            assert abs(b[i] - float(ref)) <= 1e-15 * max(1.0, abs(float(ref))), (i, b[i], float(ref))


def test_b_weights_special_values():
    # z -> 0: b_i = int l_i ; nodes {0, 1/2, 1} give Simpson's weights
    _, b = phi.weights_scalar(0.0, (0.0, 0.5, 1.0))
    np.testing.assert_allclose(b, [1 / 6, 4 / 6, 1 / 6], rtol=1e-15)
    # sum_i b_i = phi_1(-z) = (1 - e^{-z}) / z
    for z in (1e-4, 0.3, 12.0, 5000.0):
        _, b = phi.weights_scalar(z, (0.1, 0.35, 0.8))
        assert abs(sum(b) - (-math.expm1(-z)) / z) <= 1e-15 * max(1.0, sum(b))
    # large z: b_i ~ l_i(1)/z - l_i'(1)/z^2 + O(z^-3)
    c = (0.2, 0.5, 0.7)
    z = 1e6
    _, b = phi.weights_scalar(z, c)
    for i in range(3):
        li1 = _lagrange(c, i, 1.0)
        dl = (_lagrange(c, i, 1.0 + 1e-6) - _lagrange(c, i, 1.0 - 1e-6)) / 2e-6
        assert abs(b[i] - (li1 / z - dl / z ** 2)) <= 1e-16 * 1e3


@pytest.mark.parametrize("z", [1e-5, 0.01, 0.9, 2.0, 40.0])
def test_order_conditions(z):
    """sum_i b_i c_i^(j-1)/(j-1)! = phi_j(-z), j = 1..s (proof of Theorem 3.1)."""
    c = (0.05, 0.3, 0.62, 0.9)
    _, b = phi.weights_scalar(z, c)
    for j in range(1, 5):
        lhs = sum(b[i] * c[i] ** (j - 1) / math.factorial(j - 1) for i in range(4))
        with mp.workdps(60):
            ref = float(mp.quad(lambda th: mp.exp(-z * (1 - th)) * th ** (j - 1) / mp.factorial(j - 1), [0, 1]))
        assert abs(lhs - ref) <= 1e-14 * abs(ref)


# --------------------------------------------------------------------------
# P8: one EIFE step against dense matrix exponentials (tiny grids)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim,n,h", [(1, (7,), 0.05), (2, (5, 4), 0.3), (2, (3, 6), 0.01)])
def test_eife_step_bruteforce(dim, n, h):
    p = wl.tiny_problem(dim, n, seed=5, n_modes=3, s=3, D=0.7)
    d = Discretization(p)
    g = d.grid
    Md = g.dense_mass()
    Ad = g.dense_stiffness()
    L = p.D * np.linalg.solve(Md, Ad)                      # L_h in the nodal basis
    t = 0.21
    c = p.c_fine
    # eq. (2.7): b_i(-hL) = int_0^1 exp(-h(1-theta)L) l_i(theta) dtheta, by adaptive quadrature
    bmat = []
    for i in range(len(c)):
        fun = lambda th: (scipy.linalg.expm(-h * (1 - th) * L) * _lagrange(c, i, th)).ravel()
        val, _ = scipy.integrate.quad_vec(fun, 0.0, 1.0, epsabs=1e-15, epsrel=1e-13)
        bmat.append(val.reshape(L.shape))
    W0 = d.initial()
    U0 = g.to_nodal(W0).ravel()
    U1 = scipy.linalg.expm(-h * L) @ U0
    for i, ci in enumerate(c):
        F = load_field(g, p.forcing, t + ci * h).ravel()
        U1 = U1 + h * bmat[i] @ np.linalg.solve(Md, F)     # P_h f = M^{-1} F
    tab = d.tables(h, c)
    W1 = eife_step(d, W0, t, tab)
    got = g.to_nodal(W1).ravel()
    np.testing.assert_allclose(got, U1, rtol=1e-10, atol=1e-12 * np.max(np.abs(U1)))


# --------------------------------------------------------------------------
# P6: exact decay and exactness for polynomial-in-time forcing
# --------------------------------------------------------------------------

def test_free_decay_exact():
    """f = 0, u0 = a discrete sine mode: u_h(t) = e^{-D lambda t} u0 for any step."""
    p = wl.tiny_problem(2, (15, 11), seed=2)
    p = p.with_(forcing=[])
    d = Discretization(p)
    g = d.grid
    k1, k2 = 4, 9
    h1, h2 = g.axes[0].h, g.axes[1].h
    lam = sum(6 / hh ** 2 * (1 - math.cos(k * math.pi / (nn + 1))) / (2 + math.cos(k * math.pi / (nn + 1)))
              for hh, k, nn in ((h1, k1, 15), (h2, k2, 11)))
    W0 = np.zeros(p.n)
    W0[k1 - 1, k2 - 1] = 1.0
    for h, steps in ((0.5, 3), (1e-3, 40)):
        W = sequential(d, W0, 0.0, d.tables(h, p.c_fine), steps)
        expect = math.exp(-p.D * lam * h * steps)
        assert abs(W[k1 - 1, k2 - 1] - expect) <= 1e-12 * max(expect, 1e-300)
        W[k1 - 1, k2 - 1] = 0
        assert np.max(np.abs(W)) == 0.0


@pytest.mark.parametrize("s", [2, 3, 4])
def test_polynomial_forcing_integrated_exactly(s):
    """With s nodes, forcing polynomial in t of degree < s is integrated
    exactly (Lagrange interpolation is exact), so one step equals the Duhamel
    formula eq. (2.5) mode by mode."""
    rng = np.random.default_rng(s)
    c = wl.random_nodes(rng, s)
    poly = tuple(list(rng.normal(size=s)) + [0.0] * (4 - s))
    sf = (wl.sine_factor(2, 0.0, 1.0), wl.sine_factor(3, 0.0, 1.5))
    p = wl.Problem("poly", 2, (13, 10), (0.0, 0.0), (1.0, 1.5), 0.3, 0.0, 1.0,
                   [wl.Term(1.3, wl.TimeFactor(poly=poly), sf)], [], 1, 1, c, c)
    d = Discretization(p)
    t, h = 0.4, 0.7
    tab = d.tables(h, c)
    W0 = np.random.default_rng(9).normal(size=p.n)
    W1 = eife_step(d, W0, t, tab)
    ghat = d.spectral_forcing(0.0) / 1.3 / poly[0]         # spatial part of the load
    mu = p.D * d.lam
    for (a, b) in ((1, 2), (0, 0), (12, 9), (5, 3)):
        m = float(mu[a, b])
        with mp.workdps(40):
            duh = mp.quad(lambda sg: mp.exp(-m * (h - sg)) * 1.3 *
                          sum(poly[j] * (t + sg) ** j for j in range(s)), [0, h])
        expect = math.exp(-m * h) * W0[a, b] + float(duh) * ghat[a, b]
        assert abs(W1[a, b] - expect) <= 1e-13 * max(1.0, abs(expect)), (a, b)


def test_unconditional_stability():
    """No step restriction (Remark 3.1): with f = 0 the L2 norm never grows."""
    p = wl.tiny_problem(2, (20, 17), seed=4).with_(forcing=[])
    d = Discretization(p)
    W = np.random.default_rng(3).normal(size=p.n)
    for h in (1e-4, 1.0, 1e4):
        tab = d.tables(h, p.c_fine)
        assert np.all(tab.E <= 1.0) and np.all(tab.E >= 0.0)
        W2 = eife_step(d, W, 0.0, tab)
        assert np.linalg.norm(W2) <= np.linalg.norm(W)


# --------------------------------------------------------------------------
# P2-P3: the paper's printed errors
# --------------------------------------------------------------------------

def _paper_run(prob, K):
    d = Discretization(prob, q=EXACT_Q)
    tF = d.tables(prob.dt, prob.c_fine)
    tG = d.tables(prob.dT, prob.c_coarse)
    if K == 0:
        W = sequential(d, d.initial(), 0.0, tF, prob.N * prob.J)
    else:
        W = parareal(d, d.initial(), 0.0, prob.N, prob.J, tF, tG, K_max=K).iterates[-1][-1]
    return l2_error(d, W, prob.exact, prob.T)


def _rel_tol(digits):
    return 0.5 * 10.0 ** (1 - digits) * 1.05


def test_table1_spatial():
    gold = load_golden("table1_example_5_1.json")["spatial"]
    for ne, val, digits in gold["rows"]:
        err = _paper_run(wl.example_5_1(ne, gold["N"], gold["M"], 3), gold["K"])
        tol = _rel_tol(digits) if digits < 5 else 1.5e-4    # last printed digit
        assert abs(err - val) <= tol * val, (ne, err, val)


@pytest.mark.parametrize("s,rows", [(2, "EIFE-linear2"), (3, "EIFE-linear3")])
def test_table1_temporal_sequential(s, rows):
    gold = load_golden("table1_example_5_1.json")["temporal"]
    for NT, val in gold[rows][::3]:
        err = _paper_run(wl.example_5_1(gold["N_x"], NT, 1, s), 0)
        assert abs(err - val) <= 1.5e-4 * val, (NT, err, val)


def test_table1_temporal_parareal23():
    """PEIFE-linear23: G has 2 nodes, F has 3; k = 4 = N iterations."""
    gold = load_golden("table1_example_5_1.json")["temporal"]
    (N, M), val = gold["PEIFE-linear23"][1]
    err = _paper_run(wl.example_5_1(gold["N_x"], N, M, 3, s_coarse=2), 4)
    assert abs(err - val) <= 1.5e-4 * val


def test_table2_spatial():
    gold = load_golden("table2_example_5_2.json")["spatial"]
    for (nx, ny), val in gold["rows"][:3]:
        err = _paper_run(wl.example_5_2(nx, ny, gold["N"], gold["M"], 3), 2)
        assert abs(err - val) <= 5e-3 * val, (nx, err, val)


def test_table5_spatial():
    gold = load_golden("table5_example_5_3.json")["spatial"]
    for nx, val in gold["rows"][:2]:
        err = _paper_run(wl.example_5_3(nx, gold["N"], gold["M"], 3), 2)
        assert abs(err - val) <= 5e-3 * val, (nx, err, val)


def test_table4_errors_after_two_iterations():
    """Example 5.2 on 1024 x 512 elements, 8 x 8 steps, two stages: the L2
    and nodal L-infinity errors the paper prints for EIFE-linear2 and for
    PEIFE-linear22 after k = 2.  The forcing and u0 are the first Dirichlet
    sine on both axes, so only that coefficient is non-zero; the
    selected-mode oracle gives the sequential fine solution (which every
    Parareal iterate k >= 1 equals: see the Parareal pins below) on that
    mode, and the full-grid error norms evaluate it on all 1023 x 511 nodes."""
    gold = load_golden("table4_example_5_2.json")
    nx, ny = gold["elements"]
    p = wl.example_5_2(nx, ny, gold["N"], gold["M"], 2)
    modes = modal.forced_modes(p, q=EXACT_Q)
    assert modes.tolist() == [[0, 0]]
    W = np.zeros(p.n)
    W[0, 0] = modal.sequential_fine_modes(p, modes, q=EXACT_Q)[-1, 0]
    d = Discretization(p, q=EXACT_Q)
    l2, linf = l2_error(d, W, p.exact, p.T), nodal_max_error(d, W, p.exact, p.T)
    for row in ("EIFE-linear2", "PEIFE-linear22"):
        v2, vinf = gold["rows"][row]
        assert abs(l2 - v2) <= 3e-3 * v2, (row, l2, v2)
        assert abs(linf - vinf) <= 3e-3 * vinf, (row, linf, vinf)


def test_table7_errors_after_two_iterations():
    """Example 5.3 on 64^3 elements, 8 x 8 steps: PEIFE-linear22 after k = 2
    (the full-field oracle, Algorithm 1) and EIFE-linear2 (sequential), L2
    and nodal L-infinity errors against the paper's printed values."""
    gold = load_golden("table7_example_5_3.json")
    p = wl.example_5_3(gold["elements"], gold["N"], gold["M"], 2)
    d = Discretization(p, q=EXACT_Q)
    tF = d.tables(p.dt, p.c_fine)
    tG = d.tables(p.dT, p.c_coarse)
    W0 = d.initial()
    Wp = parareal(d, W0, 0.0, p.N, p.J, tF, tG, K_max=gold["K"]).iterates[-1][-1]
    modes = modal.forced_modes(p, q=EXACT_Q)
    Ws = np.zeros(p.n)
    Ws[tuple(modes.T)] = modal.sequential_fine_modes(p, modes, q=EXACT_Q)[-1]
    for row, W in (("PEIFE-linear22", Wp), ("EIFE-linear2", Ws)):
        v2, vinf = gold["rows"][row]
        l2, linf = l2_error(d, W, p.exact, p.T), nodal_max_error(d, W, p.exact, p.T)
        assert abs(l2 - v2) <= 9e-3 * v2, (row, l2, v2)
        assert abs(linf - vinf) <= 9e-3 * vinf, (row, linf, vinf)


# --------------------------------------------------------------------------
# P9: convergence rates (Lemma 3.1 / Theorem 3.1 / Theorem 4.5)
# --------------------------------------------------------------------------

def test_spatial_rate_h2():
    errs = []
    for n in (15, 31, 63):
        p = wl.config(1).with_(n=(n,), N=4, J=64, c_fine=(0.0, 1 / 3, 2 / 3))
        d = Discretization(p)
        W = sequential(d, d.initial(), 0.0, d.tables(p.dt, p.c_fine), p.N * p.J)
        errs.append(l2_error(d, W, p.exact, p.T))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.9 < r < 2.1 for r in rates), rates


@pytest.mark.parametrize("s", [2, 3])
def test_temporal_rate_random_nodes(s):
    """Error against the semi-discrete solution, which is closed-form per
    mode for an exponential time factor: W' = -mu W + g e^{alpha t}."""
    rng = np.random.default_rng(100 + s)
    c = wl.random_nodes(rng, s)
    sf = (wl.sine_factor(3, 0.0, 1.0),)
    alpha = 2.0
    p = wl.Problem("rate", 1, (31,), (0.0,), (1.0,), 0.05, 0.0, 1.0,
                   [wl.Term(1.0, wl.TimeFactor(alpha=alpha), sf)], [wl.Term(0.5, wl.TimeFactor(), sf)],
                   1, 1, c, c)
    d = Discretization(p)
    W0 = d.initial()
    g = d.spectral_forcing(0.0)
    mu = p.D * d.lam
    T = 1.0
    exact = np.exp(-mu * T) * W0 + g * (np.exp(alpha * T) - np.exp(-mu * T)) / (alpha + mu)
    errs = []
    for NT in (4, 8, 16, 32):
        W = sequential(d, W0, 0.0, d.tables(T / NT, c), NT)
        errs.append(np.linalg.norm(W - exact))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(s - 0.25 < r < s + 0.6 for r in rates[1:]), rates


# --------------------------------------------------------------------------
# P10: Parareal identities (Algorithm 1, Theorem 4.4)
# --------------------------------------------------------------------------

def _small_parareal(K, corrections=None, seed=8):
    p = wl.tiny_problem(2, (9, 7), seed=seed, N=5, J=4, s=3, n_modes=3, T=0.8)
    d = Discretization(p)
    tF = d.tables(p.dt, p.c_fine)
    tG = d.tables(p.dT, p.c_coarse)
    W0 = d.initial()
    r = parareal(d, W0, 0.0, p.N, p.J, tF, tG, K_max=K, corrections=corrections)
    return p, d, tF, tG, W0, r


def test_parareal_k0_is_sequential_coarse():
    p, d, tF, tG, W0, r = _small_parareal(1)
    np.testing.assert_array_equal(r.iterates[0], sequential_coarse(d, W0, 0.0, p.N, tG))


def test_parareal_reaches_sequential_fine_at_k_equal_N():
    """Theorem 4.4 (k >= N) and its strong form for this method: since G and
    F share the exact exponential and their forcing responses do not depend
    on the state, every iterate k >= 1 already equals the sequential fine
    solve (up to rounding)."""
    p, d, tF, tG, W0, r = _small_parareal(5)
    ref = sequential_fine(d, W0, 0.0, p.N, p.J, tF)
    scale = np.linalg.norm(ref)
    for k in range(1, len(r.iterates)):
        assert np.linalg.norm(r.iterates[k] - ref) <= 1e-14 * scale, k
    assert r.jumps[0] > 1e-6
    assert all(j <= 1e-14 for j in r.jumps[1:])
    # with a stopping tolerance the loop ends after the second fine pass
    _, _, _, _, _, r2 = _small_parareal(8)
    rr = parareal(d, W0, 0.0, p.N, p.J, tF, tG, K_max=8, tol=1e-8)
    assert rr.iterations == 2 and rr.converged


def test_parareal_residuals():
    """The residual ||U^{n+1,(k)} - F^J(U^{n,(k)})|| of each iterate:
    (i) every iterate k >= 1 is the sequential fine solve (strong form of
    Theorem 4.4), so its residual vanishes to rounding, while the coarse
    iterate's does not; (ii) with f = 0, G and F apply the same exact
    exponential (e^{-dT mu} = (e^{-dt mu})^J), so even the coarse iterate has
    no residual; (iii) when e^{-dT mu} underflows on every mode, eq. (2.8)
    gives U^{n+1,(1)} - U^{n+1,(0)} = F^J(U^{n,(0)}) - U^{n+1,(0)}: the first
    jump and the coarse residual are the same vector."""
    p, d, tF, tG, W0, r = _small_parareal(3)
    assert len(r.residuals) == 3 and r.residuals[0] > 1e-6
    assert all(v <= 1e-14 for v in r.residuals[1:]), r.residuals
    # (ii)
    p0 = p.with_(forcing=[])
    d0 = Discretization(p0)
    r0 = parareal(d0, d0.initial(), 0.0, p0.N, p0.J, d0.tables(p0.dt, p0.c_fine),
                  d0.tables(p0.dT, p0.c_coarse), K_max=2)
    assert np.linalg.norm(d0.initial()) > 1e-3
    assert all(v <= 1e-14 for v in r0.residuals), r0.residuals
    # (iii) lambda_1 D dT = pi^2 * 10 * 0.5 ~ 49: e^{-49} ~ 5e-22
    ps = wl.tiny_problem(1, (7,), seed=5, N=4, J=3, s=3, n_modes=3, D=10.0, T=2.0)
    ds = Discretization(ps)
    assert np.max(np.exp(-ps.dT * ps.D * ds.lam)) < 1e-20
    rs = parareal(ds, ds.initial(), 0.0, ps.N, ps.J, ds.tables(ps.dt, ps.c_fine),
                  ds.tables(ps.dT, ps.c_coarse), K_max=1)
    U0, U1 = rs.iterates
    jump_abs = rs.jumps[0] * np.linalg.norm(U1[1:])
    res_abs = rs.residuals[0] * np.linalg.norm(U0[1:])
    assert jump_abs > 1e-3 and abs(jump_abs - res_abs) <= 1e-12 * res_abs


def test_parareal_state_independent_correction_changes_only_k0():
    p, d, tF, tG, W0, r = _small_parareal(3)
    rng = np.random.default_rng(4)
    corr = [rng.normal(size=p.n) * 0.1 for _ in range(p.N)]
    r2 = parareal(d, W0, 0.0, p.N, p.J, tF, tG, K_max=3, corrections=corr)
    assert np.linalg.norm(r2.iterates[0] - r.iterates[0]) > 1e-3
    for k in (1, 2, 3):
        np.testing.assert_allclose(r2.iterates[k], r.iterates[k], atol=1e-14 * np.linalg.norm(r.iterates[k]))


# --------------------------------------------------------------------------
# P11: the oracle MLP of the learned coarse correction
# --------------------------------------------------------------------------

def test_mlp_backward_matches_central_differences():
    from oracle import mlp
    rng = np.random.default_rng(0)
    theta = mlp.init_params(3)
    x = rng.normal(size=(7, mlp.N_IN))
    t = rng.normal(size=7)
    L, grad = mlp.loss_and_grad(theta, x, t)
    assert abs(L - mlp.loss(theta, x, t)) <= 1e-15 * max(1.0, L)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [mlp.N_PARAMS - 1, 0, 12 * 64 + 5]])   # b4, W1[0,0], b1[5]
    for i in idx:
        h = 1e-6 * max(1.0, abs(theta[i]))
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp.loss(tp, x, t) - mlp.loss(tm, x, t)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, grad[i])


def test_mlp_gelu_and_features():
    from oracle import mlp
    from scipy.stats import norm
    xs = np.linspace(-6, 6, 41)
    np.testing.assert_allclose(mlp.gelu(xs), xs * norm.cdf(xs), rtol=1e-14, atol=1e-300)
    z = np.array([1e-8, 1e-4, 0.5, 3.0, 400.0])
    f = mlp.z_features(z)
    np.testing.assert_allclose(f[:, 1], np.exp(-z), rtol=1e-15)
    for k, zk in enumerate(z):
        with mp.workdps(50):
            zz = mp.mpf(zk)
            p1 = (1 - mp.exp(-zz)) / zz
            p2 = (zz - 1 + mp.exp(-zz)) / zz ** 2
        assert abs(f[k, 2] - float(p1)) <= 1e-14 * float(p1)
        assert abs(f[k, 3] - 2 * float(p2)) <= 1e-13 * 2 * float(p2)
    # scaling the samples leaves the inputs unchanged and scales s
    smp = np.random.default_rng(1).normal(size=(3, 8))
    x1, s1 = mlp.features(np.full(3, 0.3), smp)
    x2, s2 = mlp.features(np.full(3, 0.3), 1e-7 * smp)
    np.testing.assert_allclose(x1, x2, rtol=1e-12)
    np.testing.assert_allclose(s2, 1e-7 * s1, rtol=1e-13)
    # the basis is orthonormal and polynomial: q_j has degree j
    Q = mlp.sample_basis()
    np.testing.assert_allclose(Q.T @ Q, np.eye(8), atol=1e-14)
    t = (np.arange(8) - 3.5) / 3.5
    for deg in range(4):
        c = (t ** deg) @ Q
        assert np.max(np.abs(c[deg + 1:])) <= 1e-13 and c[deg] > 0
    # samples of a cubic in time have no high part: s = 0 and no correction
    cub = 0.3 - 1.2 * t + 0.7 * t ** 3
    _, s_cub = mlp.features(np.array([0.5]), cub[None, :])
    assert s_cub[0] <= 1e-14
    theta = mlp.init_params(0)
    assert np.all(np.abs(mlp.correction(theta, np.full(1, 0.3), cub[None, :], 0.1)) <= 1e-14)
    assert np.all(mlp.correction(theta, np.full(2, 0.3), np.zeros((2, 8)), 0.1) == 0.0)


def test_bf16_rounding_reference():
    from oracle import mlp
    v = np.array([1.0, 1.00390625, 1.001953125, 1.005859375, -3.14159265, 1e-30])
    r = mlp.to_bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0                            # 1 + 2^-8 is a tie -> even (1.0)
    assert r[2] == 1.0                                            # below half an ulp
    assert r[3] == 1.0078125                                      # above half an ulp
    assert abs(r[4] + 3.140625) < 1e-12
