"""HIP library vs the FP64 CPU oracle, element by element, through the C ABI.

Tolerance: the FP64 path must match the oracle to 1e-11 relative L2 (the
stated target for the FP64 path); tables, loads and single propagations are
held to tighter bounds that follow from FP64 rounding (summation order of
the transforms and of the stage sums differs from the oracle's).
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle.eife import Discretization, eife_step
from oracle.parareal import coarse_step, fine_prop, parareal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FP64_TOL = 1e-11


def _peifem():
    from paper_2412_01138_amd import peifem
    return peifem


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda:0")


GRIDS = [
    (1, (63,)),           # a single padded tile
    (1, (70,)),           # ragged tail
    (2, (37, 21)),
    (2, (65, 33)),        # several tiles + ragged tail on both axes
    (3, (9, 33, 7)),
]


@pytest.mark.parametrize("dim,n", GRIDS)
@pytest.mark.parametrize("s", [2, 3, 4])
def test_phi_tables(dim, n, s):
    pe = _peifem()
    prob = wl.tiny_problem(dim, n, seed=10 + s, s=s, D=0.37)
    g = pe.Grid.from_problem(prob)
    d = Discretization(prob)
    # The library evaluates lambda in closed form; the oracle takes it from
    # dense LAPACK, accurate to LAM_REL (pinned against the closed form).  A
    # relative change delta in z = h D lambda moves exp(-z) by z e^{-z} delta
    # and b_i(z) by at most ~delta * max|b| (|z b_i'(z)| <= max|b_i|).
    LAM_REL = 3e-12
    for h in (1e-4, 0.03, 2.5):
        E, B = g.phi_tables(h, prob.c_fine)
        tab = d.tables(h, prob.c_fine)
        E = E.cpu().numpy()
        B = B.cpu().numpy()
        z = h * prob.D * d.lam
        assert np.all(np.abs(E - tab.E) <= 4e-16 + LAM_REL * z * tab.E), h
        scale = np.max(np.abs(h * tab.b))
        assert np.max(np.abs(B - h * tab.b)) <= (1e-13 + 4 * LAM_REL) * scale, h


@pytest.mark.parametrize("s", [5, 6, 7, 8])
@pytest.mark.parametrize("nodes", ["uniform", "random"])
def test_phi_tables_many_stages(s, nodes):
    """s = 5..8 stages.  b_i = sum_j a_ij j! phi_{j+1}(-z) sums terms much
    larger than b_i when the Lagrange coefficients a_ij are large (up to
    ~1e8 at s = 8), so a double evaluation carries an error of a few ulps of
    sum_j |a_ij j! phi_{j+1}|, not of |b_i|: that sum, taken from the
    oracle's own Lagrange coefficients and phi values, sets the bound."""
    import mpmath as mp
    from oracle import phi as ophi
    pe = _peifem()
    prob = wl.tiny_problem(2, (37, 21), seed=10 + s, s=s, D=0.37)
    c = wl.uniform_nodes(s) if nodes == "uniform" else prob.c_fine
    g = pe.Grid.from_problem(prob)
    d = Discretization(prob)
    a = ophi.lagrange_coeffs(c)
    A = np.array([[float(abs(a[i][j]) * mp.factorial(j)) for j in range(s)] for i in range(s)])
    LAM_REL = 3e-12
    for h in (1e-4, 0.03, 2.5):
        E, B = g.phi_tables(h, c)
        tab = d.tables(h, c)
        E = E.cpu().numpy()
        B = B.cpu().numpy()
        z = h * prob.D * d.lam
        assert np.all(np.abs(E - tab.E) <= 4e-16 + LAM_REL * z * tab.E), h
        uz, inv = np.unique(z.ravel(), return_inverse=True)
        with mp.workdps(40):
            ph = np.array([[float(ophi.phi_mp(j, -mp.mpf(float(v)))) for j in range(1, s + 1)]
                           for v in uz])
        mag = (ph @ A.T)[inv].T.reshape((s,) + z.shape)      # sum_j |a_ij j! phi_{j+1}|
        scale = np.max(np.abs(h * tab.b))
        bound = (1e-13 + 4 * LAM_REL) * scale + 16 * s * 2.0 ** -52 * h * mag
        assert np.all(np.abs(B - h * tab.b) <= bound), (h, float(np.max(np.abs(B - h * tab.b) / bound)))


@pytest.mark.parametrize("dim,n", GRIDS)
def test_project_initial_value(dim, n):
    pe = _peifem()
    prob = wl.tiny_problem(dim, n, seed=4, u0_modes=3)
    prob.u0.append(wl.Term(0.6, wl.TimeFactor(),
                           tuple(wl.poly_factor(0.2, 1.0, -0.7) for _ in range(dim))))
    g = pe.Grid.from_problem(prob)
    W = g.project(prob.u0).cpu().numpy()
    ref = Discretization(prob).initial()
    assert rel(W, ref) <= 1e-13


def _fine_case(dim, n, N, J, s, seed=0, n_modes=4):
    prob = wl.tiny_problem(dim, n, seed=seed, s=s, N=N, J=J, n_modes=n_modes, T=0.9)
    d = Discretization(prob)
    rng = np.random.default_rng(seed + 1)
    Uin = rng.normal(size=(N,) + prob.n)
    return prob, d, Uin


@pytest.mark.parametrize("dim,n,N,J,s", [
    (1, (63,), 8, 16, 2),
    (1, (100,), 3, 5, 3),
    (2, (37, 70), 3, 4, 3),
    (2, (64, 64), 2, 3, 4),
    (3, (9, 33, 7), 2, 3, 4),
    (3, (20, 5, 40), 2, 2, 2),
    # axes with n = 2^m - 1 take the second even/odd level
    (2, (63, 63), 2, 3, 3),
    (2, (127, 40), 2, 2, 4),
    (2, (255, 63), 1, 2, 3),
    (3, (63, 127, 31), 1, 2, 3),
    (3, (127, 63, 63), 1, 2, 2),
    # last axis with n = 127 / 255: the generating pass takes a third level
    (2, (40, 127), 2, 2, 3),
    (2, (63, 255), 2, 2, 4),
    (2, (255, 255), 1, 2, 2),
    (3, (9, 20, 127), 2, 2, 3),
    # 511-node last axis: the generating pass with Kh = 256 (two fold levels)
    (2, (31, 511), 1, 2, 4),
    # one stage (every field takes the decay), and one field per slice
    (2, (127, 40), 2, 3, 1),
    (2, (63, 255), 2, 1, 1),
])
def test_fine_propagate(dim, n, N, J, s):
    pe = _peifem()
    prob, d, Uin = _fine_case(dim, n, N, J, s)
    g = pe.Grid.from_problem(prob)
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    out = g.fine_propagate(_dev(Uin), prob.t0, prob.dT, J, prob.c_fine, E, B).cpu().numpy()
    tab = d.tables(prob.dt, prob.c_fine)
    ref = np.stack([fine_prop(d, Uin[k], prob.t0 + k * prob.dT, tab, J) for k in range(N)])
    assert rel(out, ref) <= 1e-12


@pytest.mark.parametrize("n", [(511, 63), (511, 511)])
def test_fine_propagate_511_sampled(n):
    """511-node axes (the workload-4 kernels: the generating pass with
    Kh = 256, the fused axis-0 update with one half per block, Q = 128) on
    a random state and a forcing that reaches every mode (sine terms plus a
    polynomial term, whose 1D loads are dense in both parities): every
    output coefficient at 400 random modes, plus all modes the sine terms
    force, against the selected-mode oracle."""
    from oracle import modal
    pe = _peifem()
    prob = wl.tiny_problem(2, n, seed=61, s=4, N=2, J=2, n_modes=4, T=0.9)
    forced = modal.forced_modes(prob)                 # the sine terms' modes
    prob.forcing.append(wl.Term(0.8, wl.TimeFactor(omega=3.0, poly=(1.0, 0.5, 0.0, 0.0)),
                                (wl.poly_factor(0.2, 1.0, -0.7), wl.poly_factor(1.0, -0.3, 0.1))))
    rng = np.random.default_rng(62)
    Uin = rng.normal(size=(prob.N,) + prob.n)
    g = pe.Grid.from_problem(prob)
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    out = g.fine_propagate(_dev(Uin), prob.t0, prob.dT, prob.J, prob.c_fine, E, B).cpu().numpy()
    rng = np.random.default_rng(63)
    extra = np.stack([rng.integers(0, prob.n[a], 400) for a in range(2)], axis=1)
    modes = np.unique(np.concatenate([forced, extra]), axis=0)
    fine = modal.ModalFine(prob, modes)
    idx = tuple(modes.T)
    for k in range(prob.N):
        ref = fine.propagate(Uin[k][idx], prob.t0 + k * prob.dT)
        got = out[k][idx]
        assert rel(got, ref) <= 1e-12, k
        # the forcing's share of each coefficient is resolved too
        free = fine.E ** prob.J * Uin[k][idx]
        assert rel(got - free, ref - free) <= 1e-11, k


@pytest.mark.parametrize("s", [5, 6, 7, 8])
def test_fine_propagate_many_stages(s):
    """s = 5..8 stage rules with the paper's uniform nodes c_i = (i-1)/s
    (the b_i carry up to ~1e4 ulps of cancellation at s = 8, see
    test_phi_tables_many_stages: the FP64 bar 1e-11 still holds)."""
    pe = _peifem()
    prob, d, Uin = _fine_case(2, (63, 127), 2, 2, s, seed=50 + s)
    prob = prob.with_(c_fine=wl.uniform_nodes(s), c_coarse=wl.uniform_nodes(s))
    g = pe.Grid.from_problem(prob)
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    out = g.fine_propagate(_dev(Uin), prob.t0, prob.dT, prob.J, prob.c_fine, E, B).cpu().numpy()
    tab = d.tables(prob.dt, prob.c_fine)
    ref = np.stack([fine_prop(d, Uin[k], prob.t0 + k * prob.dT, tab, prob.J) for k in range(2)])
    assert rel(out, ref) <= FP64_TOL


@pytest.mark.parametrize("dim,n", [(1, (45,)), (2, (37, 70)), (3, (9, 20, 33))])
def test_fine_propagate_many_terms(dim, n):
    """More forcing terms than the fused quadrature path takes: the load
    vectors are written by the separate quadrature kernel instead."""
    pe = _peifem()
    prob, d, Uin = _fine_case(dim, n, 2, 3, 3, seed=7, n_modes=40)
    g = pe.Grid.from_problem(prob)
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    out = g.fine_propagate(_dev(Uin), prob.t0, prob.dT, prob.J, prob.c_fine, E, B).cpu().numpy()
    tab = d.tables(prob.dt, prob.c_fine)
    ref = np.stack([fine_prop(d, Uin[k], prob.t0 + k * prob.dT, tab, prob.J) for k in range(2)])
    assert rel(out, ref) <= 1e-12


def test_fine_propagate_batching_is_exact():
    """Smaller workspaces split the fields into more batches; every field is
    still computed by the same kernels, so the output is bitwise identical."""
    pe = _peifem()
    prob, d, Uin = _fine_case(2, (40, 33), 5, 6, 3, seed=5)
    g = pe.Grid.from_problem(prob)
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    U = _dev(Uin)
    full = g.fine_propagate(U, prob.t0, prob.dT, prob.J, prob.c_fine, E, B).cpu().numpy()
    for fields in (3, 7, 15, 2 * 5 * 3):
        work = g.workspace(g.fine_workspace_bytes(fields))
        part = g.fine_propagate(U, prob.t0, prob.dT, prob.J, prob.c_fine, E, B, work=work)
        np.testing.assert_array_equal(part.cpu().numpy(), full)


@pytest.mark.parametrize("dim,n,N,J,s", [
    (2, (63, 63), 3, 4, 3),       # Q = 16, both halves per block
    (2, (255, 40), 2, 3, 4),      # Q = 64 (the 255-node axes)
    (2, (191, 31), 2, 2, 2),      # Q = 48
    (2, (319, 17), 1, 2, 3),      # Q = 80, one half per block
    (2, (383, 12), 1, 2, 3),      # Q = 96
    (2, (511, 20), 1, 2, 2),      # Q = 128 (the 511-node axes)
    (3, (127, 20, 9), 2, 2, 3),   # Q = 32, ragged inner axes
])
def test_fused_axis0_update_matches_separate_kernels(dim, n, N, J, s):
    """Axis 0 with two fold levels: the axis-0 pass fused with the update
    gives bitwise the result of the separate pass + update kernels (which run
    when the workspace has no room for the update tables), and both match the
    oracle."""
    pe = _peifem()
    prob, d, Uin = _fine_case(dim, n, N, J, s, seed=9)
    g = pe.Grid.from_problem(prob)
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    U = _dev(Uin)
    fused = g.fine_propagate(U, prob.t0, prob.dT, J, prob.c_fine, E, B).cpu().numpy()
    per_field = g.fine_workspace_bytes(2) - g.fine_workspace_bytes(1)
    work = g.workspace(3 * 256 + per_field * s)
    sep = g.fine_propagate(U, prob.t0, prob.dT, J, prob.c_fine, E, B, work=work).cpu().numpy()
    np.testing.assert_array_equal(fused, sep)
    tab = d.tables(prob.dt, prob.c_fine)
    ref = np.stack([fine_prop(d, Uin[k], prob.t0 + k * prob.dT, tab, J) for k in range(N)])
    assert rel(fused, ref) <= 1e-12


def test_fused_update_batching_is_exact():
    """With the fused axis-0 pass + update a smaller workspace takes whole
    slices per batch (all J steps), or fewer steps of all slices when not
    even one slice fits; every mode still sees the same arithmetic, so the
    output is bitwise identical to the one-batch result."""
    pe = _peifem()
    prob, d, Uin = _fine_case(2, (63, 40), 5, 4, 3, seed=6)
    g = pe.Grid.from_problem(prob)
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    U = _dev(Uin)
    full = g.fine_propagate(U, prob.t0, prob.dT, prob.J, prob.c_fine, E, B).cpu().numpy()
    for fields in (12, 24, 36, 48, 5 * 3, 3):
        work = g.workspace(g.fine_workspace_bytes(fields))
        part = g.fine_propagate(U, prob.t0, prob.dT, prob.J, prob.c_fine, E, B, work=work)
        np.testing.assert_array_equal(part.cpu().numpy(), full)


def test_fine_propagate_without_forcing_is_pure_decay():
    pe = _peifem()
    prob, d, Uin = _fine_case(2, (17, 12), 3, 5, 3)
    prob = prob.with_(forcing=[])
    g = pe.Grid.from_problem(prob)
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    out = g.fine_propagate(_dev(Uin), prob.t0, prob.dT, prob.J, prob.c_fine, E, B).cpu().numpy()
    lam = Discretization(prob).lam
    ref = Uin * np.exp(-prob.D * lam * prob.dT)[None]
    assert rel(out, ref) <= 1e-14


@pytest.mark.parametrize("dim,n", [(1, (63,)), (2, (37, 21)), (3, (9, 12, 7))])
def test_coarse_sweep_plain_and_correction(dim, n):
    pe = _peifem()
    N = 5
    prob = wl.tiny_problem(dim, n, seed=21, N=N, J=2, s=3)
    d = Discretization(prob)
    g = pe.Grid.from_problem(prob)
    EG, BG = g.phi_tables(prob.dT, prob.c_coarse)
    tabG = d.tables(prob.dT, prob.c_coarse)
    rng = np.random.default_rng(3)
    U0 = rng.normal(size=prob.n)
    corr = rng.normal(size=(N,) + prob.n) * 0.01
    # plain sweep with a learned-style correction
    U = torch.zeros((N + 1,) + prob.n, dtype=torch.float64, device="cuda:0")
    U[0] = _dev(U0)
    r = torch.empty((N,) + prob.n, dtype=torch.float64, device="cuda:0")
    g.coarse_sweep(U, prob.t0, prob.dT, prob.c_coarse, EG, BG, r, corr=_dev(corr))
    ref = [U0]
    for k in range(N):
        ref.append(coarse_step(d, ref[k], prob.t0 + k * prob.dT, tabG, corr[k]))
    ref = np.stack(ref)
    assert rel(U.cpu().numpy(), ref) <= 1e-13
    # r_n on its own: the coarse forcing response of each slice
    rr = np.stack([eife_step(d, np.zeros(prob.n), prob.t0 + k * prob.dT, tabG) for k in range(N)])
    assert rel(r.cpu().numpy(), rr) <= 1e-12     # table accuracy bound (see test_phi_tables)
    # correction sweep (eq. 2.8) with norms
    Uprev = U.clone()
    Fout = rng.normal(size=(N,) + prob.n)
    Unew = torch.zeros_like(U)
    Unew[0] = U[0]
    norms = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    g.coarse_sweep(Unew, prob.t0, prob.dT, prob.c_coarse, EG, BG, r, compute_r=False,
                   corr=_dev(corr), Uprev=Uprev, Fout=_dev(Fout), norms=norms)
    up = Uprev.cpu().numpy()
    refn = [U0]
    for k in range(N):
        gnew = coarse_step(d, refn[k], prob.t0 + k * prob.dT, tabG, corr[k])
        gold = coarse_step(d, up[k], prob.t0 + k * prob.dT, tabG, corr[k])
        refn.append(gnew + Fout[k] - gold)
    refn = np.stack(refn)
    got = Unew.cpu().numpy()
    assert rel(got, refn) <= 1e-13
    nrm = norms.cpu().numpy()
    assert abs(nrm[0] - np.sum((refn[1:] - up[1:]) ** 2)) <= 1e-12 * nrm[0]
    assert abs(nrm[1] - np.sum(refn[1:] ** 2)) <= 1e-12 * nrm[1]
    # residual of the previous iterate against the given fine outputs
    res2 = np.sum((up[1:] - Fout) ** 2)
    assert abs(nrm[2] - res2) <= 1e-12 * res2
    # the FP64 reduction order is fixed: a second run is bitwise identical
    norms2 = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    Unew2 = torch.zeros_like(U)
    Unew2[0] = U[0]
    g.coarse_sweep(Unew2, prob.t0, prob.dT, prob.c_coarse, EG, BG, r, compute_r=False,
                   corr=_dev(corr), Uprev=Uprev, Fout=_dev(Fout), norms=norms2)
    assert torch.equal(norms, norms2) and torch.equal(Unew, Unew2)


def _oracle_parareal(prob, K, tol):
    d = Discretization(prob)
    tF = d.tables(prob.dt, prob.c_fine)
    tG = d.tables(prob.dT, prob.c_coarse)
    return parareal(d, d.initial(), prob.t0, prob.N, prob.J, tF, tG, K_max=K, tol=tol)


@pytest.mark.parametrize("case", ["cfg1", "2d", "3d", "2d-uneven-pq"])
def test_parareal_solve(case):
    pe = _peifem()
    if case == "cfg1":
        prob = wl.config(1)
    elif case == "2d":
        prob = wl.tiny_problem(2, (45, 38), seed=31, N=6, J=5, s=3, u0_modes=2)
    elif case == "3d":
        prob = wl.tiny_problem(3, (11, 17, 9), seed=32, N=4, J=3, s=4, u0_modes=2)
    else:
        prob = wl.tiny_problem(2, (30, 26), seed=33, N=5, J=4, s=3, u0_modes=1)
        prob = prob.with_(c_coarse=(0.0, 1.0))
    g, U, rep = pe.solve_problem(prob, K_max=prob.K_max, tol=1e-8)
    r = _oracle_parareal(prob, prob.K_max, 1e-8)
    assert rep.iterations == r.iterations and bool(rep.converged) == r.converged
    assert rel(U.cpu().numpy(), r.iterates[-1]) <= FP64_TOL
    assert abs(rep.jumps[0] - r.jumps[0]) <= 1e-9 * r.jumps[0]
    for k in range(1, r.iterations):
        assert rep.jumps[k] <= 1e-13
    # residuals of iterates 0..K-1: the coarse iterate's against the oracle,
    # the later ones vanish to rounding (every iterate k >= 1 is the
    # sequential fine solve)
    assert abs(rep.residuals[0] - r.residuals[0]) <= 1e-12 * r.residuals[0]
    for k in range(1, r.iterations):
        assert rep.residuals[k] <= 1e-13 and r.residuals[k] <= 1e-13
    assert all(rep.residuals[k] == 0.0 for k in range(r.iterations, pe.PE_MAX_ITERS))
    # the FP64 reductions have a fixed order: a second solve is bitwise equal
    _, U2, rep2 = pe.solve_problem(prob, K_max=prob.K_max, tol=1e-8)
    assert list(rep2.jumps) == list(rep.jumps) and list(rep2.residuals) == list(rep.residuals)
    assert torch.equal(U, U2)


def test_parareal_fixed_iterations_track_every_iterate():
    """K_max = 1, 2, 3 with tol = 0: each final iterate equals the oracle's."""
    pe = _peifem()
    prob = wl.tiny_problem(2, (33, 20), seed=40, N=4, J=3, s=2, u0_modes=1)
    r = _oracle_parareal(prob, 3, 0.0)
    for K in (1, 2, 3):
        g, U, rep = pe.solve_problem(prob, K_max=K, tol=0.0)
        assert rep.iterations == K and not rep.converged
        assert rel(U.cpu().numpy(), r.iterates[K]) <= FP64_TOL


def test_learned_style_correction_leaves_converged_answer():
    pe = _peifem()
    prob = wl.tiny_problem(2, (25, 19), seed=41, N=5, J=3, s=3, u0_modes=1)
    rng = np.random.default_rng(0)
    corr = _dev(rng.normal(size=(prob.N,) + prob.n) * 1e-3)
    _, U1, rep1 = pe.solve_problem(prob, K_max=3, tol=0.0)
    _, U2, rep2 = pe.solve_problem(prob, K_max=3, tol=0.0, corr=corr)
    assert rel(U2.cpu().numpy(), U1.cpu().numpy()) <= 1e-13
    assert abs(rep1.jumps[0] - rep2.jumps[0]) > 1e-6 * rep1.jumps[0]


def test_argument_errors():
    pe = _peifem()
    prob = wl.tiny_problem(2, (9, 8), seed=1)
    g = pe.Grid.from_problem(prob)
    with pytest.raises(pe.PeifemError) as ei:
        g.phi_tables(0.1, (0.3, 0.3))
    assert ei.value.status == pe.PE_E_ARG
    E, B = g.phi_tables(0.1, prob.c_fine)
    U = torch.zeros((2,) + prob.n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(pe.PeifemError) as ei:
        g.fine_propagate(U, 0.0, 0.1, 2, prob.c_fine, E, B, work=g.workspace(64))
    assert ei.value.status == pe.PE_E_WORKSPACE
    with pytest.raises(pe.PeifemError) as ei:
        g.fine_propagate(U, 0.0, 0.1, 2, prob.c_fine, E, B, Uout=U)
    assert ei.value.status == pe.PE_E_ARG
