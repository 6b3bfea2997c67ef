"""Non-homogeneous Dirichlet data (pe_set_boundary, pe_project_state) on the
GPU against the FP64 oracle (oracle/boundary.py), through the C ABI.

Bars as for homogeneous data: single propagations 1e-12 relative L2, the
initial-state projection 1e-13, Parareal answers 1e-11 (FP64); 2e-5 on the
split-bf16 path.  The data are time-dependent and non-zero on every face
(polynomial and shifted-sine factors), so every coupling term is exercised.
"""
import numpy as np
import pytest

import workloads as wl
from oracle.eife import Discretization, sequential
from oracle.parareal import fine_prop, parareal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

P = wl.poly_factor


def _pe():
    from paper_2412_01138_amd import peifem
    return peifem


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda:0")


def _data(dim):
    """Two data terms, non-zero on every face, time-dependent."""
    f1 = [P(1.0, 0.5, -0.2), wl.SpaceFactor(kappa=1.3, phase=0.4), P(0.8, -0.3)]
    f2 = [wl.SpaceFactor(kappa=2.1, phase=0.2), P(0.3, 1.0), wl.SpaceFactor(kappa=0.7, phase=1.1)]
    return [wl.Term(0.7, wl.TimeFactor(omega=2.0, phase=0.3), tuple(f1[:dim])),
            wl.Term(-0.4, wl.TimeFactor(alpha=-0.5, poly=(1.0, 0.3, 0.0, 0.0)), tuple(f2[:dim]))]


def _case(dim, n, N=2, J=3, s=3, seed=0, precision="fp64"):
    prob = wl.tiny_problem(dim, n, seed=seed, s=s, N=N, J=J, T=0.9, precision=precision)
    return prob.with_(boundary=_data(dim))


@pytest.mark.parametrize("dim,n,transform,precision", [
    (1, (30,), "dense", "fp64"),
    (2, (37, 21), "dense", "fp64"),
    (2, (63, 63), "dense", "fp64"),            # fused axis-0 pass + update
    (3, (9, 12, 7), "dense", "fp64"),
    (2, (63, 127), "fft", "fp64"),
    (3, (20, 9, 33), "dense", "split_bf16"),
])
def test_boundary_fine_propagate(dim, n, transform, precision):
    pe = _pe()
    print(f"boundary fine propagate dim {dim} n {n} {transform} {precision}", flush=True)
    prob = _case(dim, n, seed=4, precision=precision)
    d = Discretization(prob)
    rng = np.random.default_rng(5)
    Uin = rng.normal(size=(prob.N,) + prob.n)
    g = pe.Grid.from_problem(prob, transform=transform)
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    dt = torch.float64 if precision == "fp64" else torch.float32
    out = g.fine_propagate(_dev(Uin, dt), prob.t0, prob.dT, prob.J, prob.c_fine, E, B)
    tab = d.tables(prob.dt, prob.c_fine)
    ref = np.stack([fine_prop(d, Uin[k], prob.t0 + k * prob.dT, tab, prob.J)
                    for k in range(prob.N)])
    assert rel(out.double().cpu().numpy(), ref) <= (1e-12 if precision == "fp64" else 2e-5)


@pytest.mark.parametrize("dim,n", [(1, (25,)), (2, (37, 21)), (3, (9, 12, 7))])
def test_boundary_project_state(dim, n):
    pe = _pe()
    prob = _case(dim, n, seed=6)
    g = pe.Grid.from_problem(prob)
    W = g.project_state(prob.u0, prob.t0).cpu().numpy()
    assert rel(W, Discretization(prob).initial()) <= 1e-13
    # without data the call is the plain projection
    g.set_boundary([])
    W0 = g.project_state(prob.u0, prob.t0).cpu().numpy()
    np.testing.assert_array_equal(W0, g.project(prob.u0).cpu().numpy())


@pytest.mark.parametrize("dim,n", [(2, (45, 38)), (3, (11, 17, 9))])
def test_boundary_parareal_solve(dim, n):
    pe = _pe()
    prob = wl.tiny_problem(dim, n, seed=31, N=6, J=5, s=3, u0_modes=2).with_(boundary=_data(dim))
    g, U, rep = pe.solve_problem(prob, K_max=prob.K_max, tol=1e-8)
    d = Discretization(prob)
    r = parareal(d, d.initial(), prob.t0, prob.N, prob.J, d.tables(prob.dt, prob.c_fine),
                 d.tables(prob.dT, prob.c_coarse), K_max=prob.K_max, tol=1e-8)
    assert rep.iterations == r.iterations and bool(rep.converged) == r.converged
    assert rel(U.cpu().numpy(), r.iterates[-1]) <= 1e-11


def test_bilinear_data_stay_steady():
    """f = 0 and g = u0 bilinear: a steady state of the discrete problem."""
    pe = _pe()
    ONE = wl.TimeFactor()
    l = [wl.Term(1.0, ONE, (P(1.0), P(1.0))), wl.Term(0.5, ONE, (P(0.0, 1.0), P(1.0))),
         wl.Term(-0.3, ONE, (P(1.0), P(0.0, 1.0))), wl.Term(0.7, ONE, (P(0.0, 1.0), P(0.0, 1.0)))]
    prob = wl.tiny_problem(2, (31, 20), seed=9, N=4, J=3, s=3, u0_modes=0).with_(
        forcing=[], u0=l, boundary=l)
    g, U, rep = pe.solve_problem(prob, K_max=3, tol=1e-12)
    W0 = Discretization(prob).initial()
    Un = U.cpu().numpy()
    assert rel(Un[0], W0) <= 1e-13
    assert max(rel(Un[k], W0) for k in range(prob.N + 1)) <= 1e-12


def test_boundary_term_limits():
    pe = _pe()
    prob = _case(2, (15, 12), seed=7)
    g = pe.Grid.from_problem(prob)
    many = [prob.boundary[0]] * 11        # 11 x (2 + 2 d) = 66 > 64
    arr, m = pe.to_c_terms(many)
    assert g.L.pe_set_boundary(g.h, m, arr, None) == pe.PE_E_ARG
    # the grid keeps its data: the projection still matches the oracle
    W = g.project_state(prob.u0, prob.t0).cpu().numpy()
    assert rel(W, Discretization(prob).initial()) <= 1e-13


def test_boundary_fullsize_first_slices():
    """The 255x255 workload with Dirichlet data, at full size in the default
    batching: the converged Parareal answer at T_1 and T_2 against the
    oracle's sequential fine solution of the first two slices (after one
    fine pass the Parareal iterate is the fine solution)."""
    pe = _pe()
    prob = wl.config(2).with_(boundary=_data(2))
    print(f"boundary full size: {prob.name}, dof {prob.dof}", flush=True)
    g, U, rep = pe.solve_problem(prob)
    assert rep.converged
    d = Discretization(prob)
    tab = d.tables(prob.dt, prob.c_fine)
    W, kept = sequential(d, d.initial(), prob.t0, tab, 2 * prob.J, keep_every=prob.J)
    got = U[:3].cpu().numpy()
    err = rel(got, np.stack(kept))
    print(f"  iterations {rep.iterations}, relative L2 error on slices 0..2: {err:.3e}")
    assert err <= 1e-11
