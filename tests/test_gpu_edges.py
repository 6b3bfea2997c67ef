"""Degenerate and boundary cases of the GPU path against the FP64 oracle:
the smallest grids (one or two interior nodes per axis), a single slice, a
single fine step (F = G: the coarse solution is already the fine one), a
one-stage rule (exponential Euler), no forcing with no initial value (the
zero solution), and the learned calls on a grid without forcing."""
import numpy as np
import pytest

import workloads as wl
from oracle.eife import Discretization
from oracle.parareal import fine_prop, parareal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pe():
    from paper_2412_01138_amd import peifem
    return peifem


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))


def _oracle_solve(prob, K_max, tol):
    d = Discretization(prob)
    return parareal(d, d.initial(), prob.t0, prob.N, prob.J, d.tables(prob.dt, prob.c_fine),
                    d.tables(prob.dT, prob.c_coarse), K_max=K_max, tol=tol)


@pytest.mark.parametrize("dim,n", [(1, (1,)), (1, (2,)), (2, (1, 1)), (2, (1, 5)), (2, (2, 3)),
                                   (3, (1, 1, 1)), (3, (2, 1, 3))])
def test_smallest_grids(dim, n):
    pe = _pe()
    prob = wl.tiny_problem(dim, n, seed=11, N=3, J=2, s=3, n_modes=2, u0_modes=1)
    d = Discretization(prob)
    g = pe.Grid.from_problem(prob)
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    rng = np.random.default_rng(3)
    Uin = rng.normal(size=(prob.N,) + prob.n)
    out = g.fine_propagate(torch.as_tensor(Uin, device="cuda:0"), prob.t0, prob.dT, prob.J,
                           prob.c_fine, E, B).cpu().numpy()
    tab = d.tables(prob.dt, prob.c_fine)
    ref = np.stack([fine_prop(d, Uin[k], prob.t0 + k * prob.dT, tab, prob.J)
                    for k in range(prob.N)])
    assert rel(out, ref) <= 1e-12
    _, U, rep = pe.solve_problem(prob, K_max=4, tol=1e-10)
    r = _oracle_solve(prob, 4, 1e-10)
    assert rep.iterations == r.iterations
    assert rel(U.cpu().numpy(), r.iterates[-1]) <= 1e-11


def test_single_slice():
    pe = _pe()
    prob = wl.tiny_problem(2, (21, 14), seed=12, N=1, J=5, s=3)
    _, U, rep = pe.solve_problem(prob, K_max=3, tol=1e-10)
    r = _oracle_solve(prob, 3, 1e-10)
    assert rep.iterations == r.iterations
    assert rel(U.cpu().numpy(), r.iterates[-1]) <= 1e-11


def test_single_fine_step_needs_one_pass():
    """J = 1 with the same nodes: F = G, the coarse solution is the fine
    solution and the first jump is roundoff."""
    pe = _pe()
    prob = wl.tiny_problem(2, (17, 9), seed=13, N=4, J=1, s=2)
    _, U, rep = pe.solve_problem(prob, K_max=3, tol=1e-12)
    assert rep.iterations == 1 and rep.converged
    assert rep.jumps[0] <= 1e-14
    r = _oracle_solve(prob, 3, 1e-12)
    assert rel(U.cpu().numpy(), r.iterates[-1]) <= 1e-11


def test_one_stage_rule():
    pe = _pe()
    prob = wl.tiny_problem(2, (19, 23), seed=14, N=3, J=4, s=1)
    _, U, rep = pe.solve_problem(prob, K_max=3, tol=1e-10)
    r = _oracle_solve(prob, 3, 1e-10)
    assert rep.iterations == r.iterations
    assert rel(U.cpu().numpy(), r.iterates[-1]) <= 1e-11


def test_zero_solution():
    """No forcing and no initial value: every iterate is zero, the jump is 0
    and the first fine pass already meets any tolerance."""
    pe = _pe()
    prob = wl.tiny_problem(2, (15, 15), seed=15, N=3, J=2, s=2, u0_modes=0).with_(forcing=[])
    _, U, rep = pe.solve_problem(prob, K_max=3, tol=1e-12)
    assert rep.iterations == 1 and rep.converged and rep.jumps[0] == 0.0
    assert float(torch.count_nonzero(U)) == 0


def test_learned_calls_without_forcing():
    """Without forcing the correction is zero and there are no training rows."""
    pe = _pe()
    from oracle import mlp as omlp
    prob = wl.tiny_problem(2, (15, 12), seed=16, N=3, J=2, s=3).with_(forcing=[])
    g = pe.Grid.from_problem(prob)
    m = pe.Mlp(omlp.to_bf16(omlp.init_params(1)))
    corr, fb = g.learned_correction(m, prob.N, prob.t0, prob.dT)
    assert not fb and float(torch.count_nonzero(corr)) == 0
    zero = g.empty_states(prob.N).zero_()
    x, t, count = g.learned_rows(zero, zero, prob.t0, prob.dT)
    assert count == 0 and x.shape[0] == 0
