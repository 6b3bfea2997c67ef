"""Split-bf16 path (fp32 states, bf16 hi/lo transform products with fp32
accumulation, FP64 tables and norms) vs the FP64 CPU oracle.

Tolerance: 2e-5 relative L2 against the FP64 oracle, the stated target for
the split-bf16 path.  Each product keeps about 16 significant bits of each
operand pair (hi*hi + hi*lo + lo*hi), i.e. ~2^-17 relative per term; over
d <= 3 axes of accumulation plus the fp32 state this stays near 1e-5.
"""
import numpy as np
import pytest

import workloads as wl
from oracle.eife import Discretization
from oracle.parareal import fine_prop, parareal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SPLIT_TOL = 2e-5


def _peifem():
    from paper_2412_01138_amd import peifem
    return peifem


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _dev32(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda:0")


@pytest.mark.parametrize("dim,n", [(1, (63,)), (2, (37, 70)), (3, (9, 33, 20)), (3, (31, 63, 17)),
                                   (2, (20, 600))])
def test_split_project(dim, n):
    pe = _peifem()
    prob = wl.tiny_problem(dim, n, seed=12, u0_modes=3, precision="split_bf16")
    g = pe.Grid.from_problem(prob)
    W = g.project(prob.u0)
    assert W.dtype == torch.float32
    ref = Discretization(prob).initial()
    assert rel(W.cpu().numpy(), ref) <= SPLIT_TOL


@pytest.mark.parametrize("dim,n,N,J,s,modes", [
    (1, (100,), 3, 5, 3, 4),
    (2, (37, 70), 3, 4, 3, 4),
    (2, (64, 64), 2, 3, 4, 20),
    (3, (9, 33, 20), 2, 3, 4, 5),
    (3, (31, 63, 17), 2, 2, 3, 40),       # more terms than the fused path takes
    # axis 0 with Kh = 64 / 128: the last pass is fused with the update
    (2, (127, 40), 2, 3, 3, 4),
    (3, (100, 20, 9), 2, 2, 3, 4),
    (2, (200, 33), 1, 2, 4, 5),
    (3, (255, 9, 12), 1, 2, 3, 4),
    # a last axis with Kh = 320 (the generating pass at any length)
    (2, (20, 600), 2, 2, 3, 5),
    # one stage and one step: a single field per slice (the decay and the
    # weights of every field at once; the prefetch past the last field)
    (2, (127, 40), 2, 1, 1, 4),
])
def test_split_fine_propagate(dim, n, N, J, s, modes):
    pe = _peifem()
    prob = wl.tiny_problem(dim, n, seed=3, s=s, N=N, J=J, n_modes=modes, T=0.9,
                           precision="split_bf16")
    d = Discretization(prob)
    rng = np.random.default_rng(4)
    Uin = rng.normal(size=(N,) + prob.n)
    g = pe.Grid.from_problem(prob)
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    out = g.fine_propagate(_dev32(Uin), prob.t0, prob.dT, J, prob.c_fine, E, B)
    assert out.dtype == torch.float32
    tab = d.tables(prob.dt, prob.c_fine)
    ref = np.stack([fine_prop(d, Uin[k], prob.t0 + k * prob.dT, tab, J) for k in range(N)])
    assert rel(out.cpu().numpy(), ref) <= SPLIT_TOL


@pytest.mark.parametrize("dim,n,N,J,s", [(2, (127, 40), 3, 4, 3), (3, (200, 12, 9), 2, 2, 4)])
def test_split_fused_update_matches_separate_kernels(dim, n, N, J, s):
    """Split-bf16 grids with Kh = 64 / 128 on axis 0: the last pass fused
    with the update against the separate pass + update (which run when the
    workspace has no room for the update tables; the separate path then
    rounds the fp32 state after every step, the fused one keeps it in FP64
    across a slice's steps)."""
    pe = _peifem()
    prob = wl.tiny_problem(dim, n, seed=8, s=s, N=N, J=J, n_modes=4, T=0.9,
                           precision="split_bf16")
    rng = np.random.default_rng(9)
    Uin = _dev32(rng.normal(size=(N,) + prob.n))
    g = pe.Grid.from_problem(prob)
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    fused = g.fine_propagate(Uin, prob.t0, prob.dT, J, prob.c_fine, E, B).cpu().numpy()
    per_field = g.fine_workspace_bytes(2) - g.fine_workspace_bytes(1)
    work = g.workspace(3 * 256 + per_field * s)
    sep = g.fine_propagate(Uin, prob.t0, prob.dT, J, prob.c_fine, E, B, work=work).cpu().numpy()
    assert rel(fused, sep) <= 2e-6


def _every_chunk_sines(prob, seed):
    """Sine terms whose modes fall in every 64-wide chunk of both halves of
    axes 1 and 2 (k = 1, 2: first chunk of each half; 129, 130: the second
    chunk when Kh = 128; n - 1, n: the last)."""
    rng = np.random.default_rng(seed)
    n0, n1, n2 = prob.n
    box = list(zip(prob.lo, prob.hi))
    ks = [(1, 1, 2), (2, 2, 1), (n0, n1, n2), (n0 - 1, n1 - 1, n2 - 1),
          (3, min(129, n1), min(129, n2)), (4, min(130, n1), min(130, n2)),
          (5, min(n1, 2 * 64 - 1), 3), (6, 4, min(n2, 2 * 64))]
    terms = [wl.Term(float(rng.uniform(0.5, 1.5)) * (-1) ** i,
                     wl.TimeFactor(omega=float(rng.uniform(1.0, 20.0))),
                     tuple(wl.sine_factor(k, lo, hi) for k, (lo, hi) in zip(kk, box)))
             for i, kk in enumerate(ks)]
    return terms


@pytest.mark.parametrize("n,s", [((65, 67, 69), 3), ((100, 200, 90), 4), ((66, 100, 255), 3),
                                 ((70, 193, 200), 3), ((128, 256, 193), 2), ((230, 70, 255), 1)])
def test_split_gen_mid_sampled(n, s):
    """3D split grids whose axes 1 and 2 have Kh = 64 / 128 (odd and even n):
    the generating and middle-axis passes run as one kernel.  From a zero
    state, so that the output is the transformed loads' share alone, with
    sine terms forcing modes in every chunk and half of axes 1 and 2 and a
    polynomial term reaching every mode: each sine-forced mode against the
    selected-mode oracle (relative error 1e-3 each, 2e-5 in L2), and 400
    random modes to the split path's absolute error (relative to the largest
    coefficient)."""
    from oracle import modal
    pe = _peifem()
    prob = wl.tiny_problem(3, n, seed=23, s=s, N=2, J=2, n_modes=1, T=0.9,
                           precision="split_bf16")
    prob.forcing[:] = _every_chunk_sines(prob, 25)
    forced = modal.forced_modes(prob)                 # the sine terms' modes
    # a polynomial term reaches every mode
    prob.forcing.append(wl.Term(0.8, wl.TimeFactor(omega=3.0, poly=(1.0, 0.5, 0.0, 0.0)),
                                (wl.poly_factor(0.2, 1.0, -0.7), wl.poly_factor(1.0, -0.3, 0.1),
                                 wl.poly_factor(0.5, 0.2, 0.3))))
    g = pe.Grid.from_problem(prob)
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    zero = np.zeros((prob.N,) + prob.n)
    out = g.fine_propagate(_dev32(zero), prob.t0, prob.dT, prob.J, prob.c_fine, E, B).cpu().numpy()
    rng = np.random.default_rng(24)
    extra = np.stack([rng.integers(0, prob.n[a], 400) for a in range(3)], axis=1)
    sel = np.unique(np.concatenate([forced, extra]), axis=0)
    fine = modal.ModalFine(prob, sel)
    is_forced = np.isin(sel.view([("", sel.dtype)] * 3), forced.view([("", forced.dtype)] * 3)).ravel()
    idx = tuple(sel.T)
    for k in range(prob.N):
        ref = fine.propagate(zero[k][idx], prob.t0 + k * prob.dT)
        got = out[k][idx]
        # each sine-forced mode on its own (their values span four decades:
        # the split products' error is relative to the loads, not to the
        # decayed coefficient of a high mode)
        rel_each = np.abs(got[is_forced] - ref[is_forced]) / np.abs(ref[is_forced])
        assert rel_each.max() <= 1e-3, (k, rel_each)
        assert rel(got[is_forced], ref[is_forced]) <= SPLIT_TOL, k
        assert np.abs(got - ref).max() <= SPLIT_TOL * np.abs(ref).max(), k


@pytest.mark.parametrize("n,N,J,s,modes", [((65, 67, 69), 2, 3, 3, 4), ((100, 200, 90), 2, 2, 4, 9),
                                           ((66, 100, 255), 1, 2, 3, 32), ((128, 256, 193), 1, 1, 3, 5),
                                           # one field per slice (one step, one stage)
                                           ((100, 200, 90), 2, 1, 1, 4)])
def test_split_gen_mid_fused_matches_two_passes(n, N, J, s, modes):
    """3D split grids: the generating and middle-axis passes as one kernel
    (axis-2 results kept on chip, output with axis 0 outermost, read so by the
    fused axis-0 pass) against the two separate passes (pe_set_fusion(0)).
    Same products; the fused kernel orders each 32-wide k-step of the axis-2
    product differently, so the two agree to fp32 rounding."""
    pe = _peifem()
    prob = wl.tiny_problem(3, n, seed=21, s=s, N=N, J=J, n_modes=modes, T=0.9,
                           precision="split_bf16")
    rng = np.random.default_rng(22)
    Uin = _dev32(rng.normal(size=(N,) + prob.n))
    g = pe.Grid.from_problem(prob)
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    fused = g.fine_propagate(Uin, prob.t0, prob.dT, J, prob.c_fine, E, B).cpu().numpy()
    g.set_fusion(False)
    two = g.fine_propagate(Uin, prob.t0, prob.dT, J, prob.c_fine, E, B).cpu().numpy()
    g.set_fusion(True)
    again = g.fine_propagate(Uin, prob.t0, prob.dT, J, prob.c_fine, E, B).cpu().numpy()
    assert np.array_equal(fused, again)
    assert rel(fused, two) <= 1e-6


@pytest.mark.parametrize("dim,n", [(2, (45, 38)), (3, (15, 31, 9)), (2, (127, 20))])
def test_split_parareal(dim, n):
    pe = _peifem()
    prob = wl.tiny_problem(dim, n, seed=51, N=5, J=4, s=3, u0_modes=2, precision="split_bf16")
    g, U, rep = pe.solve_problem(prob, K_max=6, tol=1e-5)
    d = Discretization(prob)
    r = parareal(d, d.initial(), prob.t0, prob.N, prob.J, d.tables(prob.dt, prob.c_fine),
                 d.tables(prob.dT, prob.c_coarse), K_max=6, tol=1e-5)
    assert rep.converged and rep.iterations == r.iterations
    assert rel(U.cpu().numpy(), r.iterates[-1]) <= SPLIT_TOL
