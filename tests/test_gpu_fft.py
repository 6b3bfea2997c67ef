"""The FFT transform (pe_set_transform(g, PE_TRANSFORM_FFT)) against the FP64
oracle and against the dense matrix-core transform, through the C ABI.

The FFT computes the same sine coefficients with another summation order, so
every result is held to the FP64 bars of the dense path: single propagations
1e-12 relative L2 against the oracle, Parareal answers 1e-11, and the two
GPU transforms agree to 1e-13.  Cases cover every FFT length (2(n+1) = 128,
256, 512, 1024), generated and separate load quadrature, the axis-0 pass
fused with the update and the separate update, and 1, 2 and 3 axes.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import modal
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
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def _fine_case(dim, n, N, J, s, seed=0, n_modes=4):
    prob = wl.tiny_problem(dim, n, seed=seed, s=s, N=N, J=J, n_modes=n_modes, T=0.9)
    rng = np.random.default_rng(seed + 1)
    return prob, Discretization(prob), rng.normal(size=(N,) + prob.n)


def _propagate(pe, prob, Uin, transform, work_fields=None):
    g = pe.Grid.from_problem(prob, transform=transform)
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    work = None
    if work_fields is not None:
        work = g.workspace(g.fine_workspace_bytes(work_fields))
    out = g.fine_propagate(_dev(Uin), prob.t0, prob.dT, prob.J, prob.c_fine, E, B, work=work)
    return out.cpu().numpy()


@pytest.mark.parametrize("dim,n,N,J,s", [
    (1, (63,), 3, 4, 3),              # N = 128, generated, separate update
    (1, (511,), 2, 3, 2),             # N = 1024
    (2, (63, 63), 2, 3, 3),           # fused axis-0 pass, N = 128
    (2, (255, 127), 2, 2, 4),         # N = 512 fused, N = 256 generated
    (2, (511, 63), 1, 2, 3),          # N = 1024 fused
    (2, (63, 511), 2, 2, 2),          # N = 1024 generated
    (3, (63, 63, 127), 1, 2, 3),      # strided middle pass
    (3, (127, 63, 63), 1, 2, 2),
])
def test_fft_fine_propagate(dim, n, N, J, s):
    pe = _pe()
    print(f"fft fine propagate dim {dim} n {n} N {N} J {J} s {s}", flush=True)
    prob, d, Uin = _fine_case(dim, n, N, J, s, seed=3)
    out = _propagate(pe, prob, Uin, "fft")
    tab = d.tables(prob.dt, prob.c_fine)
    ref = np.stack([fine_prop(d, Uin[k], prob.t0 + k * prob.dT, tab, J) for k in range(N)])
    assert rel(out, ref) <= 1e-12
    dense = _propagate(pe, prob, Uin, "dense")
    assert rel(out, dense) <= 1e-13


def test_fft_separate_update_matches_fused():
    """A workspace without room for the update tables takes the separate
    axis-0 pass and update; it agrees with the fused kernel to rounding."""
    pe = _pe()
    prob, d, Uin = _fine_case(2, (127, 63), 2, 3, 3, seed=4)
    g = pe.Grid.from_problem(prob, transform="fft")
    E, B = g.phi_tables(prob.dt, prob.c_fine)
    U = _dev(Uin)
    fused = g.fine_propagate(U, prob.t0, prob.dT, prob.J, prob.c_fine, E, B).cpu().numpy()
    per_field = g.fine_workspace_bytes(2) - g.fine_workspace_bytes(1)
    work = g.workspace(3 * 256 + per_field * prob.q)
    sep = g.fine_propagate(U, prob.t0, prob.dT, prob.J, prob.c_fine, E, B, work=work)
    assert rel(sep.cpu().numpy(), fused) <= 1e-14
    tab = d.tables(prob.dt, prob.c_fine)
    ref = np.stack([fine_prop(d, Uin[k], prob.t0 + k * prob.dT, tab, prob.J) for k in range(2)])
    assert rel(fused, ref) <= 1e-12


def test_fft_batching_is_exact():
    """Whole slices per batch: every mode sees the same kernels and order."""
    pe = _pe()
    prob, d, Uin = _fine_case(2, (63, 127), 5, 4, 3, seed=6)
    full = _propagate(pe, prob, Uin, "fft")
    for fields in (12, 24, 36):
        np.testing.assert_array_equal(_propagate(pe, prob, Uin, "fft", fields), full)


def test_fft_many_terms_use_the_separate_quadrature():
    """More terms than the generating pass holds: the quadrature kernel writes
    the load fields and the first FFT pass reads them."""
    pe = _pe()
    prob, d, Uin = _fine_case(2, (63, 127), 2, 2, 3, seed=7, n_modes=40)
    out = _propagate(pe, prob, Uin, "fft")
    tab = d.tables(prob.dt, prob.c_fine)
    ref = np.stack([fine_prop(d, Uin[k], prob.t0 + k * prob.dT, tab, prob.J) for k in range(2)])
    assert rel(out, ref) <= 1e-12


@pytest.mark.parametrize("dim,n", [(1, (127,)), (2, (63, 255)), (3, (63, 127, 63))])
def test_fft_project(dim, n):
    """P_h u0 with polynomial terms (every mode carries energy).  The oracle's
    LAPACK eigenvectors differ from the exact sine basis by up to 3e-13 per
    column at n = 127 and 1.3e-12 at n = 255, so the bar against the oracle
    is 1e-12 here; against the dense GPU transform (the same exact basis) it
    is 1e-13."""
    pe = _pe()
    prob = wl.tiny_problem(dim, n, seed=4, u0_modes=3)
    prob.u0.append(wl.Term(0.6, wl.TimeFactor(),
                           tuple(wl.poly_factor(0.2, 1.0, -0.7) for _ in range(dim))))
    W = {}
    for tr in ("dense", "fft"):
        g = pe.Grid.from_problem(prob, transform=tr)
        W[tr] = g.project(prob.u0).cpu().numpy()
    assert rel(W["fft"], Discretization(prob).initial()) <= 1e-12
    assert rel(W["fft"], W["dense"]) <= 1e-13


def test_fft_learned_samples_match_dense():
    pe = _pe()
    prob = wl.tiny_problem(2, (63, 127), seed=8, N=3, J=2, s=3)
    out = {}
    for tr in ("dense", "fft"):
        g = pe.Grid.from_problem(prob, transform=tr)
        out[tr] = g.learned_samples(prob.N, prob.t0, prob.dT).cpu().numpy()
    assert rel(out["fft"], out["dense"]) <= 1e-13


def test_fft_parareal_solve():
    pe = _pe()
    prob = wl.tiny_problem(2, (63, 127), seed=31, N=6, J=5, s=3, u0_modes=2)
    g, U, rep = pe.solve_problem(prob, K_max=prob.K_max, tol=1e-8, transform="fft")
    d = Discretization(prob)
    r = parareal(d, d.initial(), prob.t0, prob.N, prob.J, d.tables(prob.dt, prob.c_fine),
                 d.tables(prob.dT, prob.c_coarse), K_max=prob.K_max, tol=1e-8)
    assert rep.iterations == r.iterations and bool(rep.converged) == r.converged
    assert rel(U.cpu().numpy(), r.iterates[-1]) <= 1e-11


def test_fft_rejects_unsupported_grids():
    pe = _pe()
    bad = [
        (pe.Grid((100, 63), (0, 0), (1, 1), 0.1), pe.PE_TRANSFORM_FFT),     # n + 1 not 2^k
        (pe.Grid((31, 63), (0, 0), (1, 1), 0.1), pe.PE_TRANSFORM_FFT),      # below 64
        (pe.Grid((63, 63), (0, 0), (1, 1), 0.1, precision="split_bf16"), pe.PE_TRANSFORM_FFT),
        (pe.Grid((63, 63), (0, 0), (1, 1), 0.1), 7),                         # unknown kind
    ]
    for g, kind in bad:
        st = g.L.pe_set_transform(g.h, kind)
        assert st == pe.PE_E_ARG
        assert g.transform == "dense"
    with pytest.raises(pe.PeifemError):
        pe.Grid((100, 63), (0, 0), (1, 1), 0.1, transform="fft")


@pytest.mark.parametrize("cfg", [2, 4])
def test_fft_fullsize_parareal_answer(cfg):
    """The FP64 workloads at full size with the FFT transform, in the default
    batching, against the selected-mode oracle (as for the dense path)."""
    pe = _pe()
    prob = wl.config(cfg)
    print(f"fft full size: workload {cfg}, dof {prob.dof}, N {prob.N}, J {prob.J}", flush=True)
    modes = modal.sample_modes(prob, 32, seed=100 + cfg)
    ref = modal.sequential_fine_modes(prob, modes)
    g, U, rep = pe.solve_problem(prob, transform="fft")
    assert rep.converged and rep.iterations >= 1
    flat = U.reshape(prob.N + 1, -1)
    idx = torch.as_tensor(modal.flat_index(prob, modes), device=U.device)
    err = rel(flat[:, idx].cpu().numpy(), ref)
    print(f"  iterations {rep.iterations}, relative L2 error on {len(modes)} modes: {err:.3e}")
    assert err <= 1e-11
