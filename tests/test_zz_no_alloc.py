"""pe_coarse_sweep_noalloc (norm partials in the library's static device
array, no workspace) against pe_coarse_sweep, through the C ABI: plain and
correction sweeps, two calls in a row with the second on a smaller grid,
bitwise equal states and norms (the same kernels), and the size limit."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pe():
    from paper_2412_01138_amd import peifem
    return peifem


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def _case(pe, n, N, seed):
    prob = wl.tiny_problem(2, n, seed=seed, N=N, J=2, s=3)
    g = pe.Grid.from_problem(prob)
    EG, BG = g.phi_tables(prob.dT, prob.c_coarse)
    rng = np.random.default_rng(seed)
    U = torch.zeros((N + 1,) + prob.n, dtype=torch.float64, device="cuda:0")
    U[0] = _dev(rng.normal(size=prob.n))
    r = torch.empty((N,) + prob.n, dtype=torch.float64, device="cuda:0")
    g.coarse_sweep(U, prob.t0, prob.dT, prob.c_coarse, EG, BG, r)      # fills r
    corr = _dev(rng.normal(size=(N,) + prob.n) * 0.01)
    Fout = _dev(rng.normal(size=(N,) + prob.n))
    return prob, g, EG, BG, r, corr, U, Fout


def _compare(pe, prob, g, EG, BG, r, corr, Uprev, Fout):
    N = prob.N
    for up, fo, cc in ((None, None, corr), (Uprev, Fout, None), (Uprev, Fout, corr)):
        U1 = torch.zeros_like(Uprev)
        U1[0] = Uprev[0]
        U2 = U1.clone()
        n1 = torch.full((3,), -1.0, dtype=torch.float64, device="cuda:0")
        n2 = torch.full((3,), -2.0, dtype=torch.float64, device="cuda:0")
        g.coarse_sweep(U1, prob.t0, prob.dT, prob.c_coarse, EG, BG, r, compute_r=False,
                       corr=cc, Uprev=up, Fout=fo, norms=n1)
        g.coarse_sweep_noalloc(U2, EG, r, corr=cc, Uprev=up, Fout=fo, norms=n2)
        torch.cuda.synchronize()
        assert torch.equal(U1, U2)
        assert torch.equal(n1, n2), (n1, n2)
        assert float(n1[1]) > 0 and (up is None or float(n1[0]) > 0)
    assert U1.shape[0] == N + 1


def test_noalloc_sweep_matches_workspace_sweep_twice():
    pe = _pe()
    big = _case(pe, (255, 191), 6, seed=71)
    _compare(pe, *big)
    small = _case(pe, (37, 21), 3, seed=72)       # second call: a smaller input
    _compare(pe, *small)
    _compare(pe, *big)                            # and back: nothing stale is read


def test_noalloc_sweep_rejects_grids_beyond_the_limit():
    pe = _pe()
    g = pe.Grid((330, 330, 330), (0, 0, 0), (1, 1, 1), 0.1)
    assert g.dof > pe.PE_NOALLOC_MAX_DOF
    tiny = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    p = tiny.data_ptr()
    st = g.L.pe_coarse_sweep_noalloc(g.h, 1, p, p, None, None, None, p + 16, p + 8, None)
    assert st == pe.PE_E_ARG and b"limit" in g.L.pe_last_error()
    assert torch.count_nonzero(tiny) == 0                  # nothing was launched
