"""Full-size parity: the converged Parareal answer of each workload at its
real size, in the launch configuration bench.py times (the library's default
batching), against the selected-mode FP64 oracle.

The sample is every forced mode plus seeded random modes.  With u0 = 0 and
sine-mode forcing the forced modes carry the whole solution (the forcing
reaches no other mode), so the sampled error is the L2 error of the answer;
the test also checks that the GPU answer has no energy outside the forced
modes.  Tolerances: FP64 workloads 1e-11 relative L2 over all slice ends;
split-bf16 workloads (FP32 state) 2e-5.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import modal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {2: 1e-11, 3: 2e-5, 4: 1e-11, 5: 2e-5}


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("cfg", [2, 3, 4, 5])
def test_fullsize_parareal_answer(cfg):
    from paper_2412_01138_amd import peifem as pe
    prob = wl.config(cfg)
    print(f"workload {cfg}: {prob.name}, dof {prob.dof}, N {prob.N}, J {prob.J}", flush=True)
    modes = modal.sample_modes(prob, 32, seed=100 + cfg)
    ref = modal.sequential_fine_modes(prob, modes)
    g, U, rep = pe.solve_problem(prob)
    assert rep.converged and rep.iterations >= 1
    flat = U.reshape(prob.N + 1, -1)
    idx = torch.as_tensor(modal.flat_index(prob, modes), device=U.device)
    got = flat[:, idx].double().cpu().numpy()
    err = rel(got, ref)
    print(f"  iterations {rep.iterations}, relative L2 error on {len(modes)} modes: {err:.3e}")
    assert err <= TOL[cfg]
    forced = torch.as_tensor(modal.flat_index(prob, modal.forced_modes(prob)), device=U.device)
    inside = float(torch.linalg.vector_norm(flat[:, forced].double()))
    rest = flat.clone()
    rest[:, forced] = 0
    outside = float(torch.linalg.vector_norm(rest.double()))
    print(f"  norm outside the forced modes / inside: {outside / inside:.3e}")
    assert outside <= TOL[cfg] * inside


@pytest.mark.parametrize("cfg", [4, 5])
def test_fullsize_learned_answer(cfg):
    """The learned coarse correction at full size (workload 5 on the
    split-bf16 path): a network trained with the library's kernels on 64
    forcings of the workload's family on a 31^d grid, then the full-size
    solve with it: converged, the network used (no fallback), and the answer
    against the same oracle values as the plain solve."""
    from paper_2412_01138_amd import learned_g as lg, peifem as pe
    prob = wl.config(cfg)
    X, T, S = lg.training_rows(prob, [10000 + i for i in range(64)], (31,) * prob.dim)
    W = lg.row_weights(X, S, prob.N, 0.0)
    m, _ = lg.train(X, T, 3000, batch=16384, lr=2e-3, weights=W)
    modes = modal.sample_modes(prob, 32, seed=100 + cfg)
    ref = modal.sequential_fine_modes(prob, modes)
    g, U, rep = pe.solve_problem(prob, mlp=m)
    print(f"workload {cfg} learned: iterations {rep.iterations}, jumps {list(rep.jumps[:rep.iterations])}, "
          f"learned part {rep.ms_learned:.1f} ms", flush=True)
    assert rep.converged and rep.fallback == 0 and rep.ms_learned > 0
    flat = U.reshape(prob.N + 1, -1)
    idx = torch.as_tensor(modal.flat_index(prob, modes), device=U.device)
    err = rel(flat[:, idx].double().cpu().numpy(), ref)
    print(f"  relative L2 error on {len(modes)} modes: {err:.3e}")
    assert err <= TOL[cfg]
