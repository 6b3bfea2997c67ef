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
