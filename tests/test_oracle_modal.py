"""Pins of the selected-mode oracle against the full-field oracle (CPU)."""
import numpy as np
import pytest

import workloads as wl
from oracle import modal
from oracle.eife import Discretization
from oracle.parareal import sequential_fine


@pytest.mark.parametrize("dim,n,seed", [(1, (13,), 3), (2, (9, 7), 4), (3, (5, 6, 4), 5)])
def test_modal_fine_solution_equals_full_oracle(dim, n, seed):
    prob = wl.tiny_problem(dim, n, seed=seed, N=3, J=4, s=3, n_modes=3, u0_modes=2)
    d = Discretization(prob)
    full = sequential_fine(d, d.initial(), prob.t0, prob.N, prob.J, d.tables(prob.dt, prob.c_fine))
    modes = np.stack(np.unravel_index(np.arange(prob.dof), prob.n), axis=1)
    got = modal.sequential_fine_modes(prob, modes)
    ref = full.reshape(prob.N + 1, -1)
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_forced_modes_carry_the_whole_forcing():
    prob = wl.tiny_problem(2, (15, 12), seed=9, N=2, J=2, s=2, n_modes=4, u0_modes=0)
    d = Discretization(prob)
    forced = modal.forced_modes(prob)
    assert 1 <= len(forced) <= 4          # sine modes are single spectral modes
    mask = np.zeros(prob.n, dtype=bool)
    mask[tuple(forced.T)] = True
    for t in (0.0, 0.13, 0.41):
        g = d.spectral_forcing(t)
        assert np.max(np.abs(g[~mask])) <= 1e-12 * np.max(np.abs(g))
        np.testing.assert_allclose(modal.ModalForcing(prob, forced).at(t), g[mask],
                                   rtol=1e-12, atol=1e-14 * np.max(np.abs(g)))


def test_flat_index_is_c_order():
    prob = wl.tiny_problem(3, (4, 5, 6), seed=1)
    modes = np.array([[0, 0, 0], [1, 2, 3], [3, 4, 5]])
    np.testing.assert_array_equal(modal.flat_index(prob, modes), [0, 1 * 30 + 2 * 6 + 3, 119])


@pytest.mark.parametrize("cfg", [2, 4])
def test_stored_fullsize_reference_is_the_oracles(cfg):
    """tests/golden/fullsize_modal_reference.json (read by the benchmark to
    state each answer's error) holds exactly what the selected-mode oracle
    computes for the workload."""
    from conftest import load_golden
    rec = load_golden("fullsize_modal_reference.json")["workloads"][str(cfg)]
    prob = wl.config(cfg)
    modes = modal.sample_modes(prob, 32, seed=100 + cfg)
    assert modes.tolist() == rec["modes"]
    assert modal.flat_index(prob, modes).tolist() == rec["flat_index"]
    assert modal.flat_index(prob, modal.forced_modes(prob)).tolist() == rec["forced_flat_index"]
    ref = modal.sequential_fine_modes(prob, modes)
    stored = np.array([[float.fromhex(v) for v in row] for row in rec["W"]])
    np.testing.assert_array_equal(stored, ref)
