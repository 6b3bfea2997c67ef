"""Writes fullsize_modal_reference.json: the FP64 oracle's sequential fine
solution (which every converged Parareal iterate equals) of workloads 2-5
at their full sizes, on every forced mode plus 32 seeded random modes, at
every slice end T_n, n = 0..N.  Computed by the selected-mode oracle
(oracle/modal.py) only; the benchmark reads this file to state each
result's error against the oracle without running the oracle itself.

    python tests/golden/make_fullsize_reference.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as wl          # noqa: E402
from oracle import modal        # noqa: E402


def main():
    out = {"source": "oracle/modal.py sequential_fine_modes (eq. 2.6 steps in the "
                     "M-orthonormal eigenbasis from dense LAPACK, mpmath phi tables), "
                     "written by tests/golden/make_fullsize_reference.py",
           "workloads": {}}
    for cfg in (2, 3, 4, 5):
        prob = wl.config(cfg)
        modes = modal.sample_modes(prob, 32, seed=100 + cfg)
        ref = modal.sequential_fine_modes(prob, modes)
        forced = modal.forced_modes(prob)
        out["workloads"][str(cfg)] = {
            "name": prob.name, "n": list(prob.n), "N": prob.N,
            "modes": modes.tolist(),
            "flat_index": modal.flat_index(prob, modes).tolist(),
            "forced_flat_index": modal.flat_index(prob, forced).tolist(),
            "W": [[float(v).hex() for v in row] for row in ref],
        }
        print(f"workload {cfg}: {len(modes)} modes x {prob.N + 1} slice ends", flush=True)
    with open(os.path.join(HERE, "fullsize_modal_reference.json"), "w") as fh:
        json.dump(out, fh, separators=(",", ":"))


if __name__ == "__main__":
    main()
