"""Write oracle reference values for the larger parity cases (calls only ``oracle/``).

Usage: python tests/golden/make_golden.py [name ...]

Each case runs the FP64 oracle on a seeded synthetic circuit and stores, as
JSON next to this file: per-layer f_delta, log F~, N_2g, the per-update log
(f, sum S^2, chi'), the final bond dimensions and the amplitudes <x|phi> of 64
seeded random bitstrings.  The GPU parity tests compare against these files.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2207_05612_amd import circuits  # noqa: E402
from oracle import dmrg  # noqa: E402

CASES = {
    # 36 qubits on a 6x6 grid, depth 14, Haar gates, chi 64, 2 sweeps, seeds 0-3
    "grid36_chi64_seed0": dict(kind="grid36", seed=0, chi=64, sweeps=2, depth=14),
    "grid36_chi64_seed1": dict(kind="grid36", seed=1, chi=64, sweeps=2, depth=14),
    "grid36_chi64_seed2": dict(kind="grid36", seed=2, chi=64, sweeps=2, depth=14),
    "grid36_chi64_seed3": dict(kind="grid36", seed=3, chi=64, sweeps=2, depth=14),
    # the same grid at chi 128, first 8 layers
    "grid36_chi128_seed0_d8": dict(kind="grid36", seed=0, chi=128, sweeps=2, depth=8),
    # 54-qubit fSim workload of the benchmark, first 6 layers at chi 32
    "sycamore54_chi32_seed0_d6": dict(kind="syc54", seed=0, chi=32, sweeps=2, depth=6),
}


def circuit_for(case):
    if case["kind"] == "grid36":
        return circuits.grid36_workload(case["seed"])
    if case["kind"] == "syc54":
        return circuits.sycamore_like_54_workload(case["seed"])
    raise ValueError(case["kind"])


def bitstrings(n, count=64, seed=12345):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2, size=(count, n)).astype(np.uint8)


def make(name):
    case = CASES[name]
    c = circuit_for(case)
    t0 = time.time()
    st = dmrg.run_circuit(c, chi=case["chi"], n_sweeps=case["sweeps"], depth=case["depth"])
    bits = bitstrings(c.n)
    amps = [dmrg.amplitude(st, b) for b in bits]
    f_tilde, log_f, eps = dmrg.fidelity(st)
    rec = {
        "case": case, "n": c.n, "label": c.label,
        "layer_f": st.layer_f, "log_f_tilde": log_f, "n_2q": st.n_2q, "eps_tilde": eps,
        "step_f": [r.f for r in st.step_log], "step_sum_s2": [r.sum_s2 for r in st.step_log],
        "step_chi": [r.chi_kept for r in st.step_log], "bond_dims": st.bond_dims(),
        "bits_seed": 12345, "amp_re": [a.real for a in amps], "amp_im": [a.imag for a in amps],
        "oracle_seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(rec, fh)
    print(name, "done in %.1f s" % rec["oracle_seconds"], flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES)):
        make(name)
