"""Write oracle reference values for the larger parity cases (calls only ``oracle/``).

Usage: python tests/golden/make_golden.py [name ...]

Each case runs the FP64 oracle on a seeded synthetic circuit and stores, as
JSON next to this file: per-layer f_delta, log F~, N_2g, the per-update log
(f, sum S^2, chi', the relative truncation gap S_k / S_{k+1} - 1 at the cut
and the first-order sensitivity kappa of the state to the cut), the final bond dimensions and the amplitudes <x|phi> of 64 seeded random
bitstrings.  QAOA cases store, per (gamma, beta) set, the per-layer f_delta,
log F~ and <C> = sum_E (1 - <Z_u Z_v>) / 2.  The GPU parity tests compare
against these files.
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
    # the same grid at chi 128 and 256, full depth 14, seeds 0-3
    **{"grid36_chi%d_seed%d_d14" % (chi, seed): dict(kind="grid36", seed=seed, chi=chi, sweeps=2, depth=14)
       for chi in (128, 256) for seed in range(4)},
    # 54-qubit fSim workload of the benchmark, first 6 layers at chi 32
    "sycamore54_chi32_seed0_d6": dict(kind="syc54", seed=0, chi=32, sweeps=2, depth=6),
    # the same workload, first 10 layers at chi 256 (the bonds saturate from layer 4 on)
    "sycamore54_chi256_seed0_d10": dict(kind="syc54", seed=0, chi=256, sweeps=2, depth=10),
    # ragged batch (circuits.batched_instances(64)): the instances with chi <= 128 that the
    # oracle finishes in minutes, full depth
    **{"batched64_inst%d" % i: dict(kind="batched64", index=i, sweeps=2) for i in (1, 8, 9, 10, 17)},
    # QAOA MaxCut on a random 3-regular graph of 54 nodes, p = 4, the first 8 of the seeded
    # (gamma, beta) sets, chi 64, 2 sweeps, every brick layer of the SWAP network
    "qaoa54_p4_chi64_sets8": dict(kind="qaoa54", seed=0, chi=64, sweeps=2, p=4, sets=8),
}


def circuit_for(case):
    if case["kind"] == "batched64":
        return circuits.batched_instances(64)[case["index"]][0]
    if case["kind"] == "grid36":
        return circuits.grid36_workload(case["seed"])
    if case["kind"] == "syc54":
        return circuits.sycamore_like_54_workload(case["seed"])
    raise ValueError(case["kind"])


def bitstrings(n, count=64, seed=12345):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2, size=(count, n)).astype(np.uint8)


def qaoa_instances(case):
    n = 54
    edges = circuits.random_regular_graph(n, 3, seed=case["seed"])
    sets = circuits.qaoa_parameter_sets(128, case["p"], seed=case["seed"])[:case["sets"]]
    return edges, [circuits.qaoa_maxcut_swap_network(n, edges, g, b) for g, b in sets]


def make_qaoa(name, case):
    t0 = time.time()
    edges, qs = qaoa_instances(case)
    out = []
    for q in qs:
        st = dmrg.run_circuit(q.circuit, chi=case["chi"], n_sweeps=case["sweeps"])
        cval = circuits.maxcut_expectation_from_zz(
            edges, q.final_position, lambda a, b: dmrg.expectation_zz(st, min(a, b), max(a, b)))
        out.append({"layer_f": st.layer_f, "log_f_tilde": st.log_f, "n_2q": st.n_2q, "maxcut": cval,
                    "bond_dims": st.bond_dims(), "min_gap": min(r.gap for r in st.step_log),
                    "max_kappa": max(r.kappa for r in st.step_log),
                    "step_log_len": len(st.step_log)})
        print(name, "set %d: <C> = %.6f, F~ = %.4e (%.0f s)" % (len(out) - 1, cval, np.exp(st.log_f),
                                                                 time.time() - t0), flush=True)
    rec = {"case": case, "n": 54, "edges": edges, "sets": out, "oracle_seconds": time.time() - t0}
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(rec, fh)
    print(name, "done in %.1f s" % rec["oracle_seconds"], flush=True)


def make(name):
    case = CASES[name]
    if case["kind"] == "qaoa54":
        return make_qaoa(name, case)
    c = circuit_for(case)
    if case["kind"] == "batched64":
        case = dict(case, chi=circuits.batched_instances(64)[case["index"]][1], depth=len(c.layers))
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
        "step_gap": [r.gap if np.isfinite(r.gap) else None for r in st.step_log],
        "step_kappa": [r.kappa if np.isfinite(r.kappa) else None for r in st.step_log],
        "bits_seed": 12345, "amp_re": [a.real for a in amps], "amp_im": [a.imag for a in amps],
        "oracle_seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(rec, fh)
    print(name, "done in %.1f s" % rec["oracle_seconds"], flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES)):
        make(name)
