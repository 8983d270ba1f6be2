"""Measuring the simulation against the exact state (Sec. VI and VII), on the GPU.

Runs one circuit through the compression step (an MPS) and through the exact
statevector side by side and records, after every step:
  * F = |<phi|psi>|^2 (eq:F-sup) and the estimate F~ = prod f_delta (eq:Ftilde-sup);
  * F_B = 2^N sum P Q - 1 (eq:FB-sup) and, optionally, its sample estimate
    (eq:FB-estim) with bitstrings drawn from the MPS;
  * the error rates eps = 1 - F^(1/N_2g) (eq:epsilon) and eps~ from F~;
  * eps_SVD of the best MPS: the weight kept by the chi largest Schmidt values of the
    exact state at the middle cut (Sec. VI, best possible MPS);
  * the chaotic optimum: the best bond-chi MPS of a chaotic state keeps the
    fidelity F_opt = 4 chi / 2^(N/2) (leading term of App. B, eq:F_chi_rel), and
    eps_opt = 1 - F_opt^(2/(N D)) (the error per gate with N D / 2 gates,
    App. B).  The closed form printed as eq:error_rate_asymptotics has its
    log(4 chi) term four times too small; the derivation's form is used.

Everything runs in the library (C ABI calls); this module only composes them.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional

import numpy as np

from . import circuits, mps


def chaotic_optimum_error(chi: int, n_qubits: int, depth: int) -> float:
    """Error per gate of the best bond-chi MPS of a chaotic state (App. B): with
    F_opt = 4 chi / 2^(N/2) and N D / 2 two-qubit gates, eps = 1 - F_opt^(2/(N D)),
    i.e. 1 - exp((2 / (N D)) (log(4 chi) - (N/2) log 2)).  For F_opt >= 1 the
    optimum is exact and the error 0."""
    log_f = math.log(4.0 * chi) - 0.5 * n_qubits * math.log(2.0)
    if log_f >= 0.0:
        return 0.0
    return -math.expm1(2.0 * log_f / (n_qubits * depth))


def linear_xeb(sampler, reference, n_samples: int, seed: int):
    """Linear cross-entropy (eq:FB-estim): F_B ~ 2^N <P(x)> - 1 over bitstrings x drawn from
    the MPS `sampler` (exact sequential sampling), P(x) = |<x|reference>|^2 the probabilities of
    the MPS `reference` (the exact state's when it is the exact state; a proxy otherwise).
    Returns (estimate, standard error, bitstrings)."""
    bits = sampler.sample(n_samples, seed)
    p = np.abs(reference.amplitudes(bits)) ** 2
    scale = 2.0 ** sampler.n
    est = float(scale * np.mean(p) - 1.0)
    sd = float(scale * np.std(p) / math.sqrt(n_samples))
    return est, sd, bits


def error_rate(fid: float, n_2q: int) -> float:
    """eq:epsilon: 1 - F^(1/N_2g) (0 before any two-qubit gate)."""
    if n_2q <= 0:
        return 0.0
    return 1.0 - max(fid, 0.0) ** (1.0 / n_2q)


def depth_curve(circuit, chi: int, n_sweeps: int = 1, layers_per_step: int = 1,
                precision: int = mps.MPS_FP64, update: str = "two-site", n_samples: int = 0,
                seed: int = 0, schmidt: bool = True, max_depth: Optional[int] = None,
                bond_caps: Optional[List[int]] = None) -> List[Dict]:
    """One record per compression step (K = layers_per_step layers each).  bond_caps (n + 1
    per-bond caps, e.g. circuits.group_bond_profile for a grouping with chi between groups)
    replaces the single chi in the truncations."""
    n = circuit.n
    layers = circuit.layers if max_depth is None else circuit.layers[:max_depth]
    caps = chi if bond_caps is None else list(bond_caps)
    st = mps.MPS(n, None, max_chi=chi if bond_caps is None else max(bond_caps), precision=precision)
    ex = mps.Statevector(n)
    out: List[Dict] = []
    n_2q = 0
    try:
        for d in range(0, len(layers), layers_per_step):
            step = layers[d:d + layers_per_step]
            f = st.apply_layers_dmrg(step, caps, n_sweeps, update=update)
            for layer in step:
                ex.apply_layer(layer)
                n_2q += sum(1 for g in layer if g[1] >= 0)
            r = ex.compare(st)
            fid = st.fidelity()
            depth = d + len(step)
            rec = {"depth": depth, "n_2q": n_2q, "f_delta": f, "F": r["F"], "F_tilde": fid["F_tilde"],
                   "F_B": r["F_B"], "eps": error_rate(r["F"], n_2q), "eps_tilde": error_rate(fid["F_tilde"], n_2q),
                   "eps_opt": chaotic_optimum_error(chi, n, depth), "max_bond": max(st.bond_dims())}
            if schmidt and min(n // 2, n - n // 2) <= 14:
                kept, total, _ = ex.schmidt(n // 2, chi)
                rec["F_SVD"] = kept / total
                rec["eps_SVD"] = error_rate(kept / total, n_2q)
            if n_samples > 0:
                bits = st.sample(n_samples, seed + depth)
                idx = np.array([circuits.bits_to_index(b) for b in bits], dtype=np.int64)
                p = np.abs(ex.amplitudes_at(idx)) ** 2
                rec["F_B_estimate"] = float(2.0 ** n * np.mean(p) - 1.0)
                rec["F_B_estimate_sd"] = float(np.std(2.0 ** n * p) / math.sqrt(n_samples))
            out.append(rec)
    finally:
        st.close()
        ex.close()
    return out
