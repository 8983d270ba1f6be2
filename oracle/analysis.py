"""Fidelity measures of a simulated state -- TEST INFRASTRUCTURE ONLY.

Plain definitions, written out from the paper:
  * the fidelity F = |<Psi_Q|Psi_P>|^2 of the simulated state Psi_Q against the
    perfect state Psi_P (eq:F-sup);
  * the linear cross-entropy F_B = 2^N sum_x P(x) Q(x) - 1 with P(x) = |Psi_P(x)|^2
    and Q(x) = |Psi_Q(x)|^2 (eq:FB-sup);
  * its sample estimator 2^N <P(x_i)> - 1 over samples x_i drawn from Q
    (eq:FB-estim).
"""
from __future__ import annotations

import numpy as np


def fidelity(psi_q: np.ndarray, psi_p: np.ndarray) -> float:
    """|<Psi_Q|Psi_P>|^2 (eq:F-sup)."""
    return float(abs(np.vdot(psi_q, psi_p)) ** 2)


def xeb_exact(psi_q: np.ndarray, psi_p: np.ndarray) -> float:
    """2^N sum_x P(x) Q(x) - 1 (eq:FB-sup)."""
    p = np.abs(psi_p) ** 2
    q = np.abs(psi_q) ** 2
    return float(len(p) * np.sum(p * q) - 1.0)


def xeb_estimate(p_at_samples: np.ndarray, n_qubits: int) -> float:
    """2^N times the mean ideal probability of the sampled bitstrings, minus 1 (eq:FB-estim)."""
    return float(2.0 ** n_qubits * np.mean(p_at_samples) - 1.0)
