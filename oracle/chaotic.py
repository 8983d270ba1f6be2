"""Chaotic-optimum formulas of the paper's Appendix B -- oracle test infrastructure.

* A Porter-Thomas state: complex Gaussian amplitudes of variance
  sigma^2 = 1/(2 * 2^N) per real component (App. B.1).
* Quadrant law of the rescaled singular values s = 2^{N/4} S: density
  sqrt(4 - s^2)/pi on [0, 2] (App. B.2).
* Scaling function g(x) = 2 cos(A^{-1}(pi x)/2) with A(theta) = theta - sin(theta).
* Kept weight F(chi) = integral_0^{chi / 2^{N/2}} g(x)^2 dx, leading term
  4 chi / 2^{N/2} (eq. chaotic_opt).
* Reading of eq. error_rate_asymptotics: the derivation gives
  eps_opt = 1 - F_opt^{2/(N D)}; the printed closed form has its second term
  four times too small, so the derived form is used.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate


def porter_thomas(n_qubits: int, rng: np.random.Generator) -> np.ndarray:
    sigma = np.sqrt(1.0 / (2.0 * 2 ** n_qubits))
    return rng.normal(0.0, sigma, 2 ** n_qubits) + 1j * rng.normal(0.0, sigma, 2 ** n_qubits)


def _area(theta: float) -> float:
    return theta - np.sin(theta)


def _area_inverse(y: float) -> float:
    """Inverse of A(theta) = theta - sin(theta) on [0, 2 pi] by bisection."""
    lo, hi = 0.0, 2.0 * np.pi
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _area(mid) < y:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def g(x: float) -> float:
    """Scaling function of the singular values: S_mu = 2^{-N/4} g(mu / 2^{N/2})."""
    return 2.0 * np.cos(0.5 * _area_inverse(np.pi * x))


def count_above(s0: float) -> float:
    """C(s0) = (1/pi) integral_{s0}^{2} sqrt(4 - s^2) ds (fraction above s0)."""
    return _area(2.0 * np.arccos(s0 / 2.0)) / np.pi


def kept_weight(chi: int, n_qubits: int) -> float:
    """F(chi) = integral_0^{chi/2^{N/2}} g(x)^2 dx."""
    upper = chi / 2.0 ** (n_qubits / 2.0)
    val, _ = integrate.quad(lambda x: g(x) ** 2, 0.0, upper, limit=200)
    return float(val)


def f_opt_leading(chi: int, n_qubits: int) -> float:
    return 4.0 * chi / 2.0 ** (n_qubits / 2.0)


def eps_opt(chi: int, n_qubits: int, depth: int) -> float:
    """Chaotic-optimum error per gate, eps = 1 - F_opt^{2/(N D)}."""
    return 1.0 - f_opt_leading(chi, n_qubits) ** (2.0 / (n_qubits * depth))
