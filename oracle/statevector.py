"""Brute-force statevector simulation (FP64) -- oracle test infrastructure.

The Schroedinger approach of the paper's review (eq:perfect): keep all 2^n
amplitudes and apply the gates one by one.  Site 0 is the most significant
bit of the statevector index (the tensor index i_1 of the paper's Psi).
"""
from __future__ import annotations

import numpy as np


def zero_state(n: int, bits=None) -> np.ndarray:
    psi = np.zeros(2 ** n, dtype=np.complex128)
    idx = 0
    if bits is not None:
        for b in bits:
            idx = (idx << 1) | int(b)
    psi[idx] = 1.0
    return psi


def apply_1q(psi: np.ndarray, n: int, q: int, u: np.ndarray) -> np.ndarray:
    t = psi.reshape((2,) * n)
    t = np.tensordot(u, t, axes=([1], [q]))          # new axis 0 = output of q
    t = np.moveaxis(t, 0, q)
    return t.reshape(-1)


def apply_2q(psi: np.ndarray, n: int, q0: int, q1: int, u: np.ndarray) -> np.ndarray:
    """U acts with row/column index 2*s_q0 + s_q1."""
    t = psi.reshape((2,) * n)
    u4 = u.reshape(2, 2, 2, 2)                       # [s0, s1, t0, t1]
    t = np.tensordot(u4, t, axes=([2, 3], [q0, q1]))  # axes 0,1 = outputs of q0,q1
    t = np.moveaxis(t, [0, 1], [q0, q1])
    return t.reshape(-1)


def apply_layer(psi: np.ndarray, n: int, layer) -> np.ndarray:
    """One layer: every 1q gate first (in list order), then the 2q gates."""
    for q0, q1, u in layer:
        if q1 < 0:
            psi = apply_1q(psi, n, q0, u)
    for q0, q1, u in layer:
        if q1 >= 0:
            psi = apply_2q(psi, n, q0, q1, u)
    return psi


def run(circuit, depth=None, bits=None) -> np.ndarray:
    n = circuit.n
    psi = zero_state(n, bits)
    layers = circuit.layers if depth is None else circuit.layers[:depth]
    for layer in layers:
        psi = apply_layer(psi, n, layer)
    return psi


def layer_matrix(n: int, layer) -> np.ndarray:
    """Dense 2^n x 2^n matrix of one layer (columns = images of basis states)."""
    dim = 2 ** n
    out = np.zeros((dim, dim), dtype=np.complex128)
    for x in range(dim):
        e = np.zeros(dim, dtype=np.complex128)
        e[x] = 1.0
        out[:, x] = apply_layer(e, n, layer)
    return out


def schmidt_values(psi: np.ndarray, n: int, cut: int) -> np.ndarray:
    """Singular values of psi split as (sites < cut) x (sites >= cut)."""
    m = psi.reshape(2 ** cut, 2 ** (n - cut))
    return np.linalg.svd(m, compute_uv=False)


def best_mps_weight(psi: np.ndarray, n: int, chi: int) -> np.ndarray:
    """Per cut, the weight sum_{mu < chi} S_mu^2 kept by Eckart-Young truncation."""
    out = []
    for cut in range(1, n):
        s = schmidt_values(psi, n, cut)
        out.append(float(np.sum(s[:chi] ** 2)))
    return np.array(out)
