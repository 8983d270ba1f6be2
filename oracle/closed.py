"""Closed simulation mode of the FP64 oracle -- TEST INFRASTRUCTURE ONLY.

The paper's closed mode (Sec. IV.C) computes the amplitude <x|U|0> of a
given bitstring x from two MPS: the forward MPS U_{d1} ... U_1 |0> and the
backward MPS U_{d1+d2+1}^dagger ... U_D^dagger |x>, both built with the
compression step, and contracts them with the middle part of depth d2 (the
paper's D2) between them, exactly:
  <x|U|0> = <backward| U_{d1+d2} ... U_{d1+1} |forward>.
The middle layers are the dense MPO of step_mpo, contracted site by site
between the two MPS (mpo_sandwich); d2 = 0 is the plain overlap.

A layer applies its one-qubit gates, then its two-qubit gates.  The daggered
layers applied to |x> therefore regroup as
  [2q_D^+], [1q_D^+, 2q_{D-1}^+], ..., [1q_{d1+2}^+, 2q_{d1+1}^+], [1q_{d1+1}^+]
so that each regrouped layer again has its one-qubit gates first.

Metropolis sampling over amplitudes (App. on Metropolis sampling): from x_t a
uniformly random x' is proposed and accepted with probability
min(|Psi_x'/Psi_x_t|^2, 1); a refused move repeats x_t.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from . import dmrg


def dagger_layers(layers: Sequence) -> List[list]:
    """U_1^+ ... U_m^+ applied right to left, as layers (one-qubit gates first)."""
    out = []
    m = len(layers)
    for idx in range(m, -1, -1):
        regrouped = []
        if idx < m:                       # one-qubit gates of layer idx (0-based), daggered
            regrouped += [(q0, q1, np.asarray(u).conj().T) for q0, q1, u in layers[idx] if q1 < 0]
        if idx > 0:                       # two-qubit gates of layer idx - 1, daggered
            regrouped += [(q0, q1, np.asarray(u).conj().T) for q0, q1, u in layers[idx - 1] if q1 >= 0]
        out.append(regrouped)
    return out


def mpo_sandwich(bra, layers, ket) -> complex:
    """<bra| U_K ... U_1 |ket> for the layers U_1 .. U_K (one-qubit gates first in each),
    contracted exactly: E_{k+1}[p', c', q'] = sum conj(B_k[p,s,p']) W_k[c,s,t,c'] A_k[q,t,q']
    E_k[p, c, q] with the dense step MPO W of the layers (no layers: the plain overlap)."""
    if not layers:
        return dmrg.overlap(bra, ket)
    w = dmrg.step_mpo(ket.n, layers)
    e = np.ones((1, 1, 1), dtype=np.complex128)
    for b, wk, a in zip(bra.tensors, w, ket.tensors):
        x = np.einsum("pcq,qtr->pctr", e, a)
        x = np.einsum("pctr,cstd->psdr", x, wk)
        e = np.einsum("psdr,psu->udr", x, b.conj())
    return complex(e[0, 0, 0])


def closed_amplitude(circuit, bits, chi: int, n_sweeps: int, d1: int, update: str = "two-site", d2: int = 0):
    """<x|U|0> from the forward MPS of layers [0, d1), the exact middle layers [d1, d1 + d2)
    and the backward MPS of layers [d1 + d2, D).

    Returns (amplitude, forward state, backward state); the fidelity estimate of
    the amplitude is F~_forward * F~_backward (the middle part is exact)."""
    if not (0 <= d1 and 0 <= d2 and d1 + d2 <= len(circuit.layers)):
        raise ValueError("0 <= d1, 0 <= d2, d1 + d2 <= depth required")
    fwd = dmrg.product_state(circuit.n)
    for layer in circuit.layers[:d1]:
        dmrg.apply_layer(fwd, layer, chi, n_sweeps, update=update)
    bwd = dmrg.product_state(circuit.n, bits)
    for layer in dagger_layers(circuit.layers[d1 + d2:]):
        dmrg.apply_layer(bwd, layer, chi, n_sweeps, update=update)
    return mpo_sandwich(bwd, circuit.layers[d1:d1 + d2], fwd), fwd, bwd


def metropolis(amplitude, x0, proposals, uniforms):
    """Metropolis chain over bitstrings with the given proposals and uniform draws.

    amplitude(bits) -> complex.  Returns (chain of visited bitstrings, including x0,
    number of accepted moves)."""
    x = np.asarray(x0, dtype=np.uint8).copy()
    px = abs(amplitude(x)) ** 2
    chain = [x.copy()]
    accepted = 0
    for prop, u in zip(proposals, uniforms):
        pp = abs(amplitude(prop)) ** 2
        ratio = 1.0 if px == 0.0 else min(pp / px, 1.0)
        if u < ratio:
            x, px = np.asarray(prop, dtype=np.uint8).copy(), pp
            accepted += 1
        chain.append(x.copy())
    return chain, accepted
