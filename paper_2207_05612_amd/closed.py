"""Closed simulation mode (Sec. IV.C): amplitudes <x|U|0> of chosen bitstrings.

The circuit is cut after layer d1.  The forward MPS U_{d1} ... U_1 |0> and the
backward MPS U_{d1+1}^dagger ... U_D^dagger |x> are both built by the
library's compression step; the amplitude is their overlap
<backward|forward> (mps_overlap), with fidelity estimate F~_forward *
F~_backward.

A layer of this library applies its one-qubit gates before its two-qubit
gates, so the daggered layers are regrouped: the first backward layer holds
the daggered two-qubit gates of the last layer, each later one the daggered
one-qubit gates of layer l together with the daggered two-qubit gates of
layer l - 1, and the last one the daggered one-qubit gates of layer d1 + 1.

This module only composes calls of the C ABI (mps_create with init_bits,
apply_layer_dmrg / apply_layer_dmrg_single_site, mps_overlap).
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from . import mps


def backward_layers(layers: Sequence) -> List[list]:
    """Layers that apply (U_m ... U_1)^dagger, one-qubit gates first in each."""
    m = len(layers)
    out: List[list] = []
    for pos in range(m, -1, -1):
        one_q = [] if pos == m else [(g[0], g[1], np.conj(np.asarray(g[2])).T) for g in layers[pos] if g[1] < 0]
        two_q = [] if pos == 0 else [(g[0], g[1], np.conj(np.asarray(g[2])).T) for g in layers[pos - 1] if g[1] >= 0]
        out.append(one_q + two_q)
    return out


def closed_amplitude(circuit, bits, chi: int, n_sweeps: int, d1: int, precision: int = mps.MPS_FP64,
                     update: str = "two-site"):
    """(<x|U|0>, forward state, backward state) with the cut after layer d1 (0 <= d1 <= depth).

    The caller closes the returned states (MPS.close)."""
    if not 0 <= d1 <= len(circuit.layers):
        raise ValueError("0 <= d1 <= depth required")
    bits = np.asarray(bits, dtype=np.uint8)
    fwd = mps.MPS(circuit.n, None, max_chi=chi, precision=precision)
    for layer in circuit.layers[:d1]:
        fwd.apply_layer_dmrg(layer, chi, n_sweeps, update=update)
    bwd = mps.MPS(circuit.n, bits, max_chi=chi, precision=precision)
    for layer in backward_layers(circuit.layers[d1:]):
        bwd.apply_layer_dmrg(layer, chi, n_sweeps, update=update)
    return mps.overlap(bwd, fwd), fwd, bwd
