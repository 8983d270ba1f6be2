"""Closed simulation mode (Sec. IV.C): amplitudes <x|U|0> of chosen bitstrings.

The circuit is cut into three parts: the forward MPS U_{d1} ... U_1 |0> and
the backward MPS U_{d1+d2+1}^dagger ... U_D^dagger |x> are both built by the
library's compression step, and the middle part of depth d2 (the paper's D2)
is contracted exactly between them (mps_overlap_layers):
  <x|U|0> = <backward| U_{d1+d2} ... U_{d1+1} |forward>,
with fidelity estimate F~_forward * F~_backward.  d2 = 0 is the plain overlap
(mps_overlap).

A layer of this library applies its one-qubit gates before its two-qubit
gates, so the daggered layers are regrouped: the first backward layer holds
the daggered two-qubit gates of the last layer, each later one the daggered
one-qubit gates of layer l together with the daggered two-qubit gates of
layer l - 1, and the last one the daggered one-qubit gates of layer d1 + 1.

This module only composes calls of the C ABI (mps_create with init_bits,
apply_layer_dmrg / apply_layer_dmrg_single_site, mps_overlap_layers).
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


def _check_split(circuit, d1: int, d2: int) -> None:
    if not (0 <= d1 and 0 <= d2 and d1 + d2 <= len(circuit.layers)):
        raise ValueError("0 <= d1, 0 <= d2 and d1 + d2 <= depth required")


def closed_amplitude(circuit, bits, chi: int, n_sweeps: int, d1: int, precision: int = mps.MPS_FP64,
                     update: str = "two-site", d2: int = 0):
    """(<x|U|0>, forward state, backward state): forward MPS of layers [0, d1), exact middle
    part [d1, d1 + d2), backward MPS of layers [d1 + d2, D).

    The caller closes the returned states (MPS.close)."""
    _check_split(circuit, d1, d2)
    bits = np.asarray(bits, dtype=np.uint8)
    fwd = mps.MPS(circuit.n, None, max_chi=chi, precision=precision)
    for layer in circuit.layers[:d1]:
        fwd.apply_layer_dmrg(layer, chi, n_sweeps, update=update)
    bwd = mps.MPS(circuit.n, bits, max_chi=chi, precision=precision)
    for layer in backward_layers(circuit.layers[d1 + d2:]):
        bwd.apply_layer_dmrg(layer, chi, n_sweeps, update=update)
    return mps.overlap_layers(bwd, circuit.layers[d1:d1 + d2], fwd), fwd, bwd


class ClosedAmplitudes:
    """Amplitudes <x|U|0> of one circuit for many bitstrings: the forward MPS of the
    first d1 layers is built once, a backward MPS per bitstring, the next d2 layers are
    the exact middle part."""

    def __init__(self, circuit, chi: int, n_sweeps: int, d1: int, precision: int = mps.MPS_FP64,
                 update: str = "two-site", d2: int = 0):
        _check_split(circuit, d1, d2)
        self.circuit, self.chi, self.n_sweeps, self.precision, self.update = circuit, chi, n_sweeps, precision, update
        self.middle = circuit.layers[d1:d1 + d2]
        self.back = backward_layers(circuit.layers[d1 + d2:])
        self.fwd = mps.MPS(circuit.n, None, max_chi=chi, precision=precision)
        for layer in circuit.layers[:d1]:
            self.fwd.apply_layer_dmrg(layer, chi, n_sweeps, update=update)
        self.log_f_backward = []        # log F~ of each backward MPS

    def __call__(self, bits) -> complex:
        bwd = mps.MPS(self.circuit.n, np.asarray(bits, dtype=np.uint8), max_chi=self.chi, precision=self.precision)
        try:
            for layer in self.back:
                bwd.apply_layer_dmrg(layer, self.chi, self.n_sweeps, update=self.update)
            self.log_f_backward.append(bwd.fidelity()["log_F_tilde"])
            return mps.overlap_layers(bwd, self.middle, self.fwd)
        finally:
            bwd.close()

    def close(self) -> None:
        self.fwd.close()


def metropolis(amplitude, x0, proposals, uniforms):
    """Metropolis chain over bitstrings (App. on Metropolis sampling): the proposal of each
    step is accepted when its uniform draw is below min(|Psi_x'|^2 / |Psi_x|^2, 1).
    Returns (visited bitstrings including x0, accepted moves, |Psi|^2 of each visited one)."""
    cur = np.asarray(x0, dtype=np.uint8).copy()
    w_cur = abs(amplitude(cur)) ** 2
    visited, weights, n_acc = [cur.copy()], [w_cur], 0
    for prop, u in zip(proposals, uniforms):
        w_new = abs(amplitude(prop)) ** 2
        if w_cur == 0.0 or u < min(w_new / w_cur, 1.0):
            cur, w_cur = np.asarray(prop, dtype=np.uint8).copy(), w_new
            n_acc += 1
        visited.append(cur.copy())
        weights.append(w_cur)
    return visited, n_acc, weights
