"""Amplitude bounds of the reduced-precision paths in the truncated regime.

The target bounds are 1e-5 (FP32 contractions) and 1e-3 (split BF16) on the
relative L2 error of amplitudes against the FP64 oracle.  In the truncated
regime the kept subspace of a cut can be ill-conditioned: when the smallest
kept and the largest discarded singular value are close, any perturbation of
the local tensor -- FP32 rounding included -- rotates the kept subspace, and
the state changes without a bug.  The oracle records, per truncation, the
relative gap S_k / S_{k+1} - 1 and the first-order sensitivity kappa of the
normalised state to a relative perturbation of the Gram matrix (Davis-Kahan;
see oracle.dmrg.truncated_svd_gap).  A layer contributes the largest kappa of
its truncations; rounding of relative size u then moves the final state by at
most about u * sum over layers of that kappa, to first order.

The bound of a test is therefore max(target, C_FIRST_ORDER * u * sum kappa),
with the constant and the unit roundoffs fixed here from the arithmetic (not
from measured errors):
  * u: FP32 2^-24; split BF16x3 2^-23 (the three-term split drops terms below
    2^-24 of each product, plus FP32 accumulation); split BF16x2 2^-16 (the
    dropped lo*lo term and the residual of the two-term split);
  * C_FIRST_ORDER = 10: the factor 2 of the first-order bound (the left and
    the right kept subspace both rotate), times the several roundings of a
    step (local tensor, environments, intermediate products) and the FP32
    accumulation over long contractions.
Where the target bound applies (u * sum kappa small), the test asserts the
target itself.

Per-layer f_delta: 1e-4 relative (the target of the reduced-precision
paths) for FP32 and split BF16x3.  The two-term split BF16x2 has unit
roundoff 2^-16, so the same first-order constant gives C_FIRST_ORDER * 2^-16
= 1.5e-4: it cannot promise the 1e-4 target and is held to that bound (its
use is the 1e-3 amplitude budget, not the fidelity target); where ill-conditioned cuts have moved
the state, its f_delta moves with it (f_bound).  Every test also reports the worst gap and the
MPS-MPS overlap error 1 - |<phi_gpu|phi_oracle>|^2, and asserts the overlap error against the
square of the same bound (for normalised states it is at most the squared
L2 distance).
"""
import math

import numpy as np

from oracle import dmrg

FP64, FP32, BF16X2, BF16X3 = 0, 1, 2, 3
AMP_TARGET = {FP64: 1e-9, FP32: 1e-5, BF16X2: 1e-3, BF16X3: 1e-3}
UNIT_ROUNDOFF = {FP64: 2.0 ** -53, FP32: 2.0 ** -24, BF16X3: 2.0 ** -23, BF16X2: 2.0 ** -16}
C_FIRST_ORDER = 10.0
# 1 - |<a|b>|^2 of two unit FP64 MPS is computed with an absolute error of a few
# hundred ulps (a chain of transfer-matrix products, then a cancellation near 1)
OVERLAP_FLOOR = 1e-13
F_TARGET = {FP32: 1e-4, BF16X3: 1e-4, BF16X2: C_FIRST_ORDER * UNIT_ROUNDOFF[BF16X2]}


def layer_chunks(step_log, layer_sizes):
    out, i = [], 0
    for m in layer_sizes:
        out.append(step_log[i:i + m])
        i += m
    assert i == len(step_log)
    return out


def sum_layer_kappa(records, layer_sizes):
    """Sum over layers of the largest kappa of the layer's truncations (records: oracle
    StepRecords or (gap, kappa) pairs; layer_sizes: records per layer)."""
    total = 0.0
    for chunk in layer_chunks(list(records), layer_sizes):
        ks = [r.kappa if hasattr(r, "kappa") else r[1] for r in chunk]
        ks = [k for k in ks if k is not None]
        total += max(ks, default=0.0)
    return total


def f_bound(prec, amp_err):
    """Bound on the relative per-layer f_delta error of a run whose final amplitudes differ from the
    oracle's by amp_err (relative L2).  FP32 and split BF16x3: the 1e-4 target.  Split BF16x2: its
    own first-order bound C_FIRST_ORDER u, plus twice the deviation of the state entering the layer
    (a layer's f_delta is a normalised quadratic form of that state, so to first order its relative
    change is at most twice the state's), for which the final amplitude error stands in."""
    if prec == BF16X2:
        return F_TARGET[BF16X2] + 2.0 * amp_err
    return F_TARGET[prec]


def fp64_bound(records, layer_sizes, order, target):
    """Bound of an FP64-path quantity (per-layer f_delta, amplitudes) against the oracle: the
    target, or the first-order rule of the reduced precisions where the oracle's truncations are
    ill-conditioned.  Both sides are FP64, so the perturbation that a cut amplifies is the
    backward error of the two eigensolvers, about order * eps (eps = 2^-52, order = the largest
    Gram matrix, 2 chi), not the contraction's unit roundoff."""
    u = order * 2.0 ** -52
    return max(target, C_FIRST_ORDER * u * sum_layer_kappa(records, layer_sizes))


def worst_gap(records):
    gs = [r.gap if hasattr(r, "gap") else r[0] for r in records]
    gs = [g for g in gs if g is not None and math.isfinite(g)]
    return min(gs, default=math.inf)


def amp_bound(prec, kappa_sum):
    """max(target, C_FIRST_ORDER * u * sum kappa)."""
    if prec == FP64:
        return AMP_TARGET[FP64]
    return max(AMP_TARGET[prec], C_FIRST_ORDER * UNIT_ROUNDOFF[prec] * kappa_sum)


def two_site_layer_sizes(n, n_sweeps, n_layers):
    return [1 + n_sweeps * (n - 1)] * n_layers


def gpu_tensors(st):
    return [st.tensor(k) for k in range(st.n)]


def overlap_error(st, oracle_state):
    """1 - |<phi_gpu|phi_oracle>|^2 / (<phi_gpu|phi_gpu> <phi_oracle|phi_oracle>), by the
    oracle's transfer-matrix overlap of the GPU's tensors with its own."""
    g = dmrg.OracleMPS(tensors=gpu_tensors(st), center=0)
    ov = dmrg.overlap(g, oracle_state)
    ng = dmrg.overlap(g, g).real
    no = dmrg.overlap(oracle_state, oracle_state).real
    return max(0.0, 1.0 - abs(ov) ** 2 / (ng * no))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
