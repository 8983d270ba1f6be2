"""Closed simulation mode and MPS-MPS overlap on the GPU, through the C ABI.

* mps_overlap against the oracle's overlap of the same states (FP64 MPS
  tensors: 1e-12 relative), <phi|phi> = 1, and <x|phi> equal to the
  amplitude of x.
* closed_amplitude (forward MPS of the first d1 layers, backward MPS of the
  daggered rest from |x>) against the statevector amplitude in the exact
  regime (FP64: 1e-10 relative to the largest amplitude magnitude), and
  against the oracle's closed mode in the truncated regime (FP64: 1e-9).
* The exact middle part of depth d2 (mps_overlap_layers, Sec. IV.C D2): the
  statevector amplitude in the exact regime for d2 = 1..3 at several cuts,
  the whole circuit as the middle part between the product states |0> and
  <x| (exact at chi = 1), and the oracle's closed mode with d2 = 1..3 in the
  truncated regime, FP64 and the split precision.
"""
import numpy as np
import pytest

from paper_2207_05612_amd import circuits, closed, mps
from oracle import closed as oclosed
from oracle import dmrg
from oracle import statevector as sv

pytestmark = pytest.mark.gpu

FP64, FP32 = mps.MPS_FP64, mps.MPS_FP32


def index_of(bits):
    return int("".join(str(int(b)) for b in bits), 2)


def test_backward_layers_match_oracle_regrouping():
    c = circuits.plain_fp64_workload(4)
    a = closed.backward_layers(c.layers[3:])
    b = oclosed.dagger_layers(c.layers[3:])
    assert len(a) == len(b)
    for la, lb in zip(a, b):
        assert [(g[0], g[1]) for g in la] == [(g[0], g[1]) for g in lb]
        for ga, gb in zip(la, lb):
            assert np.array_equal(ga[2], gb[2])


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_overlap(prec):
    c = circuits.plain_fp64_workload(2)
    g1 = mps.MPS(c.n, None, max_chi=8, precision=prec)
    g2 = mps.MPS(c.n, None, max_chi=16, precision=prec)
    o1, o2 = dmrg.product_state(c.n), dmrg.product_state(c.n)
    for d, layer in enumerate(c.layers[:5]):
        g1.apply_layer_dmrg(layer, 8, 2)
        dmrg.apply_layer(o1, layer, 8, 2)
        if d < 4:
            g2.apply_layer_dmrg(layer, 16, 2)
            dmrg.apply_layer(o2, layer, 16, 2)
    got = mps.overlap(g2, g1)
    # the overlap of the two GPU states against the statevectors of the same GPU states
    want = np.vdot(g2.statevector(), g1.statevector())
    assert abs(got - want) < 1e-12 * max(1.0, abs(want))
    assert abs(mps.overlap(g1, g1) - 1.0) < 1e-12
    if prec == FP64:
        assert abs(got - dmrg.overlap(o2, o1)) < 1e-10
    bits = np.random.default_rng(1).integers(0, 2, size=c.n).astype(np.uint8)
    x = mps.MPS(c.n, bits, max_chi=1, precision=prec)
    assert abs(mps.overlap(x, g1) - g1.amplitudes(bits[None, :])[0]) < 1e-12
    with pytest.raises(mps.MpsError):
        mps.overlap(mps.MPS(c.n + 1, None, max_chi=1, precision=prec), g1)


@pytest.mark.parametrize("update", ["two-site", "single-site"])
@pytest.mark.parametrize("d1", [0, 4, 8])
def test_closed_amplitude_exact_regime(d1, update):
    c = circuits.plain_fp64_workload(0)
    psi = sv.run(c)
    scale = np.abs(psi).max()
    rng = np.random.default_rng(d1 + 7)
    for _ in range(2):
        bits = rng.integers(0, 2, size=c.n)
        amp, fwd, bwd = closed.closed_amplitude(c, bits, chi=64, n_sweeps=2, d1=d1, update=update)
        assert abs(amp - psi[index_of(bits)]) < 1e-10 * scale, (amp, psi[index_of(bits)])
        assert abs(fwd.fidelity()["F_tilde"] - 1.0) < 1e-10
        assert abs(bwd.fidelity()["F_tilde"] - 1.0) < 1e-10
        fwd.close()
        bwd.close()


@pytest.mark.parametrize("update", ["two-site", "single-site"])
def test_closed_amplitude_truncated_matches_oracle(update):
    c = circuits.random_circuit(circuits.grid_from_shape(4, 4), 8, seed=5)
    rng = np.random.default_rng(11)
    for d1 in (3, 5):
        bits = rng.integers(0, 2, size=c.n)
        amp, fwd, bwd = closed.closed_amplitude(c, bits, chi=8, n_sweeps=2, d1=d1, update=update)
        want, ofwd, obwd = oclosed.closed_amplitude(c, bits, chi=8, n_sweeps=2, d1=d1, update=update)
        print("d1=%d %s amp %.3e%+.3ej oracle %.3e%+.3ej" % (d1, update, amp.real, amp.imag, want.real, want.imag))
        assert abs(amp - want) < 1e-9 * max(abs(want), 1e-3)
        assert abs(fwd.fidelity()["log_F_tilde"] - ofwd.log_f) < 1e-9
        assert abs(bwd.fidelity()["log_F_tilde"] - obwd.log_f) < 1e-9
        fwd.close()
        bwd.close()


@pytest.mark.parametrize("d1,d2", [(0, 1), (2, 2), (3, 3), (5, 3), (0, 8)])
def test_closed_amplitude_middle_part_exact(d1, d2):
    """Exact regime (chi = 64 = 2^(n/2)), and d1 = 0, d2 = D at chi = 1 (both MPS are product
    states; the whole circuit is the exact middle part): the statevector amplitude."""
    c = circuits.plain_fp64_workload(0)
    psi = sv.run(c)
    scale = np.abs(psi).max()
    chi = 1 if d2 == len(c.layers) else 64
    rng = np.random.default_rng(10 * d1 + d2)
    for _ in range(2):
        bits = rng.integers(0, 2, size=c.n)
        amp, fwd, bwd = closed.closed_amplitude(c, bits, chi=chi, n_sweeps=2, d1=d1, d2=d2)
        assert abs(amp - psi[index_of(bits)]) < 1e-10 * scale, (amp, psi[index_of(bits)])
        fwd.close()
        bwd.close()


@pytest.mark.parametrize("prec", [FP64, mps.MPS_BF16X3])
@pytest.mark.parametrize("d2", [1, 2, 3])
def test_closed_amplitude_middle_part_truncated(d2, prec):
    """16 qubits, chi = 8, cut after layer 3 with d2 middle layers, against the oracle's closed
    mode with the same split (its middle part is the dense MPO of the layers); FP64 to 1e-9,
    split precision to 1e-3 relative (the amplitude budget of that path)."""
    c = circuits.random_circuit(circuits.grid_from_shape(4, 4), 8, seed=5)
    rng = np.random.default_rng(20 + d2)
    for _ in range(2):
        bits = rng.integers(0, 2, size=c.n)
        amp, fwd, bwd = closed.closed_amplitude(c, bits, chi=8, n_sweeps=2, d1=3, d2=d2, precision=prec)
        want, _, _ = oclosed.closed_amplitude(c, bits, chi=8, n_sweeps=2, d1=3, d2=d2)
        print("d2=%d prec=%d amp %.4e%+.4ej oracle %.4e%+.4ej" % (d2, prec, amp.real, amp.imag, want.real, want.imag))
        tol = 1e-9 if prec == FP64 else 1e-3
        assert abs(amp - want) < tol * max(abs(want), 1e-3)
        fwd.close()
        bwd.close()


def test_overlap_layers_errors():
    c = circuits.plain_fp64_workload(0)
    a = mps.MPS(c.n, None, max_chi=4, precision=FP64)
    b = mps.MPS(c.n, None, max_chi=4, precision=FP64)
    with pytest.raises(mps.MpsError) as e:
        mps.overlap_layers(a, [[(0, 1, np.eye(4)), (1, 2, np.eye(4))]], b)     # overlapping gates
    assert e.value.code == mps.MPS_ERR_ARG
    assert abs(mps.overlap_layers(a, [], b) - 1.0) < 1e-14
    assert abs(mps.overlap_layers(a, [[(0, -1, circuits.SQRT_X)]], b) - circuits.SQRT_X[0, 0]) < 1e-14


def test_metropolis_chain_matches_oracle():
    """The library's closed-mode Metropolis chain (amplitudes from forward/backward MPS at
    chi = 2^(n/2)) and the oracle's chain over exact statevector amplitudes, with the same
    seeded proposals and uniforms, accept the same moves (no uniform lies within 1e-9 of its
    acceptance ratio for these draws, which the test checks)."""
    c = circuits.plain_fp64_workload(0)
    psi = sv.run(c)
    props, us = circuits.metropolis_draws(c.n, 120, seed=21)
    amps = closed.ClosedAmplitudes(c, chi=64, n_sweeps=1, d1=4)
    try:
        chain, acc, weights = closed.metropolis(amps, props[0], props[1:], us[1:])
    finally:
        amps.close()
    exact = lambda b: psi[index_of(b)]
    ochain, oacc = oclosed.metropolis(exact, props[0], props[1:], us[1:])
    p = np.abs(psi) ** 2
    cur = index_of(props[0])
    for prop, u in zip(props[1:], us[1:]):
        ratio = min(p[index_of(prop)] / p[cur], 1.0)
        assert abs(u - ratio) > 1e-9
        if u < ratio:
            cur = index_of(prop)
    assert acc == oacc
    assert all(np.array_equal(a, b) for a, b in zip(chain, ochain))
    for x, w in zip(chain, weights):
        assert abs(w - p[index_of(x)]) < 1e-10 * p.max()
    print("accepted %d of %d proposals" % (acc, len(props) - 1))
