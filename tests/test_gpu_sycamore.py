"""The paper's Sycamore topology and Sequences I / II on the GPU, against the oracle.

Layouts of n_c columns holding n_b and n_b - 1 qubits alternately (Fig. 1), chain order
column by column; every layer is a random one-qubit gate per qubit then fSim(1, pi/2) on
one coupler class (Sequence I: ABCD-CDAB, Sequence II: CDBA-BACD).

Tolerances as for the other parity tests: FP64 f within 1e-10 relative, identical bond
dimensions, amplitudes within 1e-9 (1e-7 at 54 qubits); FP32 / split exact-regime
statevectors within 1e-5 / 1e-3.
"""
import numpy as np
import pytest

from paper_2207_05612_amd import circuits, mps
from oracle import dmrg
from oracle import statevector as sv

import parity_bounds as pb

pytestmark = pytest.mark.gpu

FP64, FP32, BF16X3 = mps.MPS_FP64, mps.MPS_FP32, mps.MPS_BF16X3
AMP_TOL = {FP64: 1e-9, FP32: 1e-5, BF16X3: 1e-3}


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("K", [1, 2])
@pytest.mark.parametrize("prec", [FP64, FP32, BF16X3])
@pytest.mark.parametrize("sequence", ["I", "II"])
def test_small_layout_exact_regime(sequence, prec, K):
    """10 qubits (n_b = 3, n_c = 4), depth 8, chi = 32 = 2^(n/2): the statevector."""
    c = circuits.sycamore_circuit(circuits.SycamoreLayout(3, 4), 8, seed=2, sequence=sequence)
    st = mps.MPS(c.n, None, max_chi=32, precision=prec)
    for d in range(0, len(c.layers), K):
        st.apply_layers_dmrg(c.layers[d:d + K], 32, 1)
    err = rel_l2(st.statevector(), sv.run(c))
    print("sequence %s prec=%d K=%d exact-regime rel-L2 %.2e" % (sequence, prec, K, err))
    assert err < AMP_TOL[prec]


@pytest.mark.parametrize("sequence", ["I", "II"])
def test_small_layout_truncated_matches_oracle(sequence):
    c = circuits.sycamore_circuit(circuits.SycamoreLayout(3, 4), 8, seed=4, sequence=sequence)
    st = mps.MPS(c.n, None, max_chi=4, precision=FP64)
    fs = np.array([st.apply_layer_dmrg(layer, 4, 2) for layer in c.layers])
    ora = dmrg.run_circuit(c, chi=4, n_sweeps=2)
    sizes = pb.two_site_layer_sizes(c.n, 2, len(c.layers))
    fb = pb.fp64_bound(ora.step_log, sizes, 2 * 4, 1e-10)
    ab = pb.fp64_bound(ora.step_log, sizes, 2 * 4, AMP_TOL[FP64])
    err = np.max(np.abs(fs - np.array(ora.layer_f)) / np.array(ora.layer_f))
    amp = rel_l2(st.statevector(), dmrg.to_statevector(ora))
    print("sequence %s max rel f error %.2e (bound %.2e), amplitudes %.2e (bound %.2e), worst gap %.2e"
          % (sequence, err, fb, amp, ab, pb.worst_gap(ora.step_log)))
    assert err < fb
    assert st.bond_dims() == ora.bond_dims()
    assert amp < ab


@pytest.mark.parametrize("sequence", ["I", "II"])
def test_54_qubit_processor_matches_oracle(sequence):
    """The 54-qubit processor (n_b = 5, n_c = 12), its coupler classes in the order of each
    sequence with Haar couplers, four layers at chi = 8 (MPO bonds up to 256): per-layer f,
    bond dimensions and sampled amplitudes.

    The paper's fixed fSim with three one-qubit gates makes many Schmidt spectra exactly
    degenerate: for every chi from 3 to 24 some truncation of the first three layers cuts
    through a multiplet (or leaves a gap below 1e-11 S_max^2), where the kept subspace is not
    unique and two correct implementations part ways.  Haar couplers have no such ties: every
    truncation here has a gap of at least 2e-10 S_max^2 (measured with the oracle)."""
    c = circuits.sycamore_circuit(circuits.SycamoreLayout(5, 12), 4, seed=3, sequence=sequence, two_qubit="haar")
    st = mps.MPS(c.n, None, max_chi=8, precision=FP64)
    fs = np.array([st.apply_layer_dmrg(layer, 8, 1) for layer in c.layers])
    ora = dmrg.product_state(c.n)
    for layer in c.layers:
        dmrg.apply_layer(ora, layer, 8, 1)
    of = np.array(ora.layer_f)
    print("sequence %s f %s (oracle %s)" % (sequence, fs, of))
    assert np.max(np.abs(fs - of) / of) < 1e-10
    assert st.bond_dims() == ora.bond_dims()
    bits = np.random.default_rng(1).integers(0, 2, size=(32, c.n)).astype(np.uint8)
    want = np.array([dmrg.amplitude(ora, b) for b in bits])
    assert rel_l2(st.amplitudes(bits), want) < 1e-7


@pytest.mark.parametrize("sequence", ["I", "II"])
def test_54_qubit_fixed_fsim_first_layer_is_exact(sequence):
    """The first layer of either sequence couples disjoint pairs: chi = 16 holds it exactly
    (f = 1, the oracle's bond dimensions and amplitudes)."""
    c = circuits.sycamore_54_workload(0, sequence=sequence)
    st = mps.MPS(c.n, None, max_chi=16, precision=FP64)
    f = st.apply_layer_dmrg(c.layers[0], 16, 1)
    ora = dmrg.product_state(c.n)
    dmrg.apply_layer(ora, c.layers[0], 16, 1)
    assert abs(f - 1.0) < 1e-12
    assert st.bond_dims() == ora.bond_dims()
    bits = np.random.default_rng(2).integers(0, 2, size=(32, c.n)).astype(np.uint8)
    want = np.array([dmrg.amplitude(ora, b) for b in bits])
    assert rel_l2(st.amplitudes(bits), want) < 1e-9


@pytest.mark.parametrize("prec", [FP32, BF16X3])
def test_54_qubit_sequences_full_depth_properties(prec):
    """Both sequences at full depth 20 on the 54-qubit processor, chi = 64: 0 < f <= 1 up to
    the path's f tolerance, F~ the product of the layer f, bond dimensions <= chi."""
    for sequence in ("I", "II"):
        c = circuits.sycamore_54_workload(0, sequence=sequence)
        st = mps.MPS(c.n, None, max_chi=64, precision=prec)
        fs = np.array([st.apply_layer_dmrg(layer, 64, 1) for layer in c.layers])
        assert np.all(fs > 0) and np.all(fs <= 1 + 1e-4)
        fid = st.fidelity()
        assert abs(fid["log_F_tilde"] - np.sum(np.log(fs))) < 1e-9
        assert fid["n_2q"] == c.n_2q and max(st.bond_dims()) <= 64
        print("sequence %s chi 64 prec %d: F~ %.3e, eps~ %.4f" % (sequence, prec, fid["F_tilde"], fid["eps_tilde"]))
