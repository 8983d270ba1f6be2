"""Qubit groupings on the GPU (apply_layers_dmrg_bonds): per-bond caps against the oracle.

A grouping of the qubits into tensors with bond chi between them is run as an MPS of
single qubits whose bonds inside a group are uncapped and whose bonds between groups are
capped at chi (circuits.group_bond_profile).

* A constant profile is the single-chi step, bit for bit.
* Haar couplers on the Sycamore layout (no degenerate Schmidt spectra, so every truncation
  is unique): per-layer f within 1e-10 of the oracle in FP64, identical bond dimensions,
  statevectors within 1e-9; FP32 and split f within 1e-4.
* The paper's fixed fSim: layers whose couplers stay inside the column groups have
  f_delta = 1 (to 1e-12 in FP64) at chi = 4 between groups, at 21 qubits.
"""
import numpy as np
import pytest

from paper_2207_05612_amd import circuits, mps
from oracle import dmrg
from oracle import statevector as sv

pytestmark = pytest.mark.gpu

FP64, FP32, BF16X3 = mps.MPS_FP64, mps.MPS_FP32, mps.MPS_BF16X3


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_constant_profile_equals_single_chi():
    c = circuits.plain_fp64_workload(1)
    a = mps.MPS(c.n, None, max_chi=8, precision=FP64)
    b = mps.MPS(c.n, None, max_chi=8, precision=FP64)
    prof = [1] + [6] * (c.n - 1) + [1]
    for layer in c.layers:
        assert a.apply_layer_dmrg(layer, 6, 2) == b.apply_layers_dmrg([layer], prof, 2)
    assert np.array_equal(a.statevector(), b.statevector())


@pytest.mark.parametrize("update", ["two-site", "single-site"])
@pytest.mark.parametrize("columns", [[2, 2], [1, 2, 1]])
def test_grouping_matches_oracle_fp64(columns, update):
    lay = circuits.SycamoreLayout(3, 4)
    prof = circuits.group_bond_profile(circuits.sycamore_column_groups(lay, columns), 2)
    c = circuits.sycamore_circuit(lay, 8, seed=6, sequence="I", two_qubit="haar")
    st = mps.MPS(c.n, None, max_chi=max(prof), precision=FP64)
    fs = np.array([st.apply_layers_dmrg([layer], prof, 2, update=update) for layer in c.layers])
    ora = dmrg.product_state(c.n)
    for layer in c.layers:
        dmrg.apply_layers(ora, [layer], prof, 2, update=update)
    of = np.array(ora.layer_f)
    print("columns %s %s f %s" % (columns, update, np.round(fs, 6)))
    assert np.max(np.abs(fs - of) / of) < 1e-10
    assert st.bond_dims() == ora.bond_dims()
    assert rel_l2(st.statevector(), dmrg.to_statevector(ora)) < 1e-9


@pytest.mark.parametrize("prec", [FP32, BF16X3])
def test_grouping_reduced_precision_f(prec):
    lay = circuits.SycamoreLayout(3, 4)
    prof = circuits.group_bond_profile(circuits.sycamore_column_groups(lay, [2, 2]), 2)
    c = circuits.sycamore_circuit(lay, 8, seed=6, sequence="I", two_qubit="haar")
    st = mps.MPS(c.n, None, max_chi=max(prof), precision=prec)
    fs = np.array([st.apply_layers_dmrg([layer], prof, 2) for layer in c.layers])
    ora = dmrg.product_state(c.n)
    for layer in c.layers:
        dmrg.apply_layers(ora, [layer], prof, 2)
    assert np.max(np.abs(fs - np.array(ora.layer_f)) / np.array(ora.layer_f)) < 1e-4


def test_layers_inside_groups_are_trivial_21_qubits():
    """Sequence I with the fixed fSim on 21 qubits (n_b = 4, n_c = 6), columns grouped in pairs:
    the A and C layers stay inside the groups (f = 1 and the exact image of the layer), the B
    and D layers truncate the bonds between groups at chi = 4."""
    lay = circuits.SycamoreLayout(4, 6)
    sizes = circuits.sycamore_column_groups(lay, [2, 2, 2])
    prof = circuits.group_bond_profile(sizes, 4)
    cuts = np.cumsum(sizes)[:-1]
    c = circuits.sycamore_circuit(lay, 8, seed=1, sequence="I")
    st = mps.MPS(c.n, None, max_chi=max(prof), precision=FP64)
    for d, layer in enumerate(c.layers):
        before = st.statevector()
        f = st.apply_layers_dmrg([layer], prof, 1)
        letter = circuits.SEQUENCE_I[d % 8]
        if letter in "AC":
            target = sv.apply_layer(before, c.n, layer)
            assert abs(f - 1.0) < 1e-12, (d, letter, f)
            assert abs(abs(np.vdot(st.statevector(), target)) - 1.0) < 1e-10
        print("layer %d (%s) f=%.6f bonds at group cuts %s" % (d, letter, f, [st.bond_dims()[k] for k in cuts]))
        assert all(st.bond_dims()[k] <= 4 for k in cuts)
    assert st.fidelity()["F_tilde"] < 0.999


def test_row_grouping_trivial_layers_21_qubits():
    """H1 (row pairs, the chain relabelled so each group is contiguous) on 21 qubits: the A and
    D layers are exact at chi = 4 between groups; the bonds between groups stay <= 4."""
    lay = circuits.SycamoreLayout(4, 6)
    order, sizes = circuits.sycamore_row_groups(lay, 0)
    c = circuits.relabel_circuit(circuits.sycamore_circuit(lay, 8, seed=2, sequence="I"), order)
    prof = circuits.group_bond_profile(sizes, 4)
    cuts = np.cumsum(sizes)[:-1]
    st = mps.MPS(c.n, None, max_chi=max(prof), precision=FP64)
    for d, layer in enumerate(c.layers):
        before = st.statevector()
        f = st.apply_layers_dmrg([layer], prof, 1)
        if circuits.SEQUENCE_I[d % 8] in "AD":
            assert abs(f - 1.0) < 1e-12, (d, f)
            target = sv.apply_layer(before, c.n, layer)
            assert abs(abs(np.vdot(st.statevector(), target)) - 1.0) < 1e-10
        assert all(st.bond_dims()[k] <= 4 for k in cuts)
    assert st.fidelity()["F_tilde"] < 0.999


@pytest.mark.parametrize("direction,trivial", [("up", "AB"), ("down", "CD")])
def test_diagonal_grouping_21_qubits(direction, trivial):
    """D groupings (one group per diagonal line, the chain relabelled so that each line is
    contiguous) on 21 qubits with the paper's fixed fSim: the layers along the lines are exact
    at chi = 4 between groups, the bonds between groups stay <= 4; and with Haar couplers on the
    same grouping, per-layer f and bond dimensions as the oracle's (FP64)."""
    lay = circuits.SycamoreLayout(4, 6)
    order, sizes = circuits.sycamore_diagonal_groups(lay, direction)
    prof = circuits.group_bond_profile(sizes, 4)
    cuts = np.cumsum(sizes)[:-1]
    c = circuits.relabel_circuit(circuits.sycamore_circuit(lay, 8, seed=2, sequence="I"), order)
    st = mps.MPS(c.n, None, max_chi=max(prof), precision=FP64)
    for d, layer in enumerate(c.layers):
        before = st.statevector()
        f = st.apply_layers_dmrg([layer], prof, 1)
        if circuits.SEQUENCE_I[d % 8] in trivial:
            assert abs(f - 1.0) < 1e-12, (d, f)
            target = sv.apply_layer(before, c.n, layer)
            assert abs(abs(np.vdot(st.statevector(), target)) - 1.0) < 1e-10
        assert all(st.bond_dims()[k] <= 4 for k in cuts)
    assert st.fidelity()["F_tilde"] < 0.999
    st.close()
    h = circuits.relabel_circuit(circuits.sycamore_circuit(lay, 6, seed=6, sequence="I", two_qubit="haar"), order)
    g = mps.MPS(h.n, None, max_chi=max(prof), precision=FP64)
    fs = np.array([g.apply_layers_dmrg([layer], prof, 2) for layer in h.layers])
    ora = dmrg.product_state(h.n)
    for layer in h.layers:
        dmrg.apply_layers(ora, [layer], prof, 2)
    of = np.array(ora.layer_f)
    print("diagonal %s f %s" % (direction, np.round(fs, 6)))
    assert np.max(np.abs(fs - of) / of) < 1e-10
    assert g.bond_dims() == ora.bond_dims()
    g.close()
