"""The exact on-GPU statevector and the measurement of an MPS against it, through the C ABI.

* sv_apply_layer against the oracle's brute-force statevector, every amplitude (FP64 in
  both: within 1e-13 absolute for unit-norm states of up to 2^20 amplitudes, a few
  roundings per gate).
* sv_compare_mps against the oracle's plain definitions of F (eq:F-sup) and F_B
  (eq:FB-sup) applied to the GPU MPS's own statevector and the oracle's exact state.
* At 32 qubits, where the oracle cannot hold the state: circuits of four independent
  8-qubit blocks.  Every amplitude is a product of block amplitudes that the oracle
  computes one by one; an exact MPS has F = 1 and 1 + F_B = prod_b (1 + F_B,b).
"""
import math

import numpy as np
import pytest

from paper_2207_05612_amd import circuits, mps
from oracle import analysis, chaotic, dmrg
from oracle import statevector as sv

pytestmark = pytest.mark.gpu

FP64 = mps.MPS_FP64


def all_amplitudes(s):
    return s.amplitudes_at(np.arange(2 ** s.n))


def test_layers_match_oracle_12_qubits():
    """Every layer of the 12-qubit workload, plus layers with reversed pairs, one-qubit gates
    only (an odd number of them), repeated one-qubit gates on a site, and an empty layer."""
    c = circuits.plain_fp64_workload(0)
    rng = np.random.default_rng(3)
    haar = lambda: circuits.haar_unitary_from_normals(rng.standard_normal(32))
    extra = [
        [(5, 2, haar()), (11, 0, haar()), (3, -1, circuits.SQRT_X)],
        [(1, -1, circuits.SQRT_Y), (4, -1, circuits.SQRT_W), (9, -1, circuits.SQRT_X)],
        [(7, -1, circuits.SQRT_X), (7, -1, circuits.SQRT_Y), (7, 8, haar()), (7, -1, circuits.SQRT_W)],
        [],
    ]
    g = mps.Statevector(c.n)
    psi = sv.zero_state(c.n)
    for layer in c.layers + extra:
        g.apply_layer(layer)
        psi = sv.apply_layer(psi, c.n, layer)
        err = np.max(np.abs(all_amplitudes(g) - psi))
        assert err < 1e-13, err
    g.close()


def test_layers_match_oracle_20_qubits_from_bits():
    c = circuits.random_circuit(circuits.grid_from_shape(5, 4), 6, seed=7)
    bits = np.random.default_rng(2).integers(0, 2, size=c.n).astype(np.uint8)
    g = mps.Statevector(c.n, bits)
    psi = sv.zero_state(c.n, bits)
    for layer in c.layers:
        g.apply_layer(layer)
        psi = sv.apply_layer(psi, c.n, layer)
    err = np.max(np.abs(all_amplitudes(g) - psi))
    print("20 qubits max amplitude error %.2e" % err)
    assert err < 1e-13


def test_errors_leave_the_state_unchanged():
    c = circuits.plain_fp64_workload(1)
    g = mps.Statevector(c.n)
    g.apply_layer(c.layers[0])
    ref = all_amplitudes(g)
    with pytest.raises(mps.MpsError) as e:
        g.apply_layer([(0, 1, np.eye(4)), (1, 2, np.eye(4))])
    assert e.value.code == mps.MPS_ERR_ARG
    with pytest.raises(mps.MpsError) as e:
        g.apply_layer([(0, 12, np.eye(4))])
    assert e.value.code == mps.MPS_ERR_ARG
    with pytest.raises(mps.MpsError) as e:
        g.amplitudes_at([0, 4096])
    assert e.value.code == mps.MPS_ERR_ARG
    assert np.array_equal(all_amplitudes(g), ref)
    m = mps.MPS(c.n + 1, None, max_chi=2, precision=FP64)
    with pytest.raises(mps.MpsError) as e:
        g.compare(m)
    assert e.value.code == mps.MPS_ERR_ARG


@pytest.mark.parametrize("prec", [mps.MPS_FP64, mps.MPS_FP32, mps.MPS_BF16X3])
def test_compare_matches_the_definitions(prec):
    """F, F_B and norms of a truncated 16-qubit MPS (chi = 8) against the exact state."""
    c = circuits.random_circuit(circuits.grid_from_shape(4, 4), 8, seed=5)
    st = mps.MPS(c.n, None, max_chi=8, precision=prec)
    g = mps.Statevector(c.n)
    for layer in c.layers:
        st.apply_layer_dmrg(layer, 8, 2)
        g.apply_layer(layer)
    psi = sv.run(c)
    phi = st.statevector()
    r = g.compare(st)
    print("F %.6e (F~ %.6e) F_B %.6e" % (r["F"], st.fidelity()["F_tilde"], r["F_B"]))
    assert abs(r["F"] - analysis.fidelity(phi, psi)) < 1e-12
    assert abs(r["F_B"] - analysis.xeb_exact(phi, psi)) < 1e-10
    assert abs(r["overlap"] - np.vdot(phi, psi)) < 1e-12
    assert abs(r["norm_exact"] - 1.0) < 1e-12 and abs(r["norm_mps"] - np.vdot(phi, phi).real) < 1e-12


def block_circuit(n_blocks, width, depth, seed):
    """Layers whose two-qubit gates stay inside contiguous blocks of `width` chain sites."""
    rng = np.random.default_rng(seed)
    n = n_blocks * width
    layers = []
    for d in range(depth):
        layer = [(q, -1, circuits.ONE_QUBIT_SET[int(rng.integers(3))]) for q in range(n)]
        for b in range(n_blocks):
            perm = rng.permutation(width) + b * width
            for k in range(0, width - 1, 2):
                layer.append((int(perm[k]), int(perm[k + 1]),
                              circuits.haar_unitary_from_normals(rng.standard_normal(32))))
        layers.append(layer)
    return circuits.Circuit(n=n, layers=layers, label="blocks")


def test_full_size_32_qubits_block_circuit():
    """32 qubits (64 GiB of amplitudes): sampled amplitudes equal the products of the oracle's
    block amplitudes; an exact MPS (chi = 16) has F = 1 and 1 + F_B = prod_b (1 + F_B,b)."""
    width, n_blocks = 8, 4
    c = block_circuit(n_blocks, width, 6, seed=11)
    g = mps.Statevector(c.n)
    for layer in c.layers:
        g.apply_layer(layer)
    blocks = []
    for b in range(n_blocks):
        lo, hi = b * width, (b + 1) * width
        sub = [[(q0 - lo, (q1 - lo) if q1 >= 0 else -1, u) for q0, q1, u in layer
                if lo <= q0 < hi] for layer in c.layers]
        blocks.append(sv.run(circuits.Circuit(n=width, layers=sub)))
    idx = np.random.default_rng(1).integers(0, 2 ** 32, size=512, dtype=np.int64)
    idx[:2] = [0, 2 ** 32 - 1]
    want = np.ones(len(idx), dtype=np.complex128)
    for b in range(n_blocks):
        shift = (n_blocks - 1 - b) * width
        want *= blocks[b][(idx >> shift) & (2 ** width - 1)]
    got = g.amplitudes_at(idx)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    print("32 qubits sampled amplitude error (relative to the largest) %.2e" % err)
    assert err < 1e-11
    st = mps.MPS(c.n, None, max_chi=16, precision=FP64)
    for layer in c.layers:
        st.apply_layer_dmrg(layer, 16, 1)
    r = g.compare(st)
    want_fb = np.prod([1 + analysis.xeb_exact(bk, bk) for bk in blocks]) - 1
    print("32 qubits F %.15f F_B %.10f (oracle %.10f)" % (r["F"], r["F_B"], want_fb))
    assert abs(r["F"] - 1.0) < 1e-10 and abs(r["norm_exact"] - 1.0) < 1e-10
    assert abs(r["F_B"] - want_fb) < 1e-9 * max(1.0, want_fb)
    g.close()


def test_xeb_sample_estimate_matches_exact_value():
    """eq:FB-estim with samples from the GPU MPS and P from the GPU statevector agrees with
    eq:FB-sup within 5 standard errors (20 qubits, chi = 8, 50000 samples)."""
    c = circuits.random_circuit(circuits.grid_from_shape(5, 4), 10, seed=2)
    st = mps.MPS(c.n, None, max_chi=8, precision=FP64)
    g = mps.Statevector(c.n)
    for layer in c.layers:
        st.apply_layer_dmrg(layer, 8, 1)
        g.apply_layer(layer)
    r = g.compare(st)
    bits = st.sample(50000, seed=3)
    idx = np.array([circuits.bits_to_index(b) for b in bits], dtype=np.int64)
    p = np.abs(g.amplitudes_at(idx)) ** 2
    est = analysis.xeb_estimate(p, c.n)
    sd = np.std(2.0 ** c.n * p) / np.sqrt(len(p))
    print("F %.4f F~ %.4f sqrt(F) %.4f F_B %.4f estimate %.4f +- %.4f" % (
        r["F"], st.fidelity()["F_tilde"], np.sqrt(r["F"]), r["F_B"], est, sd))
    assert abs(est - r["F_B"]) < 5 * sd


@pytest.mark.parametrize("cut", [3, 8, 12])
def test_schmidt_weights_match_the_svd(cut):
    """Squared Schmidt values of a 16-qubit state at cuts with the smaller side on either
    end, against LAPACK's SVD of the oracle's state (1e-13 absolute, unit-norm state), and the
    best-MPS weights sum_{mu < chi} S_mu^2."""
    c = circuits.random_circuit(circuits.grid_from_shape(4, 4), 10, seed=8)
    g = mps.Statevector(c.n)
    for layer in c.layers:
        g.apply_layer(layer)
    want = sv.schmidt_values(sv.run(c), c.n, cut) ** 2
    for chi in (1, 5, 64):
        kept, total, s2 = g.schmidt(cut, chi)
        assert abs(total - 1.0) < 1e-12
        assert abs(kept - np.sum(want[:chi])) < 1e-12
    assert np.max(np.abs(s2 - want)) < 1e-13
    with pytest.raises(mps.MpsError):
        g.schmidt(0, 4)


def test_depth_curve_matches_the_oracle():
    """analysis.depth_curve (12 qubits, chi = 6) against the same quantities built from the
    oracle: its MPS, its statevector, LAPACK's Schmidt values and its F / F_B definitions."""
    from paper_2207_05612_amd import analysis as gan
    c = circuits.plain_fp64_workload(2)
    recs = gan.depth_curve(c, chi=6, n_sweeps=2, n_samples=2000, seed=1)
    st = dmrg.product_state(c.n)
    psi = sv.zero_state(c.n)
    for d, (layer, rec) in enumerate(zip(c.layers, recs)):
        dmrg.apply_layer(st, layer, 6, 2)
        psi = sv.apply_layer(psi, c.n, layer)
        phi = dmrg.to_statevector(st)
        assert rec["depth"] == d + 1
        assert abs(rec["F"] - analysis.fidelity(phi, psi)) < 1e-9
        assert abs(rec["F_B"] - analysis.xeb_exact(phi, psi)) < 1e-8
        assert abs(rec["F_tilde"] - math.exp(st.log_f)) < 1e-9
        s2 = sv.schmidt_values(psi, c.n, c.n // 2) ** 2
        assert abs(rec["F_SVD"] - np.sum(s2[:6]) / np.sum(s2)) < 1e-12
        assert rec["F"] <= rec["F_SVD"] + 1e-12            # no bond-6 MPS beats the best cut
        assert abs(rec["eps_opt"] - chaotic.eps_opt(6, c.n, d + 1)) < 1e-12
        assert abs(rec["F_B_estimate"] - rec["F_B"]) < 5 * rec["F_B_estimate_sd"] + 1e-12
    print("depth F F~ F_B F_SVD:", [(r["depth"], round(r["F"], 4), round(r["F_tilde"], 4), round(r["F_B"], 4),
                                     round(r["F_SVD"], 4)) for r in recs])


def test_linear_xeb_of_split_samples_against_oracle_probabilities():
    """The bench's XEB leg at 20 qubits: bitstrings sampled from the split-precision MPS, scored
    with the probabilities of the FP64 path's MPS (analysis.linear_xeb), against the exact value
    2^N sum_x Q(x) P(x) - 1 with Q from the split MPS's statevector and P from the oracle's MPS
    (eq:FB-sup / eq:FB-estim), within 5 standard errors."""
    from paper_2207_05612_amd import analysis as gan
    c = circuits.random_circuit(circuits.grid_from_shape(5, 4), 8, seed=4)
    split = mps.MPS(c.n, None, max_chi=16, precision=mps.MPS_BF16X3)
    ref = mps.MPS(c.n, None, max_chi=16, precision=FP64)
    for layer in c.layers:
        split.apply_layer_dmrg(layer, 16, 2)
        ref.apply_layer_dmrg(layer, 16, 2)
    ora = dmrg.run_circuit(c, chi=16, n_sweeps=2)
    want = analysis.xeb_exact(dmrg.to_statevector(ora), split.statevector())
    est, sd, bits = gan.linear_xeb(split, ref, 200000, seed=7)
    print("XEB estimate %.5f +- %.5f, exact against the oracle MPS %.5f" % (est, sd, want))
    assert abs(est - want) < 5 * sd
    split.close()
    ref.close()
