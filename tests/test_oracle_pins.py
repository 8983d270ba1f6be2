"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Every test here runs on the CPU.  Each pin checks the oracle against something
other than itself: a brute-force statevector, a closed form, an invariant, a
published known-answer vector, or brute force on a tiny input.
"""
import math
import os

import numpy as np
import pytest

from paper_2207_05612_amd import circuits
from oracle import chaotic, dmrg, philox
from oracle import statevector as sv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ gate set -----
def test_gates_unitary_and_square_roots():
    for g, p in zip(circuits.ONE_QUBIT_SET, (circuits.PAULI_X, circuits.PAULI_Y, circuits.PAULI_W)):
        assert np.allclose(g.conj().T @ g, np.eye(2), atol=1e-14)
        assert np.allclose(g @ g, -1j * p, atol=1e-14)           # sqrt(G)^2 = -iG
    assert np.allclose(circuits.fsim(0.0, 0.0), np.eye(4), atol=1e-15)
    f = circuits.fsim(np.pi / 2, 0.0)                              # iSWAP-like block
    assert np.allclose(np.abs(f[1, 2]), 1.0) and np.allclose(f[1, 1], 0.0, atol=1e-15)
    rng = np.random.default_rng(5)
    acc = np.zeros((4, 4))
    for _ in range(4000):
        u = circuits.haar_unitary_from_normals(rng.standard_normal(32))
        assert np.allclose(u.conj().T @ u, np.eye(4), atol=1e-13)
        acc += np.abs(u) ** 2
    acc /= 4000
    assert np.allclose(acc, 0.25, atol=0.02)                      # E|U_ij|^2 = 1/4


def test_snake_grid_and_patterns():
    g = circuits.grid_from_shape(3, 4)                             # width 3, 4 rows
    assert g.width == 3 and g.rows == 4
    sites = sorted(g.site(r, c) for r, c in g.coords())
    assert sites == list(range(12))
    assert g.site(1, 0) == 5 and g.site(1, 2) == 3                 # odd row reversed
    for letter in "ABCD":
        pairs = g.pattern_pairs(letter)
        flat = [s for p in pairs for s in p]
        assert len(flat) == len(set(flat))                         # a matching
    # horizontal patterns are chain neighbours
    assert all(j - i == 1 for i, j in g.pattern_pairs("A") + g.pattern_pairs("B"))
    # the 12-qubit depth-8 workload has 34 two-qubit gates
    assert circuits.plain_fp64_workload(0).n_2q == 34


# --------------------------------------------------------------- MPO -------
@pytest.mark.parametrize("swap_order", [False, True])
def test_gate_split_reconstructs(swap_order):
    rng = np.random.default_rng(1)
    u = circuits.haar_unitary_from_normals(rng.standard_normal(32))
    q0, q1 = (5, 2) if swap_order else (2, 5)
    sg = dmrg.split_two_qubit(q0, q1, u)
    assert (sg.i, sg.j) == (2, 5) and sg.x.shape[0] == 4
    rec = np.einsum("ast,auv->sutv", sg.x, sg.y).reshape(4, 4)     # [(s_i s_j), (t_i t_j)]
    u4 = u.reshape(2, 2, 2, 2)
    want = (u4 if not swap_order else u4.transpose(1, 0, 3, 2)).reshape(4, 4)
    assert np.allclose(rec, want, atol=1e-13)


def test_gate_split_ranks():
    assert dmrg.split_two_qubit(0, 1, circuits.zz_phase(0.3)).x.shape[0] == 2
    assert dmrg.split_two_qubit(0, 1, circuits.SWAP).x.shape[0] == 4
    assert dmrg.split_two_qubit(0, 1, np.eye(4)).x.shape[0] == 1


def _mpo_dense(mpo):
    n = len(mpo)
    t = mpo[0][0]                                                  # [s, t, b]
    t = t.reshape(2, 2, -1)
    for k in range(1, n):
        t = np.einsum("xyb,bstc->xsytc", t, mpo[k]).reshape(2 ** (k + 1), 2 ** (k + 1), -1)
    return t[:, :, 0]


def test_mpo_equals_dense_layer():
    """The MPO contracted to a 2^n x 2^n matrix equals the ordered gate product."""
    n = 7
    rng = np.random.default_rng(3)
    haar = lambda: circuits.haar_unitary_from_normals(rng.standard_normal(32))
    layer = [(0, -1, circuits.SQRT_X), (3, -1, circuits.SQRT_Y), (3, -1, circuits.SQRT_W),
             (6, -1, circuits.SQRT_W), (5, -1, circuits.SQRT_X),
             (0, 4, haar()), (5, 1, haar()), (2, 6, haar()), (3, -1, circuits.SQRT_X)]
    mpo, gates = dmrg.layer_mpo(n, layer)
    dims = dmrg.mpo_bond_dims(mpo)
    assert dims == [1, 4, 16, 64, 64, 16, 4, 1]
    assert np.allclose(_mpo_dense(mpo), sv.layer_matrix(n, layer), atol=1e-12)


def _random_layer(n, rng, pairs):
    haar = lambda: circuits.haar_unitary_from_normals(rng.standard_normal(32))
    layer = [(int(q), -1, circuits.ONE_QUBIT_SET[int(rng.integers(3))]) for q in rng.permutation(n)[: n // 2]]
    return layer + [(a, b, haar()) for a, b in pairs]


def test_step_mpo_equals_ordered_layer_product():
    """K > 1 layers per step: the step MPO contracted to a 2^n x 2^n matrix equals
    U_3 U_2 U_1 built gate by gate from the statevector module (order of the layers, gates
    that reach past each other, q0 > q1, an empty layer in the middle)."""
    n = 6
    rng = np.random.default_rng(11)
    l1 = _random_layer(n, rng, [(0, 3), (4, 1), (2, 5)])
    l2 = []
    l3 = _random_layer(n, rng, [(1, 2), (5, 0), (3, 4)])
    l4 = _random_layer(n, rng, [(0, 1), (2, 4)])
    mpo = dmrg.step_mpo(n, [l1, l2, l3, l4])
    want = sv.layer_matrix(n, l4) @ sv.layer_matrix(n, l3) @ sv.layer_matrix(n, l1)
    assert np.allclose(_mpo_dense(mpo), want, atol=1e-12)
    # bond dimensions multiply over the layers
    per = [dmrg.mpo_bond_dims(dmrg.layer_mpo(n, l)[0]) for l in (l1, l3, l4)]
    assert dmrg.mpo_bond_dims(mpo) == [a * b * c for a, b, c in zip(*per)]


def test_mpo_rejects_overlapping_gates():
    with pytest.raises(ValueError):
        dmrg.layer_mpo(4, [(0, 1, np.eye(4)), (1, 2, np.eye(4))])


# ----------------------------------------------------- truncation rule -----
def test_truncation_eckart_young():
    rng = np.random.default_rng(7)
    m = rng.standard_normal((12, 9)) + 1j * rng.standard_normal((12, 9))
    u, s, vh, total = dmrg.truncated_svd(m, 4)
    s_all = np.linalg.svd(m, compute_uv=False)
    assert np.isclose(total, np.sum(np.abs(m) ** 2))
    assert np.allclose(s, s_all[:4])
    # best rank-4 error = discarded weight (Eckart-Young)
    err = np.linalg.norm(m - (u * s) @ vh) ** 2
    assert np.isclose(err, np.sum(s_all[4:] ** 2))
    # exact zeros are never kept, even when chi allows them
    low = rng.standard_normal((10, 3)) @ rng.standard_normal((3, 10))
    _, s2, _, _ = dmrg.truncated_svd(low.astype(np.complex128), 8)
    assert len(s2) == 3


# -------------------------------------------------- oracle vs statevector --
def test_exact_regime_plain_workload():
    """P1: chi >= 2^(n/2): the oracle is the statevector, F~ = 1 (12 qubits)."""
    c = circuits.plain_fp64_workload(0)
    st = dmrg.run_circuit(c, chi=64, n_sweeps=2)
    psi = sv.run(c)
    phi = dmrg.to_statevector(st)
    assert np.linalg.norm(phi - psi) / np.linalg.norm(psi) < 1e-12
    f_tilde, _, eps = dmrg.fidelity(st)
    assert abs(f_tilde - 1.0) < 1e-12 and abs(eps) < 1e-13
    # bond dimensions are the exact Schmidt ranks
    ranks = [1] + [int(np.count_nonzero(sv.schmidt_values(psi, c.n, k) > 1e-7))
                   for k in range(1, c.n)] + [1]
    assert st.bond_dims() == ranks
    for x in (0, 1, 1234, 4095):
        bits = [(x >> (c.n - 1 - k)) & 1 for k in range(c.n)]
        assert abs(dmrg.amplitude(st, bits) - psi[x]) < 1e-13


def test_shallow_depth_fidelity_one():
    """P2: while every exact Schmidt rank <= chi, F~ = 1."""
    c = circuits.plain_fp64_workload(1)
    st = dmrg.run_circuit(c, chi=4, n_sweeps=1, depth=2)
    assert abs(dmrg.fidelity(st)[0] - 1.0) < 1e-12


def _exact_until(c, depth, chi_exact):
    st = dmrg.run_circuit(c, chi=chi_exact, n_sweeps=1, depth=depth)
    return st


def test_single_truncated_cut_is_eckart_young():
    """P3: only one cut exceeds chi -> f_delta = top-chi Schmidt weight there."""
    c = circuits.random_brickwork(8, 10, seed=11)
    st = _exact_until(c, 9, 16)
    psi_prev = sv.run(c, depth=9)
    assert np.linalg.norm(dmrg.to_statevector(st) - psi_prev) < 1e-11
    psi = sv.run(c, depth=10)
    ranks = [int(np.count_nonzero(sv.schmidt_values(psi, 8, k) > 1e-8)) for k in range(1, 8)]
    assert ranks == [2, 4, 8, 16, 8, 4, 2]
    f = dmrg.apply_layer(st, c.layers[9], chi=8, n_sweeps=6)
    s = sv.schmidt_values(psi, 8, 4)
    assert abs(f - float(np.sum(s[:8] ** 2))) < 1e-9
    # the fitted state is the Eckart-Young truncation itself
    phi = dmrg.to_statevector(st)
    assert abs(abs(np.vdot(psi, phi)) ** 2 - f) < 1e-9


def test_invariants_truncated_regime():
    """P4: ||phi|| = 1, 0 < f <= 1, f non-decreasing, f = |<phi|U|psi>|^2."""
    c = circuits.plain_fp64_workload(2)
    st = dmrg.product_state(c.n)
    psi = sv.zero_state(c.n)
    for d, layer in enumerate(c.layers):
        before = len(st.step_log)
        prev_vec = dmrg.to_statevector(st)
        f = dmrg.apply_layer(st, layer, chi=6, n_sweeps=2)
        phi = dmrg.to_statevector(st)
        assert abs(np.linalg.norm(phi) - 1.0) < 1e-12
        assert 0.0 < f <= 1.0 + 1e-12
        fs = [r.f for r in st.step_log[before:]]
        assert all(b >= a - 1e-12 for a, b in zip(fs, fs[1:]))
        target = sv.apply_layer(prev_vec, c.n, layer)
        assert abs(abs(np.vdot(phi, target)) ** 2 - f) < 1e-11
        assert max(st.bond_dims()) <= 6


def test_fidelity_upper_bound_and_band():
    """P5: F <= min_k top-chi weight of the exact state.  P6: F~ close to F."""
    c = circuits.plain_fp64_workload(3)
    psi = sv.run(c)
    for chi in (4, 8, 16):
        st = dmrg.run_circuit(c, chi=chi, n_sweeps=2)
        phi = dmrg.to_statevector(st)
        F = abs(np.vdot(psi, phi)) ** 2
        bound = float(np.min(sv.best_mps_weight(psi, c.n, chi)))
        assert F <= bound + 1e-12
        f_tilde = dmrg.fidelity(st)[0]
        assert abs(f_tilde - F) < 0.1 * F


def test_product_state_bits_and_zero_sweeps():
    c = circuits.random_brickwork(6, 3, seed=4)
    bits = [1, 0, 1, 1, 0, 0]
    st = dmrg.run_circuit(c, chi=8, n_sweeps=0, bits=bits)
    psi = sv.run(c, bits=bits)
    assert np.linalg.norm(dmrg.to_statevector(st) - psi) < 1e-12
    assert st.center == c.n - 1 or st.center == 0


# --------------------------------------------------- chaotic optimum -------
def test_quadrant_law_scaling_function():
    assert abs(chaotic.g(0.0) - 2.0) < 1e-9 and abs(chaotic.g(1.0)) < 1e-6
    assert abs(chaotic.kept_weight(2 ** 10, 20) - 1.0) < 1e-6    # integral of g^2 over [0,1]
    assert abs(chaotic.count_above(0.0) - 1.0) < 1e-12
    # leading term 4 chi / 2^{N/2} for chi << 2^{N/2}
    assert abs(chaotic.kept_weight(1, 40) / chaotic.f_opt_leading(1, 40) - 1.0) < 1e-3


def test_truncation_of_porter_thomas_matches_chaotic_optimum():
    """P7: top-chi weight of a Porter-Thomas state = integral of g^2 (N = 20)."""
    rng = np.random.default_rng(2024)
    n_q, chi = 20, 16
    psi = chaotic.porter_thomas(n_q, rng)
    psi /= np.linalg.norm(psi)
    m = psi.reshape(2 ** (n_q // 2), 2 ** (n_q // 2))
    _, s, _, total = dmrg.truncated_svd(m, chi)
    kept = float(np.sum(s ** 2) / total)
    assert abs(kept - chaotic.kept_weight(chi, n_q)) < 0.03 * kept
    # the printed eps_opt closed form misses a factor 4 in its second term
    eps = chaotic.eps_opt(chi, n_q, 20)
    approx = (math.log(2) - 2 * math.log(4 * chi) / n_q) / 20
    assert abs(eps - approx) < 0.05 * eps


def test_random_state_moments():
    """P8: independent Haar states: <F> = 1/N, <F_B> = 0 (N = 2^6)."""
    rng = np.random.default_rng(9)
    dim, trials = 64, 4000
    fs, fbs = [], []
    for _ in range(trials):
        a = chaotic.porter_thomas(6, rng); a /= np.linalg.norm(a)
        b = chaotic.porter_thomas(6, rng); b /= np.linalg.norm(b)
        fs.append(abs(np.vdot(a, b)) ** 2)
        fbs.append(dim * np.sum(np.abs(a) ** 2 * np.abs(b) ** 2) - 1.0)
    assert abs(np.mean(fs) - 1.0 / dim) < 4 * np.std(fs) / math.sqrt(trials)
    assert abs(np.mean(fbs)) < 4 * np.std(fbs) / math.sqrt(trials)
    assert abs(np.var(fbs) - (dim - 1) / (dim + 1) ** 2) < 0.15 * (dim - 1) / (dim + 1) ** 2


# ---------------------------------------------------------- sampling -------
def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        rows = [line.split() for line in fh if line.strip() and not line.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        v = [int(x, 16) for x in row]
        assert philox.philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])


@pytest.mark.parametrize("n_sweeps", [1, 2])
def test_sampler_matches_born_rule(n_sweeps):
    """P10: chi^2 test of the sample histogram against |phi(x)|^2 (n = 6)."""
    c = circuits.random_brickwork(6, 6, seed=21)
    st = dmrg.run_circuit(c, chi=4, n_sweeps=n_sweeps)
    probs = np.abs(dmrg.to_statevector(st)) ** 2
    ns = 20000
    bits = dmrg.sample(st, ns, seed=77)
    idx = bits.astype(np.int64) @ (1 << np.arange(5, -1, -1))
    counts = np.bincount(idx, minlength=64)
    expect = probs * ns
    mask = expect > 5
    chi2 = float(np.sum((counts[mask] - expect[mask]) ** 2 / expect[mask]))
    dof = int(mask.sum()) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


# ------------------------------------------------------------- QAOA ---------
def _qaoa_direct(n, edges, gammas, betas):
    psi = np.ones(2 ** n, dtype=np.complex128) / np.sqrt(2 ** n)
    for gam, bet in zip(gammas, betas):
        for u, v in edges:
            psi = sv.apply_2q(psi, n, u, v, circuits.zz_phase(gam))
        for s in range(n):
            psi = sv.apply_1q(psi, n, s, circuits.rx(2 * bet))
    return psi


def test_regular_graph_is_simple_and_regular():
    edges = circuits.random_regular_graph(54, 3, seed=0)
    assert len(edges) == 81
    deg = np.bincount(np.array(edges).reshape(-1), minlength=54)
    assert np.all(deg == 3) and all(a < b for a, b in edges) and len(set(edges)) == 81


def test_qaoa_swap_network_equals_direct_circuit():
    """The routed chain circuit is the QAOA state, up to the tracked permutation."""
    n = 8
    edges = circuits.random_regular_graph(n, 3, seed=2)
    gammas, betas = circuits.qaoa_parameter_sets(1, 2, seed=3)[0]
    q = circuits.qaoa_maxcut_swap_network(n, edges, gammas, betas)
    psi = sv.run(q.circuit)
    logical = np.transpose(psi.reshape((2,) * n), q.final_position).reshape(-1)
    assert abs(abs(np.vdot(logical, _qaoa_direct(n, edges, gammas, betas))) - 1.0) < 1e-12
    # <C> from the oracle MPS (exact chi) equals the statevector value
    st = dmrg.run_circuit(q.circuit, chi=16, n_sweeps=1)
    c_mps = circuits.maxcut_expectation_from_zz(edges, q.final_position,
                                                lambda i, j: dmrg.expectation_zz(st, min(i, j), max(i, j)))
    probs = np.abs(_qaoa_direct(n, edges, gammas, betas)) ** 2
    c_sv = 0.0
    for x in range(2 ** n):
        bits = [(x >> (n - 1 - k)) & 1 for k in range(n)]
        c_sv += probs[x] * sum(bits[u] != bits[v] for u, v in edges)
    assert abs(c_mps - c_sv) < 1e-10


# ------------------------------------------------- single-site update ------
def test_single_site_exact_regime_matches_statevector():
    """P1 for the single-site update: chi >= 2^(n/2) keeps the state exact and F~ = 1."""
    c = circuits.plain_fp64_workload(0)
    st = dmrg.product_state(c.n)
    for layer in c.layers:
        dmrg.apply_layer(st, layer, chi=64, n_sweeps=2, update="single-site")
    psi = sv.run(c)
    phi = dmrg.to_statevector(st)
    assert np.linalg.norm(phi - psi) / np.linalg.norm(psi) < 1e-12
    assert abs(math.exp(st.log_f) - 1.0) < 1e-12
    assert st.n_2q == c.n_2q


@pytest.mark.parametrize("chi", [3, 6])
def test_single_site_invariants_and_overlap(chi):
    """P4 for the single-site update: ||phi|| = 1, every non-centre tensor an isometry, f
    non-decreasing from the zip-up over all steps of the layer, and f_delta equal to the exact
    overlap |<phi|U|psi>|^2 computed by statevector simulation of the layer."""
    c = circuits.plain_fp64_workload(3)
    st = dmrg.product_state(c.n)
    for layer in c.layers:
        before = len(st.step_log)
        prev_vec = dmrg.to_statevector(st)
        dims_before = st.bond_dims()
        f = dmrg.apply_layer(st, layer, chi=chi, n_sweeps=3, update="single-site")
        phi = dmrg.to_statevector(st)
        assert abs(np.linalg.norm(phi) - 1.0) < 1e-12
        assert 0.0 < f <= 1.0 + 1e-12
        fs = [r.f for r in st.step_log[before:]]
        assert all(b >= a - 1e-12 for a, b in zip(fs, fs[1:])), fs
        target = sv.apply_layer(prev_vec, c.n, layer)
        assert abs(abs(np.vdot(phi, target)) ** 2 - f) < 1e-11
        assert max(st.bond_dims()) <= chi
        # odd number of sweeps: the centre ends where the zip-up started
        ctr = st.center
        for k, a in enumerate(st.tensors):
            if k == ctr:
                continue
            if k < ctr:
                m = a.reshape(-1, a.shape[2])
                assert np.allclose(m.conj().T @ m, np.eye(m.shape[1]), atol=1e-12)
            else:
                m = a.reshape(a.shape[0], -1)
                assert np.allclose(m @ m.conj().T, np.eye(m.shape[0]), atol=1e-12)
        assert st.bond_dims()[0] == st.bond_dims()[-1] == 1
        del dims_before


@pytest.mark.parametrize("update", ["two-site", "single-site"])
@pytest.mark.parametrize("K", [2, 3])
def test_multi_layer_steps_exact_regime(K, update):
    """P1 with K layers per step: chi >= 2^(n/2) reproduces the statevector, F~ = 1, and the
    layer and gate counts cover every layer."""
    c = circuits.plain_fp64_workload(0)
    st = dmrg.product_state(c.n)
    for d in range(0, len(c.layers), K):
        f = dmrg.apply_layers(st, c.layers[d:d + K], chi=64, n_sweeps=2, update=update)
        assert abs(f - 1.0) < 1e-12
    psi = sv.run(c)
    assert np.linalg.norm(dmrg.to_statevector(st) - psi) / np.linalg.norm(psi) < 1e-12
    assert abs(math.exp(st.log_f) - 1.0) < 1e-12
    assert st.n_layers == len(c.layers) and st.n_2q == c.n_2q
    assert len(st.layer_f) == -(-len(c.layers) // K)


@pytest.mark.parametrize("update", ["two-site", "single-site"])
def test_multi_layer_step_invariants_truncated(update):
    """P4 with K = 2: ||phi|| = 1, 0 < f <= 1, f non-decreasing over the sweeps, and f_delta
    equal to |<phi|U_2 U_1|psi>|^2 from statevector simulation of both layers."""
    c = circuits.plain_fp64_workload(2)
    st = dmrg.product_state(c.n)
    for d in range(0, len(c.layers) - 1, 2):
        before = len(st.step_log)
        prev_vec = dmrg.to_statevector(st)
        f = dmrg.apply_layers(st, c.layers[d:d + 2], chi=6, n_sweeps=2, update=update)
        phi = dmrg.to_statevector(st)
        assert abs(np.linalg.norm(phi) - 1.0) < 1e-12
        assert 0.0 < f <= 1.0 + 1e-12
        fs = [r.f for r in st.step_log[before:]]
        if update == "single-site":
            assert all(b >= a - 1e-12 for a, b in zip(fs, fs[1:])), fs
        target = sv.apply_layer(sv.apply_layer(prev_vec, c.n, c.layers[d]), c.n, c.layers[d + 1])
        assert abs(abs(np.vdot(phi, target)) ** 2 - f) < 1e-11
        assert max(st.bond_dims()) <= 6


def test_empty_layers_leave_a_step_unchanged():
    """A step of one layer padded with empty layers (the identity) is the one-layer step."""
    c = circuits.plain_fp64_workload(1)
    a, b = dmrg.product_state(c.n), dmrg.product_state(c.n)
    for layer in c.layers[:6]:
        fa = dmrg.apply_layer(a, layer, chi=5, n_sweeps=2)
        fb = dmrg.apply_layers(b, [[], layer, []], chi=5, n_sweeps=2)
        assert abs(fa - fb) < 1e-13
    assert np.allclose(dmrg.to_statevector(a), dmrg.to_statevector(b), atol=1e-12)


def test_single_site_update_is_the_local_optimum():
    """eq:optimization with one free tensor: with every other tensor fixed, M = F/|F| maximises
    |<phi(M)|U|psi>|^2 and the maximum is |F|^2 (brute force over random perturbations)."""
    rng = np.random.default_rng(5)
    c = circuits.random_brickwork(6, 3, seed=11)
    st = dmrg.run_circuit(c, chi=3, n_sweeps=1, depth=2)
    prev_vec = dmrg.to_statevector(st)
    layer = c.layers[2]
    dmrg.apply_layer(st, layer, chi=3, n_sweeps=1, update="single-site")
    target = sv.apply_layer(prev_vec, c.n, layer)
    f_best = st.layer_f[-1]
    ctr = st.center
    base = st.tensors[ctr].copy()
    for _ in range(20):
        pert = base + 0.05 * (rng.standard_normal(base.shape) + 1j * rng.standard_normal(base.shape))
        st.tensors[ctr] = pert / np.linalg.norm(pert)
        val = abs(np.vdot(dmrg.to_statevector(st), target)) ** 2
        assert val <= f_best + 1e-12
    st.tensors[ctr] = base
    assert abs(abs(np.vdot(dmrg.to_statevector(st), target)) ** 2 - f_best) < 1e-12


# ------------------------------------------------------ closed mode ---------
def test_dagger_layers_invert_the_circuit():
    """The regrouped daggered layers applied after the circuit give back the input state."""
    from oracle import closed
    c = circuits.plain_fp64_workload(4)
    psi = sv.run(c)
    for layer in closed.dagger_layers(c.layers):
        psi = sv.apply_layer(psi, c.n, layer)
    want = sv.zero_state(c.n)
    assert np.linalg.norm(psi - want) < 1e-12


@pytest.mark.parametrize("d1", [0, 3, 8])
@pytest.mark.parametrize("update", ["two-site", "single-site"])
def test_closed_amplitude_exact_regime(d1, update):
    """Closed mode at chi = 2^(n/2): <x|U|0> equals the statevector amplitude for every split d1."""
    from oracle import closed
    c = circuits.plain_fp64_workload(0)
    psi = sv.run(c)
    rng = np.random.default_rng(d1)
    for _ in range(3):
        bits = rng.integers(0, 2, size=c.n)
        amp, fwd, bwd = closed.closed_amplitude(c, bits, chi=64, n_sweeps=2, d1=d1, update=update)
        idx = int("".join(str(int(b)) for b in bits), 2)       # site 0 = most significant bit
        assert abs(amp - psi[idx]) < 1e-12 * max(1.0, abs(psi[idx])) + 1e-13
        assert abs(fwd.log_f) < 1e-12 and abs(bwd.log_f) < 1e-12


@pytest.mark.parametrize("d1,d2,whole", [(0, 4, True), (2, 3, False), (3, 1, False), (5, 3, False)])
def test_closed_amplitude_middle_part(d1, d2, whole):
    """The exact middle part of depth d2 (Sec. IV.C, D2): in the exact regime (chi = 64) the
    amplitude equals the statevector's for every split; with d1 = 0 and d2 = D the two MPS
    are the product states |0> and |x> and the amplitude is exact at any chi (chi = 1 here),
    so the sandwich contraction alone is pinned against the brute-force statevector.  That
    case uses an 8-qubit circuit of depth 4: the middle part's dense MPO multiplies the bond
    dimensions of its layers (up to 4^d2), and 4^8 on 12 qubits does not fit in memory."""
    from oracle import closed
    c = circuits.random_circuit(circuits.grid_from_shape(2, 4), 4, seed=3) if whole else circuits.plain_fp64_workload(0)
    psi = sv.run(c)
    rng = np.random.default_rng(10 * d1 + d2)
    chi = 1 if (d1 == 0 and d2 == len(c.layers)) else 64
    for _ in range(3):
        bits = rng.integers(0, 2, size=c.n)
        amp, fwd, bwd = closed.closed_amplitude(c, bits, chi=chi, n_sweeps=2, d1=d1, d2=d2)
        idx = int("".join(str(int(b)) for b in bits), 2)
        assert abs(amp - psi[idx]) < 1e-12 * max(1.0, abs(psi[idx])) + 1e-13


def test_closed_amplitude_truncated_bounds():
    """With truncation, the closed-mode amplitude is |<bwd|fwd>| <= 1 and its error against the
    exact amplitude is bounded by the infidelity of the two MPS (Cauchy-Schwarz with
    |phi_fwd - P psi_fwd|^2 <= 2 (1 - sqrt F))."""
    from oracle import closed
    c = circuits.plain_fp64_workload(1)
    psi = sv.run(c)
    rng = np.random.default_rng(9)
    for d1 in (3, 5):
        bits = rng.integers(0, 2, size=c.n)
        amp, fwd, bwd = closed.closed_amplitude(c, bits, chi=4, n_sweeps=2, d1=d1)
        idx = int("".join(str(int(b)) for b in bits), 2)
        exact_fwd = sv.run(c, depth=d1)
        # |<bwd|fwd> - <bwd_exact|fwd_exact>| <= |fwd - fwd_exact| + |bwd - bwd_exact|
        xb = sv.zero_state(c.n, bits)
        for layer in closed.dagger_layers(c.layers[d1:]):
            xb = sv.apply_layer(xb, c.n, layer)
        pf, pb = dmrg.to_statevector(fwd), dmrg.to_statevector(bwd)
        # align global phases (the MPS carry the phase of the exact states up to the fit)
        ef = np.linalg.norm(pf - exact_fwd * np.exp(1j * np.angle(np.vdot(exact_fwd, pf))))
        eb = np.linalg.norm(pb - xb * np.exp(1j * np.angle(np.vdot(xb, pb))))
        assert abs(abs(amp) - abs(psi[idx])) <= ef + eb + 1e-12
        assert abs(np.vdot(xb, exact_fwd) - psi[idx]) < 1e-12      # exact closed identity


def test_metropolis_acceptance_integral_is_ln2():
    """The paper's average acceptance for independent exponential weights,
    int_0^inf int_0^inf min(x/y, 1) e^-x e^-y dx dy, equals ln 2 = 0.693 (its "~70%")."""
    from scipy import integrate

    def inner(y):          # integral over x, split at the kink x = y of min(x/y, 1)
        a = integrate.quad(lambda x: x / y * math.exp(-x), 0.0, y, epsabs=1e-13)[0]
        return a + integrate.quad(lambda x: math.exp(-x), y, math.inf, epsabs=1e-13)[0]

    val = integrate.quad(lambda y: math.exp(-y) * inner(y), 0.0, math.inf, epsabs=1e-12, limit=200)[0]
    assert abs(val - math.log(2)) < 1e-8


def test_metropolis_chain_on_porter_thomas_state():
    """Oracle Metropolis chain over the exact amplitudes of a chaotic 12-qubit state: the visited
    bitstrings follow |Psi|^2 (collision probability sum p^2 = 2/2^n for Porter-Thomas), and at
    stationarity the mean acceptance is 1/2 (the current weight is size-biased, Gamma(2)); for a
    uniformly drawn current bitstring it is the paper's ln 2."""
    from oracle import closed
    c = circuits.random_circuit(circuits.Grid(12, 3), 14, seed=2)
    psi = sv.run(c)
    p = np.abs(psi) ** 2
    n = c.n
    amp = lambda bits: psi[int("".join(str(int(b)) for b in bits), 2)]
    props, us = circuits.metropolis_draws(n, 40000, seed=3)
    chain, acc = closed.metropolis(amp, props[0], props[1:], us[1:])
    rate = acc / (len(chain) - 1)
    assert abs(rate - 0.5) < 0.02, rate
    idx = np.array([int("".join(str(int(b)) for b in x), 2) for x in chain[2000:]])
    # E_chain[p(x)] = sum p^2: Porter-Thomas gives 2/2^n
    mean_p = p[idx].mean() * 2 ** n
    assert abs(mean_p - 2.0 * (p ** 2).sum() * 2 ** n / 2.0) < 0.1
    assert abs((p ** 2).sum() * 2 ** n - 2.0) < 0.15
    # uniformly drawn current states: mean of min(p'/p, 1) is ln 2
    rng = np.random.default_rng(4)
    a, b = rng.integers(0, 2 ** n, 200000), rng.integers(0, 2 ** n, 200000)
    assert abs(np.minimum(p[b] / p[a], 1.0).mean() - math.log(2)) < 0.02


# ------------------------------------------------------- Sycamore layout ---
def test_sycamore_layout_couplers():
    """Fig. 1 topology: n_c columns of n_b and n_b - 1 qubits (54 for n_b = 5, n_c = 12); each
    coupler class is a matching and the four classes split the nearest-neighbour couplers."""
    lay = circuits.SycamoreLayout(5, 12)
    assert lay.n == 54
    coords = lay.coords()
    assert len(set(coords)) == 54 and sorted(lay.site(c, y) for c, y in coords) == list(range(54))
    nn = set()
    for a, (c1, y1) in enumerate(coords):
        for b, (c2, y2) in enumerate(coords):
            if a < b and abs(c1 - c2) == 1 and abs(y1 - y2) == 1:
                nn.add((lay.site(c1, y1), lay.site(c2, y2)))
    seen = []
    for letter in "ABCD":
        pairs = lay.pattern_pairs(letter)
        flat = [q for p in pairs for q in p]
        assert len(flat) == len(set(flat))                         # a matching
        seen += pairs
    assert len(seen) == len(set(seen)) and set(seen) == {(min(p), max(p)) for p in nn}
    degree = np.bincount([q for p in seen for q in p], minlength=54)
    assert degree.max() == 4 and degree.min() >= 1


def test_sycamore_sequence_two_is_the_quarter_turn():
    """The letter map that takes Sequence I's string to Sequence II's (A->C, B->D, C->B,
    D->A) is the map of coupler classes under a quarter turn of the lattice."""
    mp = dict(zip(circuits.SEQUENCE_I, circuits.SEQUENCE_II))
    assert mp == {"A": "C", "B": "D", "C": "B", "D": "A"}

    def cls(p, q):
        (c1, y1), (c2, y2) = sorted([p, q])
        return {(0, 1): "A", (1, 1): "B", (0, -1): "C", (1, -1): "D"}[(c1 % 2, y2 - y1)]

    lay = circuits.SycamoreLayout(7, 10)
    pos = {lay.site(c, y): (c, y) for c, y in lay.coords()}
    turn = lambda c, y: (-y + 1, c + 1)
    for letter in "ABCD":
        for i, j in lay.pattern_pairs(letter):
            assert cls(pos[i], pos[j]) == letter
            assert cls(turn(*pos[i]), turn(*pos[j])) == mp[letter]


def test_fixed_fsim_has_four_schmidt_values():
    """fSim(1, pi/2) has four non-zero operator-Schmidt values (the hard regime of the
    paper's Sequences I and II), so every coupler multiplies the MPO bond by 4.  The
    spectrum of fSim(theta, phi) has the closed form
    sqrt(1 + cos^2 theta +- 2 cos theta cos(phi/2)), sin theta, sin theta."""
    for th, ph in ((circuits.FSIM_THETA, circuits.FSIM_PHI), (0.3, 2.5), (1.2, 0.4)):
        g = dmrg.split_two_qubit(0, 1, circuits.fsim(th, ph))
        got = np.sort(np.einsum("ast,ast->a", g.x.conj(), g.x).real)     # |X_a|^2 = sigma_a
        c = np.cos(th)
        want = np.sort([np.sqrt(1 + c * c + 2 * c * np.cos(ph / 2)), np.sqrt(1 + c * c - 2 * c * np.cos(ph / 2)),
                        np.sin(th), np.sin(th)])
        assert g.x.shape[0] == 4 and np.allclose(got, want, atol=1e-12)


@pytest.mark.parametrize("sequence", ["I", "II"])
def test_sycamore_circuit_exact_regime(sequence):
    """Sequences I and II on a 10-qubit layout (n_b = 3, n_c = 4): chi = 32 = 2^(n/2)
    reproduces the statevector, one and two layers per step."""
    c = circuits.sycamore_circuit(circuits.SycamoreLayout(3, 4), 8, seed=2, sequence=sequence)
    assert c.n == 10 and c.n_2q == sum(len(circuits.SycamoreLayout(3, 4).pattern_pairs(
        {"I": circuits.SEQUENCE_I, "II": circuits.SEQUENCE_II}[sequence][d % 8])) for d in range(8))
    psi = sv.run(c)
    st = dmrg.run_circuit(c, chi=32, n_sweeps=1)
    assert np.linalg.norm(dmrg.to_statevector(st) - psi) < 1e-12
    st2 = dmrg.product_state(c.n)
    for d in range(0, 8, 2):
        dmrg.apply_layers(st2, c.layers[d:d + 2], chi=32, n_sweeps=1)
    assert np.linalg.norm(dmrg.to_statevector(st2) - psi) < 1e-12


# ------------------------------------------------------- fidelity measures -
def test_fidelity_measures_special_cases():
    """F and F_B on states where they are fixed: F(psi, psi) = 1; F_B = 0 exactly against a
    uniform-modulus state; F_B of a product of independent blocks factorises as
    prod_b (1 + F_B,b) - 1; F <= 1 with equality only up to a phase."""
    from oracle import analysis
    rng = np.random.default_rng(4)
    a = chaotic.porter_thomas(8, rng); a /= np.linalg.norm(a)
    assert abs(analysis.fidelity(a, a) - 1.0) < 1e-13
    assert abs(analysis.fidelity(a, 1j * a) - 1.0) < 1e-13
    flat = np.exp(2j * np.pi * rng.random(256)) / 16.0
    assert abs(analysis.xeb_exact(flat, a)) < 1e-13 and abs(analysis.xeb_exact(a, flat)) < 1e-13
    b1 = chaotic.porter_thomas(4, rng); b1 /= np.linalg.norm(b1)
    b2 = chaotic.porter_thomas(4, rng); b2 /= np.linalg.norm(b2)
    c1 = chaotic.porter_thomas(4, rng); c1 /= np.linalg.norm(c1)
    c2 = chaotic.porter_thomas(4, rng); c2 /= np.linalg.norm(c2)
    whole = analysis.xeb_exact(np.kron(b1, b2), np.kron(c1, c2))
    parts = (1 + analysis.xeb_exact(b1, c1)) * (1 + analysis.xeb_exact(b2, c2)) - 1
    assert abs(whole - parts) < 1e-12
    assert analysis.fidelity(b1, c1) < 1.0


def test_xeb_estimator_converges_to_the_exact_value():
    """eq:FB-estim: samples drawn from Q give an unbiased estimate of eq:FB-sup."""
    from oracle import analysis
    rng = np.random.default_rng(6)
    p = chaotic.porter_thomas(10, rng); p /= np.linalg.norm(p)
    q = 0.8 * p + 0.6 * chaotic.porter_thomas(10, rng) / 32.0
    q /= np.linalg.norm(q)
    exact = analysis.xeb_exact(q, p)
    probs_q = np.abs(q) ** 2
    xs = rng.choice(1024, size=200000, p=probs_q / probs_q.sum())
    est = analysis.xeb_estimate(np.abs(p[xs]) ** 2, 10)
    sd = np.std(1024 * np.abs(p[xs]) ** 2) / math.sqrt(len(xs))
    assert abs(est - exact) < 4 * sd, (est, exact, sd)


# ------------------------------------------------------- qubit groupings ---
def test_constant_bond_profile_is_a_single_chi():
    """A per-bond cap equal to chi everywhere is the single-chi step."""
    c = circuits.plain_fp64_workload(1)
    a, b = dmrg.product_state(c.n), dmrg.product_state(c.n)
    for layer in c.layers:
        fa = dmrg.apply_layer(a, layer, 5, 2)
        fb = dmrg.apply_layers(b, [layer], [1] + [5] * (c.n - 1) + [1], 2)
        assert fa == fb
    assert np.array_equal(dmrg.to_statevector(a), dmrg.to_statevector(b))


@pytest.mark.parametrize("columns,trivial", [([2, 2], "AC"), ([1, 2, 1], "BD")])
def test_layers_inside_groups_are_trivial(columns, trivial):
    """Sec. V.C: with qubits grouped by columns, a layer whose couplers stay inside the groups
    has f_delta = 1 for any chi (here chi = 2 between groups) and reproduces the exact image of
    the layer; the other layers keep the bonds between groups at chi or below."""
    lay = circuits.SycamoreLayout(3, 4)
    sizes = circuits.sycamore_column_groups(lay, columns)
    prof = circuits.group_bond_profile(sizes, 2)
    cuts = np.cumsum(sizes)[:-1]
    c = circuits.sycamore_circuit(lay, 8, seed=3, sequence="I")
    st = dmrg.product_state(c.n)
    for d, layer in enumerate(c.layers):
        before = dmrg.to_statevector(st)
        f = dmrg.apply_layers(st, [layer], prof, 2)
        letter = circuits.SEQUENCE_I[d % 8]
        if letter in trivial:
            target = sv.apply_layer(before, c.n, layer)
            assert abs(f - 1.0) < 1e-12, (d, letter, f)
            assert abs(abs(np.vdot(dmrg.to_statevector(st), target)) - 1.0) < 1e-12
        assert all(st.bond_dims()[k] <= 2 for k in cuts)
    assert min(st.layer_f) < 0.99        # the crossing layers do truncate at chi = 2


def _internal_letters(layout, groups_of_site):
    """Coupler classes whose couplers all stay inside one group."""
    out = ""
    for letter in "ABCD":
        if all(groups_of_site[i] == groups_of_site[j] for i, j in layout.pattern_pairs(letter)):
            out += letter
    return out


def test_groupings_make_the_paper_s_trivial_layers():
    """The layers the paper calls trivial for each grouping (Sec. V.C) are exactly the coupler
    classes that stay inside its groups under this reading of classes A-D: B and D for V1
    (columns 5, 2, 5 of the 54-qubit processor: 23, 9 and 22 qubits), A and D for H1, B and C
    for H2."""
    lay = circuits.SycamoreLayout(5, 12)
    sizes = circuits.sycamore_column_groups(lay, [5, 2, 5])
    assert sizes == [23, 9, 22]
    gid = np.repeat(np.arange(3), sizes)
    assert _internal_letters(lay, gid) == "BD"
    for offset, want in ((0, "AD"), (1, "BC")):
        order, hs = circuits.sycamore_row_groups(lay, offset)
        gid = np.empty(lay.n, dtype=int)
        gid[np.array(order)] = np.repeat(np.arange(len(hs)), hs)
        assert _internal_letters(lay, gid) == want, (offset, _internal_letters(lay, gid))


def test_row_grouping_layers_are_trivial_after_relabelling():
    """H1 on the 10-qubit layout: the chain is relabelled so that each row pair is contiguous;
    the A and D layers are then exact at chi = 2 between groups."""
    lay = circuits.SycamoreLayout(3, 4)
    order, sizes = circuits.sycamore_row_groups(lay, 0)
    c = circuits.relabel_circuit(circuits.sycamore_circuit(lay, 8, seed=3, sequence="I"), order)
    prof = circuits.group_bond_profile(sizes, 2)
    st = dmrg.product_state(c.n)
    for d, layer in enumerate(c.layers):
        before = dmrg.to_statevector(st)
        f = dmrg.apply_layers(st, [layer], prof, 2)
        if circuits.SEQUENCE_I[d % 8] in "AD":
            assert abs(f - 1.0) < 1e-12
            target = sv.apply_layer(before, c.n, layer)
            assert abs(abs(np.vdot(dmrg.to_statevector(st), target)) - 1.0) < 1e-12
    assert min(st.layer_f) < 0.99


@pytest.mark.parametrize("direction,trivial", [("up", "AB"), ("down", "CD")])
def test_diagonal_groupings_trivial_layers(direction, trivial):
    """D groupings (one group per diagonal line of the layout): exactly the two coupler classes
    that run along the lines stay inside the groups (checked on the 54-qubit processor), and on
    the 10-qubit layout, relabelled so that each line is contiguous, those layers are exact at
    chi = 2 between groups while the others truncate."""
    big = circuits.SycamoreLayout(5, 12)
    order, sizes = circuits.sycamore_diagonal_groups(big, direction)
    assert sorted(order) == list(range(big.n)) and sum(sizes) == big.n
    gid = np.empty(big.n, dtype=int)
    gid[np.array(order)] = np.repeat(np.arange(len(sizes)), sizes)
    assert _internal_letters(big, gid) == trivial
    lay = circuits.SycamoreLayout(3, 4)
    order, sizes = circuits.sycamore_diagonal_groups(lay, direction)
    c = circuits.relabel_circuit(circuits.sycamore_circuit(lay, 8, seed=3, sequence="I"), order)
    prof = circuits.group_bond_profile(sizes, 2)
    cuts = np.cumsum(sizes)[:-1]
    st = dmrg.product_state(c.n)
    for d, layer in enumerate(c.layers):
        before = dmrg.to_statevector(st)
        f = dmrg.apply_layers(st, [layer], prof, 2)
        if circuits.SEQUENCE_I[d % 8] in trivial:
            assert abs(f - 1.0) < 1e-12, (d, f)
            target = sv.apply_layer(before, c.n, layer)
            assert abs(abs(np.vdot(dmrg.to_statevector(st), target)) - 1.0) < 1e-12
        assert all(st.bond_dims()[k] <= 2 for k in cuts)
    assert min(st.layer_f) < 0.99


# ------------------------------------------- conditioning of a truncation --
@pytest.mark.parametrize("gap", [1e-1, 1e-3, 1e-5])
def test_truncation_sensitivity_bounds_the_state_change(gap):
    """2 u kappa (truncated_svd_gap) bounds, to first order, how far a relative perturbation u
    of the Gram matrices moves the normalised truncated state (Davis-Kahan on the left and on
    the right kept subspace); the gap is the one constructed, and the bound is attained within
    a modest factor by the worst perturbation (one that couples the last kept and the first
    discarded singular vectors)."""
    rng = np.random.default_rng(11)
    n, k = 40, 10

    def haar(m):
        q, r = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
        return q * (np.diag(r) / np.abs(np.diag(r)))

    s = np.sort(rng.uniform(0.2, 1.0, n))[::-1]
    s[k:] *= s[k - 1] / (s[k] * (1.0 + gap))          # S_k / S_{k+1} = 1 + gap exactly
    s[k:] = np.minimum(s[k:], s[k - 1] / (1.0 + gap))
    u_, v_ = haar(n), haar(n)
    m = (u_ * s) @ v_.conj().T
    _, ks, _, total, (g, kappa) = dmrg.truncated_svd_gap(m, k)
    assert len(ks) == k and abs(g - gap) < 1e-9 * max(1.0, gap)

    def state(mat):
        uu, ss, vv, _ = dmrg.truncated_svd(mat, k)
        t = (uu * ss) @ vv
        return t / np.linalg.norm(t)

    ref = state(m)
    eps = 1e-9
    worst_ratio = 0.0
    for trial in range(6):
        if trial == 0:
            # worst case: rotate the k-th kept into the first discarded left singular vector
            e = np.outer(u_[:, k], u_[:, k - 1].conj()) + np.outer(u_[:, k - 1], u_[:, k].conj())
            e = e @ m
        else:
            e = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        e *= eps * np.linalg.norm(m, 2) / np.linalg.norm(e, 2)     # relative perturbation of m (2x in m m^H)
        phi = state(m + e)
        ph = np.vdot(ref, phi)
        d = np.linalg.norm(phi * np.conj(ph) / abs(ph) - ref)
        worst_ratio = max(worst_ratio, d / (2 * eps * kappa))
    print("gap %.0e kappa %.3g worst ratio %.3f" % (gap, kappa, worst_ratio))
    assert worst_ratio <= 2.0          # first-order bound (2 eps = relative size of the Gram change)
    assert worst_ratio >= 0.1          # and not vacuous: the worst perturbation comes close to it


# --------------------------------------------- groupings (r_tau qubits per tensor) ---
# Sec. IV.A: a tensor may hold r_tau consecutive qubits (physical dimension 2^r_tau); the
# compression step is unchanged on such sites.

def _grouped_run(c, sizes, chi, n_sweeps, update="two-site"):
    st = dmrg.group_state(dmrg.product_state(c.n), sizes)
    fs = [dmrg.apply_layers(st, [layer], chi, n_sweeps, update, sizes=sizes) for layer in c.layers]
    return st, np.array(fs)


@pytest.mark.parametrize("update", ["two-site", "single-site"])
def test_grouped_sites_of_one_qubit_are_the_plain_oracle(update):
    """r_tau = 1 everywhere: the same arithmetic as the plain oracle, bit for bit."""
    c = circuits.random_circuit(circuits.grid_from_shape(3, 4), 6, seed=4)
    st, fs = _grouped_run(c, [1] * c.n, 6, 2, update)
    ref = dmrg.product_state(c.n)
    fr = np.array([dmrg.apply_layer(ref, layer, 6, 2, update=update) for layer in c.layers])
    assert np.array_equal(fs, fr)
    assert np.array_equal(dmrg.to_statevector(st), dmrg.to_statevector(ref))


@pytest.mark.parametrize("sizes", [[3, 3, 3, 3], [2] * 6, [4, 4, 4], [1, 3, 4, 2, 2]])
def test_grouped_sites_exact_regime_match_the_statevector(sizes):
    """chi at least the largest Schmidt rank of a cut between groups: the grouped simulation is
    exact (every f_delta = 1, amplitudes equal to the brute-force state) whatever the grouping."""
    c = circuits.random_circuit(circuits.grid_from_shape(3, 4), 6, seed=5)
    st, fs = _grouped_run(c, sizes, 64, 2)
    assert np.all(np.abs(fs - 1.0) < 1e-12)
    want = sv.run(c)
    got = dmrg.to_statevector(st)
    assert np.linalg.norm(got - want) < 1e-10
    assert [a.shape[1] for a in st.tensors] == [2 ** r for r in sizes]


def test_one_group_holds_the_whole_state():
    """One tensor of all n qubits: the MPS is the state vector itself, the zip-up applies the layer
    exactly and no truncation happens, even at chi = 1 (a chain of one site has no inner bond)."""
    c = circuits.random_circuit(circuits.grid_from_shape(2, 4), 5, seed=6)
    st, fs = _grouped_run(c, [c.n], 1, 2)
    assert np.all(np.abs(fs - 1.0) < 1e-12)
    assert np.linalg.norm(dmrg.to_statevector(st) - sv.run(c)) < 1e-10


@pytest.mark.parametrize("update", ["two-site", "single-site"])
def test_grouped_sites_truncated_invariants(update):
    """Truncated (chi = 4 between groups of 2): every step keeps f <= the local tensor's weight,
    0 < f_delta <= 1, the state stays normalised, F~ is the product of the f_delta, the bonds
    between groups respect chi, and the fidelity with the brute-force state is at most 1."""
    c = circuits.random_circuit(circuits.grid_from_shape(3, 4), 8, seed=7)
    sizes = [2] * 6
    st, fs = _grouped_run(c, sizes, 4, 2, update)
    assert np.all(fs <= 1.0 + 1e-12) and np.all(fs > 0.0)
    for rec in st.step_log:
        assert rec.f <= rec.sum_s2 * (1.0 + 1e-12)
    v = dmrg.to_statevector(st)
    assert abs(np.vdot(v, v).real - 1.0) < 1e-10
    _, log_f, _ = dmrg.fidelity(st)
    assert abs(log_f - np.sum(np.log(fs))) < 1e-12
    assert all(a.shape[0] <= 4 and a.shape[2] <= 4 for a in st.tensors)
    assert abs(np.vdot(sv.run(c), v)) ** 2 <= 1.0 + 1e-12
