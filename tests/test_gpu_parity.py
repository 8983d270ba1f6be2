"""GPU parity: the HIP library against the FP64 oracle, through the C ABI.

Tolerances:
  * GEMM kernel alone: |C - C_ref| <= 4 eps K max|A| max|B| (eps of the
    working precision; operands are rounded to it first);
  * FP64 path: per-layer f_delta within 1e-10 relative, amplitudes within
    1e-9 relative L2, kept bond dimensions identical;
  * FP32 and split paths: per-layer f_delta within 1e-4 relative; amplitudes
    within 1e-5 (FP32) or 1e-3 (split) relative L2 of the oracle, unless the
    oracle's own truncations are ill-conditioned: then the bound is the
    first-order one of tests/parity_bounds.py (10 u times the summed
    sensitivity kappa of the layers, from the oracle's singular values), and
    the worst gap and the MPS-MPS overlap error are reported and the overlap
    error asserted beside it.
"""
import math

import numpy as np
import pytest

from paper_2207_05612_amd import circuits, mps
from oracle import dmrg
from oracle import statevector as sv

import parity_bounds as pb

pytestmark = pytest.mark.gpu

FP64, FP32, BF16X2, BF16X3 = mps.MPS_FP64, mps.MPS_FP32, mps.MPS_BF16X2, mps.MPS_BF16X3
F_TOL = {FP64: 1e-10, **pb.F_TARGET}
AMP_TOL = pb.AMP_TARGET
OVERLAP_FLOOR = pb.OVERLAP_FLOOR
EPS = {FP64: 2.2e-16, FP32: 1.2e-7, BF16X3: 2.4e-7, BF16X2: 3.1e-5}


def _rc(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


GEMM_SHAPES = [(1, 1, 1), (5, 7, 3), (37, 45, 29), (64, 64, 8), (128, 128, 16), (130, 257, 70), (300, 64, 513),
               (128, 128, 4096), (70, 90, 9001), (40, 300, 20000)]    # the last three take the split-K path


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("opa,opb", [(0, 0), (0, 1), (0, 2), (2, 0), (2, 1), (2, 2)])
def test_cgemm_kernel_matches_numpy(prec, opa, opb):
    rng = np.random.default_rng(100 + 10 * opa + opb)
    for M, N, K in GEMM_SHAPES:
        a = _rc(rng, M, K) if opa == 0 else _rc(rng, K, M)
        b = _rc(rng, K, N) if opb == 0 else _rc(rng, N, K)
        A = a if opa == 0 else a.conj().T
        B = b if opb == 0 else (b.T if opb == 1 else b.conj().T)
        want = A @ B
        got = mps.selftest_cgemm(prec, opa, opb, a, b)
        bound = 4 * EPS[prec] * K * np.abs(A).max() * np.abs(B).max()
        assert np.abs(got - want).max() <= bound, (M, N, K)


@pytest.mark.parametrize("prec", [BF16X3, BF16X2])
def test_split_bf16_kernel_matches_numpy(prec):
    """The split-precision kernels (C = A B^T, both k-contiguous): three terms at FP32-level
    accuracy, two terms at about 2^-16 relative per product."""
    rng = np.random.default_rng(77)
    for M, N, K in GEMM_SHAPES + [(256, 130, 40), (33, 300, 257)]:
        a, b = _rc(rng, M, K), _rc(rng, N, K)
        want = a @ b.T
        got = mps.selftest_cgemm(prec, 0, 1, a, b)
        bound = 4 * EPS[prec] * K * np.abs(a).max() * np.abs(b).max()
        assert np.abs(got - want).max() <= bound, (M, N, K)
        if prec == BF16X2 and K >= 64:
            # more accurate than plain BF16 (relative 2^-8): the lo terms are used
            rel = np.linalg.norm(got - want) / np.linalg.norm(want)
            assert rel < 1e-4, (M, N, K, rel)


@pytest.mark.parametrize("prec", [BF16X3, BF16X2])
def test_split_planes_equal_staged_split(prec):
    """The compression step splits each operand once into BF16 planes (mps_kernel_selftest_cgemm
    runs that path); the allocation-free entry point splits every k tile while staging it.  Same
    terms, k tiles and MFMA order: the products must agree bit for bit, on ragged shapes (rows
    past the tile, k past a multiple of 16), several tiles and the split-K path."""
    import torch
    rng = np.random.default_rng(31)
    shapes = GEMM_SHAPES + [(256, 130, 40), (33, 300, 257), (257, 129, 17), (513, 385, 1000), (600, 260, 12000)]
    for M, N, K in shapes:
        a = _rc(rng, M, K).astype(np.complex64).astype(np.complex128)
        b = _rc(rng, N, K).astype(np.complex64).astype(np.complex128)
        ref = mps.selftest_cgemm(prec, 0, 1, a, b)
        ar = torch.tensor(np.ascontiguousarray(a.real), dtype=torch.float32, device="cuda")
        ai = torch.tensor(np.ascontiguousarray(a.imag), dtype=torch.float32, device="cuda")
        br = torch.tensor(np.ascontiguousarray(b.real), dtype=torch.float32, device="cuda")
        bi = torch.tensor(np.ascontiguousarray(b.imag), dtype=torch.float32, device="cuda")
        cr = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
        ci = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        mps.cgemm_noalloc(prec, 0, 1, M, N, K, (ar.data_ptr(), ai.data_ptr()), K, (br.data_ptr(), bi.data_ptr()), K,
                          (cr.data_ptr(), ci.data_ptr()), N)
        torch.cuda.synchronize()
        got = cr.double().cpu().numpy() + 1j * ci.double().cpu().numpy()
        assert np.array_equal(got, ref), (M, N, K, np.abs(got - ref).max())


@pytest.mark.parametrize("prec", [BF16X3, BF16X2])
def test_split_planes_of_transposed_operand(prec):
    """opb = 0 splits b^T into planes straight from b (K x N), the environment update's path: the
    same planes as splitting the explicit transpose, so the same bits as opb = 1 on b^T."""
    rng = np.random.default_rng(47)
    for M, N, K in [(5, 7, 3), (130, 257, 70), (300, 64, 513), (70, 90, 9001), (257, 129, 17)]:
        a = _rc(rng, M, K).astype(np.complex64).astype(np.complex128)
        b = _rc(rng, K, N).astype(np.complex64).astype(np.complex128)
        got = mps.selftest_cgemm(prec, 0, 0, a, b)
        ref = mps.selftest_cgemm(prec, 0, 1, a, np.ascontiguousarray(b.T))
        assert np.array_equal(got, ref), (M, N, K, np.abs(got - ref).max())


def run_gpu(circuit, chi, n_sweeps, prec, depth=None, bits=None):
    st = mps.MPS(circuit.n, bits, max_chi=max(chi, 1), precision=prec)
    layers = circuit.layers if depth is None else circuit.layers[:depth]
    fs = [st.apply_layer_dmrg(layer, chi, n_sweeps) for layer in layers]
    return st, np.array(fs)


rel_l2 = pb.rel_l2


def check_amplitudes(prec, err, st, ora, n_sweeps, label):
    """Assert the amplitude error against the bound of parity_bounds and the overlap error
    against its square; report both with the worst truncation gap."""
    sizes = pb.two_site_layer_sizes(ora.n, n_sweeps, ora.n_layers)
    ksum = pb.sum_layer_kappa(ora.step_log, sizes)
    bound = pb.amp_bound(prec, ksum)
    ovl = pb.overlap_error(st, ora)
    print("%s prec=%d amplitude rel-L2 %.2e (bound %.2e; target %.0e) overlap error %.2e worst gap %.2e "
          "sum kappa %.3g" % (label, prec, err, bound, AMP_TOL[prec], ovl, pb.worst_gap(ora.step_log), ksum))
    assert err < bound
    assert ovl <= max(bound ** 2, OVERLAP_FLOOR)
    return bound


@pytest.mark.parametrize("prec", [FP64, FP32, BF16X2, BF16X3])
def test_exact_regime_plain_workload(prec):
    """12 qubits, 3x4 grid, depth 8, chi = 64 (exact), 2 sweeps, seed 0."""
    c = circuits.plain_fp64_workload(0)
    st, fs = run_gpu(c, 64, 2, prec)
    psi = sv.run(c)
    assert rel_l2(st.statevector(), psi) < AMP_TOL[prec]
    fid = st.fidelity()
    assert abs(fid["F_tilde"] - 1.0) < F_TOL[prec] * 10
    assert fid["n_2q"] == c.n_2q == 34
    ora = dmrg.run_circuit(c, chi=64, n_sweeps=2)
    assert st.bond_dims() == ora.bond_dims()
    # the zip-up truncates its intermediate bonds (chi w) to chi even here; every cut is resolved
    sep = st.cut_separations()
    assert sep.shape == (len(c.layers),) and np.all(sep > 0)


@pytest.mark.parametrize("prec", [FP64, FP32, BF16X2, BF16X3])
@pytest.mark.parametrize("chi", [4, 8, 16])
def test_truncated_parity_plain_workload(prec, chi):
    c = circuits.plain_fp64_workload(1)
    st, fs = run_gpu(c, chi, 2, prec)
    ora = dmrg.run_circuit(c, chi=chi, n_sweeps=2)
    of = np.array(ora.layer_f)
    assert np.max(np.abs(fs - of) / of) < F_TOL[prec]
    err = rel_l2(st.statevector(), dmrg.to_statevector(ora))
    check_amplitudes(prec, err, st, ora, 2, "12 qubits chi=%d" % chi)
    f_log, s2_log, k_log = st.step_log()
    assert len(f_log) == len(ora.step_log)
    ofl = np.array([r.f for r in ora.step_log])
    assert np.max(np.abs(f_log - ofl) / ofl) < F_TOL[prec]
    if prec == FP64:
        assert list(k_log) == [r.chi_kept for r in ora.step_log]
        assert st.bond_dims() == ora.bond_dims()
    gf = st.fidelity()
    assert abs(gf["log_F_tilde"] - ora.log_f) < F_TOL[prec] * 10 * len(c.layers)
    sep = st.cut_separations()          # truncation at chi happens: some separation is finite
    assert sep.shape == (len(c.layers),) and np.all(sep >= 0) and np.isfinite(sep).any()


@pytest.mark.parametrize("prec", [FP64, FP32, BF16X2, BF16X3])
def test_grid_20_qubits_truncated(prec):
    """20 qubits on a 4x5 grid (snake width 4), Haar gates, depth 10, chi 16."""
    c = circuits.random_circuit(circuits.grid_from_shape(5, 4), 10, seed=3)
    st, fs = run_gpu(c, 16, 2, prec)
    ora = dmrg.run_circuit(c, chi=16, n_sweeps=2)
    of = np.array(ora.layer_f)
    assert np.max(np.abs(fs - of) / of) < F_TOL[prec]
    rng = np.random.default_rng(0)
    bits = rng.integers(0, 2, size=(64, c.n)).astype(np.uint8)
    amp_gpu = st.amplitudes(bits)
    amp_ora = np.array([dmrg.amplitude(ora, b) for b in bits])
    err = rel_l2(amp_gpu, amp_ora)
    check_amplitudes(prec, err, st, ora, 2, "20 qubits chi=16")


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_zero_sweeps_and_initial_bits(prec):
    c = circuits.random_brickwork(9, 6, seed=8)
    bits = [1, 0, 0, 1, 1, 0, 1, 0, 1]
    st, fs = run_gpu(c, 4, 0, prec, bits=bits)
    ora = dmrg.run_circuit(c, chi=4, n_sweeps=0, bits=bits)
    assert np.max(np.abs(fs - np.array(ora.layer_f)) / np.array(ora.layer_f)) < F_TOL[prec]
    assert rel_l2(st.statevector(), dmrg.to_statevector(ora)) < AMP_TOL[prec]


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_odd_sweeps_and_reversed_gates(prec):
    """Three sweeps per layer and two-qubit gates given with q0 > q1."""
    c = circuits.random_brickwork(8, 6, seed=9)
    layers = [[(q1, q0, u.reshape(2, 2, 2, 2).transpose(1, 0, 3, 2).reshape(4, 4)) if q1 >= 0 else (q0, q1, u)
               for (q0, q1, u) in layer] for layer in c.layers]
    rc = circuits.Circuit(n=c.n, layers=layers)
    st, fs = run_gpu(rc, 4, 3, prec)
    ora = dmrg.run_circuit(c, chi=4, n_sweeps=3)
    assert np.max(np.abs(fs - np.array(ora.layer_f)) / np.array(ora.layer_f)) < F_TOL[prec]
    assert rel_l2(st.statevector(), dmrg.to_statevector(ora)) < AMP_TOL[prec]


def test_degenerate_sizes():
    # one site: only one-qubit gates; f = 1
    st = mps.MPS(1, None, max_chi=4, precision=FP64)
    f = st.apply_layer_dmrg([(0, -1, circuits.SQRT_X)], 4, 2)
    assert abs(f - 1.0) < 1e-14
    assert np.allclose(st.statevector(), circuits.SQRT_X[:, 0], atol=1e-14)
    # an empty layer is the identity
    st2 = mps.MPS(5, [1, 0, 1, 1, 0], max_chi=4, precision=FP64)
    assert abs(st2.apply_layer_dmrg([], 4, 2) - 1.0) < 1e-14
    psi = sv.zero_state(5, [1, 0, 1, 1, 0])
    assert rel_l2(st2.statevector(), psi) < 1e-14
    # two sites, one Haar gate, chi = 1 truncates to the largest Schmidt value
    u = circuits.haar_unitary_from_normals(np.random.default_rng(4).standard_normal(32))
    st3 = mps.MPS(2, None, max_chi=2, precision=FP64)
    f3 = st3.apply_layer_dmrg([(0, 1, u)], 1, 2)
    s = np.linalg.svd(u[:, 0].reshape(2, 2), compute_uv=False)
    assert abs(f3 - s[0] ** 2) < 1e-12


@pytest.mark.parametrize("prec", [FP64, FP32, BF16X3])
def test_sampler_matches_oracle_bitstrings(prec):
    c = circuits.random_brickwork(10, 6, seed=12)
    st, _ = run_gpu(c, 8, 2, prec)
    ora = dmrg.run_circuit(c, chi=8, n_sweeps=2)
    n_s = 400
    got = st.sample(n_s, seed=2024)
    want = dmrg.sample(ora, n_s, seed=2024)
    same = np.mean(np.all(got == want, axis=1))
    assert same >= (0.995 if prec == FP64 else 0.98)


def test_sampler_born_rule_gpu():
    c = circuits.random_brickwork(6, 6, seed=21)
    st, _ = run_gpu(c, 4, 1, FP32)
    probs = np.abs(st.statevector()) ** 2
    ns = 200000
    bits = st.sample(ns, seed=5)
    idx = bits.astype(np.int64) @ (1 << np.arange(5, -1, -1))
    counts = np.bincount(idx, minlength=64)
    expect = probs * ns
    mask = expect > 5
    chi2 = float(np.sum((counts[mask] - expect[mask]) ** 2 / expect[mask]))
    dof = int(mask.sum()) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_expect_zz_matches_oracle():
    c = circuits.random_brickwork(8, 5, seed=13)
    st, _ = run_gpu(c, 8, 2, FP64)
    ora = dmrg.run_circuit(c, chi=8, n_sweeps=2)
    for i, j in [(0, 1), (2, 5), (3, 3), (7, 0)]:
        assert abs(st.expect_zz(i, j) - dmrg.expectation_zz(ora, min(i, j), max(i, j))) < 1e-10


def test_argument_errors_leave_state_usable():
    c = circuits.random_brickwork(6, 3, seed=1)
    st = mps.MPS(6, None, max_chi=8, precision=FP64)
    with pytest.raises(mps.MpsError) as e:
        st.apply_layer_dmrg(c.layers[0], 16, 2)             # chi > max_chi
    assert e.value.code == mps.MPS_ERR_ARG
    with pytest.raises(mps.MpsError) as e:
        st.apply_layer_dmrg([(0, 1, np.eye(4)), (1, 2, np.eye(4))], 4, 2)   # overlapping
    assert e.value.code == mps.MPS_ERR_ARG
    with pytest.raises(mps.MpsError) as e:
        st.apply_layer_dmrg([(0, 9, np.eye(4))], 4, 2)        # site out of range
    assert e.value.code == mps.MPS_ERR_ARG
    bad = circuits.pack_layer([(0, 1, np.eye(4))])
    bad[0]["m"][0] = np.nan
    with pytest.raises(mps.MpsError) as e:
        st.apply_layer_dmrg(bad, 4, 2)
    assert e.value.code == mps.MPS_ERR_ARG
    for layer in c.layers:
        st.apply_layer_dmrg(layer, 8, 2)
    ora = dmrg.run_circuit(c, chi=8, n_sweeps=2)
    assert rel_l2(st.statevector(), dmrg.to_statevector(ora)) < 1e-9


@pytest.mark.parametrize("prec", [FP64, BF16X3])
def test_torch_caching_allocator_parity(prec):
    """A state whose device memory comes from PyTorch's caching allocator (the ABI's allocator
    callbacks) gives the same layers as the oracle; its blocks are PyTorch's while it lives and
    are all returned when it is destroyed."""
    import torch
    c = circuits.plain_fp64_workload(1)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    st = mps.MPS(c.n, None, max_chi=8, precision=prec, torch_allocator=True)
    fs = np.array([st.apply_layer_dmrg(layer, 8, 2) for layer in c.layers])
    assert torch.cuda.memory_allocated() > base          # the tensors of the state live in torch's pool
    ora = dmrg.run_circuit(c, chi=8, n_sweeps=2)
    of = np.array(ora.layer_f)
    assert np.max(np.abs(fs - of) / of) < F_TOL[prec]
    err = rel_l2(st.statevector(), dmrg.to_statevector(ora))
    check_amplitudes(prec, err, st, ora, 2, "torch allocator")
    # the same layers on a state with the library's own pool: identical kernels, identical results
    ref, fr = run_gpu(c, 8, 2, prec)
    assert np.array_equal(fs, fr)
    st.close()
    ref.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


@pytest.mark.parametrize("prec", [FP64, BF16X3])
def test_right_block_on_second_stream_same_result(prec, monkeypatch):
    """MPS_OVERLAP=1 builds the next pair's right block on the state's second stream while the
    current pair is truncated: the same kernels on the same data, so the same bits as the default
    schedule (one stream), on a truncated 20-qubit case with saturated bonds."""
    c = circuits.random_circuit(circuits.grid_from_shape(5, 4), 8, seed=5)
    ref, fr = run_gpu(c, 16, 2, prec)
    monkeypatch.setenv("MPS_OVERLAP", "1")
    st, fs = run_gpu(c, 16, 2, prec)
    assert np.array_equal(fs, fr)
    assert np.array_equal(st.statevector(), ref.statevector())
    st.close()
    ref.close()


def test_eigensolver_counts():
    """Every truncation is counted once by the path that diagonalised it; orders up to 128 take
    the single-workgroup reduction, larger ones the persistent one; no fallback happens."""
    c = circuits.random_circuit(circuits.grid_from_shape(5, 4), 10, seed=3)
    st, fs = run_gpu(c, 128, 1, FP64)
    cnt = st.counters()
    n_trunc = len(c.layers) * (2 * (c.n - 1))          # zip-up (n - 1) + one sweep (n - 1) per layer
    print(cnt, st.bond_dims())
    assert sum(cnt.values()) == n_trunc
    assert cnt["fallback_library"] == 0 and cnt["single_workgroup"] > 0
    if max(st.bond_dims()) > 64:                        # a Gram matrix of order > 128 was diagonalised
        assert cnt["persistent"] > 0
