"""The allocation-free GEMM entry point (mps_cgemm_noalloc) against the allocating one.

mps_cgemm_noalloc runs the products of mps_kernel_selftest_cgemm on device
operands with its split-K partial sums in the library's static scratch array
(for the split precisions it splits each k tile while staging it, where the
selftest splits the operands once beforehand: same terms, same bits).  Two
calls in a row (the second smaller, so the scratch keeps the first call's
partial sums) must each equal mps_kernel_selftest_cgemm on the same operands
bit for bit (same split of K), and so meet the same bound against NumPy as
the kernel tests.  A product whose partial sums exceed the scratch
array is refused before any work.
"""
import numpy as np
import pytest

from paper_2207_05612_amd import mps

pytestmark = pytest.mark.gpu

FP64, FP32, BF16X2, BF16X3 = mps.MPS_FP64, mps.MPS_FP32, mps.MPS_BF16X2, mps.MPS_BF16X3
EPS = {FP64: 2.2e-16, FP32: 1.2e-7, BF16X3: 2.4e-7, BF16X2: 3.1e-5}


def _rc(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _planar(torch, x, dtype):
    re = torch.tensor(np.ascontiguousarray(x.real), dtype=dtype, device="cuda")
    im = torch.tensor(np.ascontiguousarray(x.imag), dtype=dtype, device="cuda")
    return re, im


def _noalloc(torch, prec, opa, opb, a, b):
    dtype = torch.float64 if prec == FP64 else torch.float32
    M, K = (a.shape[0], a.shape[1]) if opa == 0 else (a.shape[1], a.shape[0])
    N = b.shape[1] if opb == 0 else b.shape[0]
    ar, ai = _planar(torch, a, dtype)
    br, bi = _planar(torch, b, dtype)
    cr = torch.full((M, N), float("nan"), dtype=dtype, device="cuda")
    ci = torch.full((M, N), float("nan"), dtype=dtype, device="cuda")
    torch.cuda.synchronize()
    mps.cgemm_noalloc(prec, opa, opb, M, N, K, (ar.data_ptr(), ai.data_ptr()), a.shape[1],
                      (br.data_ptr(), bi.data_ptr()), b.shape[1], (cr.data_ptr(), ci.data_ptr()), N)
    torch.cuda.synchronize()
    return cr.double().cpu().numpy() + 1j * ci.double().cpu().numpy()


@pytest.mark.parametrize("prec,opa,opb", [(FP32, 0, 0), (FP32, 2, 1), (FP64, 0, 2), (BF16X3, 0, 1), (BF16X2, 0, 1)])
def test_noalloc_equals_allocating_entry_point(prec, opa, opb):
    import torch
    rng = np.random.default_rng(5)
    # first a long contraction (split-K through the scratch array), then a smaller one
    for M, N, K in ((300, 200, 20000), (70, 90, 9001)):
        a = _rc(rng, M, K) if opa == 0 else _rc(rng, K, M)
        b = _rc(rng, K, N) if opb == 0 else _rc(rng, N, K)
        if prec in (FP32, BF16X2, BF16X3):
            a = a.astype(np.complex64).astype(np.complex128)
            b = b.astype(np.complex64).astype(np.complex128)
        got = _noalloc(torch, prec, opa, opb, a, b)
        ref = mps.selftest_cgemm(prec, opa, opb, a, b)
        assert np.array_equal(got, ref), (M, N, K, np.abs(got - ref).max())
        A = a if opa == 0 else a.conj().T
        B = b if opb == 0 else (b.T if opb == 1 else b.conj().T)
        bound = 4 * EPS[prec] * K * np.abs(A).max() * np.abs(B).max()
        assert np.abs(got - A @ B).max() <= bound


def test_noalloc_refuses_products_beyond_the_scratch():
    import torch
    t = torch.zeros(16, dtype=torch.float32, device="cuda")
    p = (t.data_ptr(), t.data_ptr())
    # M N = 2^24 outputs with K split in many chunks: far beyond 64 MiB of partial sums
    with pytest.raises(mps.MpsError) as e:
        mps.cgemm_noalloc(FP32, 0, 0, 4096, 4096, 65536, p, 65536, p, 4096, p, 4096)
    assert e.value.code == mps.MPS_ERR_ARG and "scratch" in str(e.value)
    with pytest.raises(mps.MpsError) as e:
        mps.cgemm_noalloc(BF16X3, 0, 0, 4, 4, 4, p, 4, p, 4, p, 4)
    assert e.value.code == mps.MPS_ERR_ARG
