"""The library's tridiagonal divide and conquer, through the C ABI.

The truncation of a two-site step (Sec. VI.A) needs every eigenvalue of the
Gram matrix (the discarded weight) and the eigenvectors of the kept ones; after
the tridiagonal reduction this solver computes them.  Checked on seeded
tridiagonal matrices against LAPACK (scipy.linalg.eigh_tridiagonal, FP64):
  * eigenvalues within 1e-13 ||T|| (backward-stable: a few n eps ||T||),
  * residual max |T Z - Z diag(w)| / ||T|| and max |Z^T Z - I| below 1e-13,
and against closed forms: the (-1, 2, -1) matrix of order n has the
eigenvalues 2 - 2 cos(k pi / (n + 1)) with the sine vectors, a diagonal
matrix its own entries with unit vectors.
The inputs exercise every branch of the merges: deflation of small update
components (graded and rank-deficient Gram spectra, exactly zero off-diagonal
entries), deflation by rotation (clusters, repeated entries, Wilkinson's W+),
ragged trees (n not a power of two) and the largest order (2048).
"""
import numpy as np
import pytest
from scipy.linalg import eigh_tridiagonal, hessenberg

from paper_2207_05612_amd import mps

pytestmark = pytest.mark.gpu

TOL = 1e-13


def tridiagonal_of(spectrum, seed):
    """Householder tridiagonal form of Q diag(spectrum) Q^T (Q random orthogonal)."""
    n = len(spectrum)
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    h = hessenberg((q * spectrum) @ q.T)
    return np.diag(h).copy(), np.diag(h, 1).copy()


def case(kind, n, seed=0):
    rng = np.random.default_rng(seed)
    if kind == "random":
        return rng.standard_normal(n), rng.standard_normal(n - 1)
    if kind == "gram_graded":                 # PSD spectrum over 30 decades, as in a truncated Gram matrix
        return tridiagonal_of(10.0 ** -np.linspace(0, 30, n), seed)
    if kind == "gram_half_zero":              # rank n/2: the rest exactly zero
        return tridiagonal_of(np.concatenate([rng.random(n // 2), np.zeros(n - n // 2)]), seed)
    if kind == "clusters":                    # ten clusters of width 1e-14
        return tridiagonal_of(np.repeat(rng.random(10), -(-n // 10))[:n] + 1e-14 * rng.random(n), seed)
    if kind == "wilkinson":                   # W+: pairs of eigenvalues agreeing to many digits
        return np.abs(np.arange(n) - (n - 1) / 2.0), np.ones(n - 1)
    if kind == "split_zeros":                 # exactly zero couplings
        e = rng.standard_normal(n - 1)
        e[::7] = 0.0
        return rng.standard_normal(n), e
    if kind == "constant":                    # repeated diagonal entries, e = 0
        return np.full(n, 0.5), np.zeros(n - 1)
    raise ValueError(kind)


def check(d, e, label):
    n = d.shape[0]
    w, z = mps.selftest_stedc(d, e)
    t = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    tn = max(np.abs(np.linalg.eigvalsh(t)).max() if n > 1 else abs(d[0]), 1e-300)
    w_ref = eigh_tridiagonal(d, e, eigvals_only=True) if n > 1 else d.copy()
    ew = np.abs(w - w_ref).max() / tn
    res = np.abs(t @ z - z * w).max() / tn
    orth = np.abs(z.T @ z - np.eye(n)).max()
    msg = "%s n=%d eig %.1e res %.1e orth %.1e" % (label, n, ew, res, orth)
    print(msg)
    assert np.all(np.diff(w) >= 0), msg
    assert ew < TOL and res < TOL and orth < TOL, msg
    return w, z


@pytest.mark.parametrize("n", [1, 2, 3, 5, 64, 100, 257, 1000, 2047, 2048])
def test_random(n):
    d, e = case("random", n, seed=n)
    check(d, e, "random")


@pytest.mark.parametrize("kind", ["gram_graded", "gram_half_zero", "clusters", "split_zeros", "constant"])
@pytest.mark.parametrize("n", [97, 1024, 2048])
def test_structured(kind, n):
    d, e = case(kind, n, seed=7)
    check(d, e, kind)


@pytest.mark.parametrize("n", [21, 101, 1001])
def test_wilkinson(n):
    d, e = case("wilkinson", n)
    check(d, e, "wilkinson")


@pytest.mark.parametrize("n", [4, 255, 2048])
def test_closed_form_second_difference(n):
    d, e = np.full(n, 2.0), np.full(n - 1, -1.0)
    w, z = check(d, e, "second difference")
    k = np.arange(1, n + 1)
    exact = 2.0 - 2.0 * np.cos(k * np.pi / (n + 1))
    assert np.abs(w - np.sort(exact)).max() < 4 * n * 2.0 ** -52
    # eigenvector k: sin(i k pi / (n + 1)) normalised, up to sign
    i = np.arange(1, n + 1)
    for kk in (1, n // 2, n):
        v = np.sin(i * kk * np.pi / (n + 1))
        v /= np.linalg.norm(v)
        j = int(np.argmin(np.abs(w - (2.0 - 2.0 * np.cos(kk * np.pi / (n + 1))))))
        assert abs(abs(v @ z[:, j]) - 1.0) < 1e-10


def test_diagonal_closed_form():
    d = np.random.default_rng(3).standard_normal(300)
    w, z = mps.selftest_stedc(d, np.zeros(299))
    order = np.argsort(d, kind="stable")
    assert np.array_equal(w, d[order])
    assert np.array_equal(np.abs(z), np.eye(300)[:, order])


def test_rejects_bad_order():
    with pytest.raises(mps.MpsError):
        mps.selftest_stedc(np.zeros(2049), np.zeros(2048))
