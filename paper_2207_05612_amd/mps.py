"""Python binding of the C ABI in ``include/mps_dmrg.h`` (argument marshalling only).

Every computation runs in the HIP library ``libmpsdmrg.so``; this module only
converts NumPy arrays to pointers and status codes to exceptions.  Loading
fails loudly when the library has not been built: there is no fallback.

PyTorch supplies the HIP stream (``torch.cuda.current_stream()``) when it is
importable and a GPU is visible; otherwise the default stream is used.  With
``torch_allocator=True`` a state takes its device memory from PyTorch's
caching allocator (``torch.cuda.caching_allocator_alloc`` / ``_delete``)
through the ABI's allocator callbacks.

States and statevectors still open when the interpreter exits are destroyed
by an exit hook registered after PyTorch's own, so it runs first, while the
HIP runtime is still whole.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Optional, Sequence

import numpy as np

from . import circuits

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpsdmrg.so")

MPS_OK, MPS_ERR_ARG, MPS_ERR_OOM, MPS_ERR_DEVICE, MPS_ERR_NUMERIC, MPS_ERR_STATE = 0, -1, -2, -3, -4, -5
MPS_FP64, MPS_FP32, MPS_BF16X2, MPS_BF16X3 = 0, 1, 2, 3
MPS_UPDATE_TWO_SITE, MPS_UPDATE_SINGLE_SITE = 0, 1
_UPDATES = {"two-site": MPS_UPDATE_TWO_SITE, "single-site": MPS_UPDATE_SINGLE_SITE}
KCLASS = {"contract": 0, "mpo": 1, "gram": 2, "eigh": 3, "other": 4, "tridiag": 5}

# every symbol declared in include/mps_dmrg.h
EXPORTS = ("mps_create", "mps_destroy", "apply_layer_dmrg", "apply_layer_dmrg_single_site",
           "apply_layer_dmrg_batched", "fidelity", "sample",
           "mps_last_error",
           "mps_amplitude", "mps_to_statevector", "mps_bond_dims", "mps_get_tensor", "mps_step_log",
           "mps_expect_zz", "mps_set_profiling", "mps_kernel_stats", "mps_kernel_selftest_cgemm",
           "mps_kernel_selftest_eigh", "mps_overlap", "apply_layers_dmrg",
           "sv_create", "sv_destroy", "sv_apply_layer", "sv_amplitudes", "sv_compare_mps",
           "sv_schmidt_weights", "apply_layers_dmrg_bonds", "mps_eigensolver_counts", "mps_cgemm_noalloc",
           "mps_overlap_layers", "mps_batch_stats", "mps_kernel_selftest_stedc",
           "mps_cut_separations")

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class MpsAllocator(ctypes.Structure):
    """struct mps_allocator of the ABI."""
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]

_lib = None
_live = weakref.WeakSet()        # open MPS / Statevector handles, closed by the exit hook


def _close_all() -> None:
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


class MpsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("mps status %d: %s" % (code, msg))
        self.code = code


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmpsdmrg.so and declare the ABI; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("HIP library %s is not built; run `python -m paper_2207_05612_amd.build`" % path)
    try:
        # the library shares PyTorch's HIP runtime; let PyTorch map it first
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    # registered after PyTorch's exit hooks, so it runs before them
    atexit.register(_close_all)
    P = ctypes.c_void_p
    i32, i64, u64, dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    sig = {
        "mps_create": (i32, [i32, P, i32, i32, P, ctypes.POINTER(MpsAllocator), ctypes.POINTER(P)]),
        "mps_eigensolver_counts": (i32, [P, ctypes.POINTER(i64)]),
        "mps_cgemm_noalloc": (i32, [i32, i32, i32, i32, i32, i32, P, P, i64, P, P, i64, P, P, i64, P]),
        "mps_destroy": (i32, [P]),
        "apply_layer_dmrg": (i32, [P, P, i32, i32, i32, dp]),
        "apply_layer_dmrg_single_site": (i32, [P, P, i32, i32, i32, dp]),
        "apply_layer_dmrg_batched": (i32, [ctypes.POINTER(P), i32, ctypes.POINTER(P), ip, ip, i32, dp]),
        "fidelity": (i32, [P, dp, dp, ip, ctypes.POINTER(i64)]),
        "sample": (i32, [P, i64, u64, P]),
        "mps_last_error": (ctypes.c_char_p, []),
        "mps_amplitude": (i32, [P, i32, P, dp]),
        "mps_to_statevector": (i32, [P, dp]),
        "mps_bond_dims": (i32, [P, ip]),
        "mps_get_tensor": (i32, [P, i32, dp]),
        "mps_step_log": (i32, [P, dp, dp, ip, i32, ip]),
        "mps_cut_separations": (i32, [P, dp, i32, ip]),
        "mps_expect_zz": (i32, [P, i32, i32, dp]),
        "mps_set_profiling": (i32, [P, i32]),
        "mps_kernel_stats": (i32, [P, i32, ctypes.POINTER(i64), dp, dp, dp]),
        "mps_kernel_selftest_cgemm": (i32, [i32, i32, i32, i32, i32, i32, dp, dp, dp]),
        "mps_kernel_selftest_eigh": (i32, [i32, dp, i32, dp, dp, ip]),
        "mps_kernel_selftest_stedc": (i32, [i32, dp, dp, dp, dp]),
        "mps_overlap": (i32, [P, P, dp, dp]),
        "mps_overlap_layers": (i32, [P, P, P, ip, i32, dp, dp]),
        "mps_batch_stats": (i32, [ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "apply_layers_dmrg": (i32, [P, P, ip, i32, i32, i32, i32, dp]),
        "sv_create": (i32, [i32, P, P, ctypes.POINTER(P)]),
        "sv_destroy": (i32, [P]),
        "sv_apply_layer": (i32, [P, P, i32]),
        "sv_amplitudes": (i32, [P, i64, P, dp]),
        "sv_compare_mps": (i32, [P, P, dp, dp, dp, dp]),
        "sv_schmidt_weights": (i32, [P, i32, i32, dp, dp, dp]),
        "apply_layers_dmrg_bonds": (i32, [P, P, ip, i32, ip, i32, i32, dp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(code: int) -> None:
    if code != MPS_OK:
        raise MpsError(code, _lib.mps_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def current_stream() -> Optional[int]:
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except ImportError:
        pass
    return None


def _torch_allocator():
    """Allocator callbacks onto PyTorch's caching allocator (current device): the ABI
    struct and the two ctypes callback objects, which must stay alive with it."""
    import torch
    dev = torch.cuda.current_device()

    def alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream or 0)
        except Exception:
            return None

    def free(ptr, stream, user):
        torch.cuda.caching_allocator_delete(ptr)

    fa, ff = ALLOC_FN(alloc), FREE_FN(free)
    return MpsAllocator(fa, ff, None), (fa, ff)


class MPS:
    """Handle of one on-GPU MPS (owns an ``mps_state*``).

    torch_allocator=True: device memory from PyTorch's caching allocator (the
    ABI's allocator callbacks); otherwise the library's own stream-ordered pool."""

    def __init__(self, n: int, bits: Optional[Sequence[int]] = None, max_chi: int = 1024,
                 precision: int = MPS_FP32, stream: Optional[int] = None, torch_allocator: bool = False):
        lib = load_library()
        self.n = n
        self.precision = precision
        self._h = ctypes.c_void_p()
        bits_arr = None if bits is None else np.ascontiguousarray(bits, dtype=np.uint8)
        if stream is None:
            stream = current_stream()
        # the callbacks must outlive the state
        self._alloc, self._alloc_fns = _torch_allocator() if torch_allocator else (None, None)
        _check(lib.mps_create(n, None if bits_arr is None else bits_arr.ctypes.data, max_chi, precision,
                              stream, ctypes.byref(self._alloc) if self._alloc is not None else None,
                              ctypes.byref(self._h)))
        _live.add(self)

    def close(self) -> None:
        if self._h:
            _lib.mps_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the compression step ------------------------------------------------
    def apply_layer_dmrg(self, layer, chi: int, n_sweeps: int, update: str = "two-site") -> float:
        """update = "two-site" (apply_layer_dmrg) or "single-site" (apply_layer_dmrg_single_site)."""
        rec = layer if isinstance(layer, np.ndarray) else circuits.pack_layer(layer)
        rec = np.ascontiguousarray(rec, dtype=circuits.GATE_DTYPE)
        f = ctypes.c_double(0.0)
        if update == "two-site":
            fn = _lib.apply_layer_dmrg
        elif update == "single-site":
            fn = _lib.apply_layer_dmrg_single_site
        else:
            raise ValueError("update must be 'two-site' or 'single-site'")
        _check(fn(self._h, rec.ctypes.data, len(rec), chi, n_sweeps, ctypes.byref(f)))
        return f.value

    def apply_layers_dmrg(self, layers, chi, n_sweeps: int, update: str = "two-site") -> float:
        """One compression step over K = len(layers) consecutive layers (apply_layers_dmrg).

        chi is one cap for every bond, or n + 1 per-bond caps (apply_layers_dmrg_bonds; see
        circuits.group_bond_profile for qubit groupings)."""
        if update not in _UPDATES:
            raise ValueError("update must be 'two-site' or 'single-site'")
        recs = [np.ascontiguousarray(l if isinstance(l, np.ndarray) else circuits.pack_layer(l),
                                     dtype=circuits.GATE_DTYPE) for l in layers]
        counts = np.ascontiguousarray([len(r) for r in recs], dtype=np.int32)
        allrec = np.ascontiguousarray(np.concatenate(recs) if recs else np.zeros(0, circuits.GATE_DTYPE),
                                      dtype=circuits.GATE_DTYPE)
        f = ctypes.c_double(0.0)
        gp = allrec.ctypes.data if len(allrec) else None
        if np.isscalar(chi):
            _check(_lib.apply_layers_dmrg(self._h, gp, _iptr(counts), len(recs), int(chi), n_sweeps,
                                          _UPDATES[update], ctypes.byref(f)))
        else:
            caps = np.ascontiguousarray(chi, dtype=np.int32)
            if caps.shape != (self.n + 1,):
                raise ValueError("a per-bond chi needs n + 1 entries")
            _check(_lib.apply_layers_dmrg_bonds(self._h, gp, _iptr(counts), len(recs), _iptr(caps), n_sweeps,
                                                _UPDATES[update], ctypes.byref(f)))
        return f.value

    def fidelity(self):
        F, lf, nl, n2 = ctypes.c_double(), ctypes.c_double(), ctypes.c_int(), ctypes.c_int64()
        _check(_lib.fidelity(self._h, ctypes.byref(F), ctypes.byref(lf), ctypes.byref(nl), ctypes.byref(n2)))
        eps = 1.0 - F.value ** (1.0 / n2.value) if n2.value > 0 else 0.0
        return {"F_tilde": F.value, "log_F_tilde": lf.value, "n_layers": nl.value,
                "n_2q": n2.value, "eps_tilde": eps}

    def sample(self, n_samples: int, seed: int) -> np.ndarray:
        """(n_samples, n) uint8 bits."""
        words = (self.n + 63) // 64
        out = np.zeros((n_samples, words), dtype=np.uint64)
        _check(_lib.sample(self._h, n_samples, seed, out.ctypes.data))
        bits = np.zeros((n_samples, self.n), dtype=np.uint8)
        for k in range(self.n):
            bits[:, k] = ((out[:, k // 64] >> np.uint64(k % 64)) & np.uint64(1)).astype(np.uint8)
        return bits

    # -- inspection --------------------------------------------------------------
    def amplitudes(self, bits: np.ndarray) -> np.ndarray:
        b = np.ascontiguousarray(np.atleast_2d(bits), dtype=np.uint8)
        out = np.zeros(2 * b.shape[0])
        _check(_lib.mps_amplitude(self._h, b.shape[0], b.ctypes.data, _dptr(out)))
        return out[0::2] + 1j * out[1::2]

    def statevector(self) -> np.ndarray:
        out = np.zeros(2 * 2 ** self.n)
        _check(_lib.mps_to_statevector(self._h, _dptr(out)))
        return out[0::2] + 1j * out[1::2]

    def bond_dims(self):
        out = np.zeros(self.n + 1, dtype=np.int32)
        _check(_lib.mps_bond_dims(self._h, _iptr(out)))
        return [int(x) for x in out]

    def tensor(self, site: int) -> np.ndarray:
        d = self.bond_dims()
        out = np.zeros(2 * d[site] * 2 * d[site + 1])
        _check(_lib.mps_get_tensor(self._h, site, _dptr(out)))
        return (out[0::2] + 1j * out[1::2]).reshape(d[site], 2, d[site + 1])

    def step_log(self):
        n = ctypes.c_int()
        _check(_lib.mps_step_log(self._h, None, None, None, 0, ctypes.byref(n)))
        m = n.value
        f, s2 = np.zeros(max(m, 1)), np.zeros(max(m, 1))
        k = np.zeros(max(m, 1), dtype=np.int32)
        _check(_lib.mps_step_log(self._h, _dptr(f), _dptr(s2), _iptr(k), m, ctypes.byref(n)))
        return f[:m], s2[:m], k[:m]

    def cut_separations(self):
        """Per applied step, the smallest (lambda_k - lambda_k+1) / lambda_1 at a cut where chi
        limited the kept count (inf where it limited none); see mps_cut_separations."""
        n = ctypes.c_int()
        _check(_lib.mps_cut_separations(self._h, None, 0, ctypes.byref(n)))
        m = n.value
        out = np.zeros(max(m, 1))
        _check(_lib.mps_cut_separations(self._h, _dptr(out), m, ctypes.byref(n)))
        return out[:m]

    def counters(self) -> dict:
        """Eigensolver paths of the truncations so far (mps_eigensolver_counts)."""
        c = (ctypes.c_int64 * 4)()
        _check(_lib.mps_eigensolver_counts(self._h, c))
        return {"persistent": c[0], "single_workgroup": c[1], "fallback_library": c[2], "library": c[3]}

    def expect_zz(self, i: int, j: int) -> float:
        v = ctypes.c_double()
        _check(_lib.mps_expect_zz(self._h, i, j, ctypes.byref(v)))
        return v.value

    # -- measurement -------------------------------------------------------------
    def set_profiling(self, on: bool) -> None:
        _check(_lib.mps_set_profiling(self._h, 1 if on else 0))

    def kernel_stats(self, cls: str):
        n, ms, fl, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(_lib.mps_kernel_stats(self._h, KCLASS[cls], ctypes.byref(n), ctypes.byref(ms),
                                     ctypes.byref(fl), ctypes.byref(by)))
        return {"launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}


def selftest_cgemm(precision: int, opa: int, opb: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """C = op(a) op(b) through the library's GEMM kernel (see mps_kernel_selftest_cgemm)."""
    lib = load_library()
    a = np.ascontiguousarray(a, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    M, K = (a.shape[0], a.shape[1]) if opa == 0 else (a.shape[1], a.shape[0])
    N = b.shape[1] if opb == 0 else b.shape[0]
    c = np.zeros((M, N), dtype=np.complex128)
    _check(lib.mps_kernel_selftest_cgemm(precision, opa, opb, M, N, K, _dptr(a.view(np.float64)),
                                         _dptr(b.view(np.float64)), _dptr(c.view(np.float64))))
    return c


def cgemm_noalloc(precision: int, opa: int, opb: int, M: int, N: int, K: int, a, lda: int, b, ldb: int, c,
                  ldc: int, stream: Optional[int] = None) -> None:
    """mps_cgemm_noalloc on device planar operands: a, b, c are (re, im) pairs of device
    pointers (ints, e.g. torch tensors' data_ptr()); queued on `stream`, not awaited."""
    lib = load_library()
    if stream is None:
        stream = current_stream()
    _check(lib.mps_cgemm_noalloc(precision, opa, opb, M, N, K, a[0], a[1], lda, b[0], b[1], ldb, c[0], c[1], ldc,
                                 stream))


def overlap(bra: "MPS", ket: "MPS") -> complex:
    """<bra|ket> (see mps_overlap)."""
    re, im = ctypes.c_double(), ctypes.c_double()
    _check(_lib.mps_overlap(bra._h, ket._h, ctypes.byref(re), ctypes.byref(im)))
    return complex(re.value, im.value)


def overlap_layers(bra: "MPS", layers, ket: "MPS") -> complex:
    """<bra| U_K ... U_1 |ket> with the layers contracted exactly (see mps_overlap_layers)."""
    recs = [np.ascontiguousarray(l if isinstance(l, np.ndarray) else circuits.pack_layer(l),
                                 dtype=circuits.GATE_DTYPE) for l in layers]
    counts = np.ascontiguousarray([len(r) for r in recs], dtype=np.int32)
    allrec = np.ascontiguousarray(np.concatenate(recs) if recs else np.zeros(0, circuits.GATE_DTYPE),
                                  dtype=circuits.GATE_DTYPE)
    re, im = ctypes.c_double(), ctypes.c_double()
    _check(_lib.mps_overlap_layers(bra._h, ket._h, allrec.ctypes.data if len(allrec) else None, _iptr(counts),
                                   len(recs), ctypes.byref(re), ctypes.byref(im)))
    return complex(re.value, im.value)


EIGH_ROCSOLVER, EIGH_PERSISTENT = 0, 1


def selftest_eigh(a: np.ndarray, method: int = EIGH_PERSISTENT):
    """Eigenvalues (ascending), eigenvectors (columns) and the method that ran, through the
    library's FP64 eigensolver (see mps_kernel_selftest_eigh).  Only the lower triangle of a is read."""
    lib = load_library()
    a = np.ascontiguousarray(a, dtype=np.complex128)
    n = a.shape[0]
    w = np.zeros(n)
    z = np.zeros((n, n), dtype=np.complex128)      # filled column-major: z.T[j] is eigenvector j
    used = ctypes.c_int(-1)
    _check(lib.mps_kernel_selftest_eigh(n, _dptr(a.view(np.float64)), method, _dptr(w),
                                        _dptr(z.view(np.float64)), ctypes.byref(used)))
    return w, np.ascontiguousarray(z.T), used.value


def selftest_stedc(d: np.ndarray, e: np.ndarray):
    """Eigenvalues (ascending) and eigenvectors (columns) of the real symmetric tridiagonal
    matrix (d, e) through the library's divide and conquer (see mps_kernel_selftest_stedc)."""
    lib = load_library()
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    n = d.shape[0]
    if e.shape[0] != max(n - 1, 0):
        raise ValueError("e must have n - 1 entries")
    w = np.zeros(n)
    z = np.zeros((n, n))                           # filled column-major: z.T[j] is eigenvector j
    _check(lib.mps_kernel_selftest_stedc(n, _dptr(d), _dptr(e) if n > 1 else None, _dptr(w), _dptr(z)))
    return w, np.ascontiguousarray(z.T)


# free functions with the ABI's names
def mps_create(n, bits=None, max_chi=1024, precision=MPS_FP32, stream=None, torch_allocator=False) -> MPS:
    return MPS(n, bits, max_chi, precision, stream, torch_allocator)


def apply_layer_dmrg(state: MPS, layer, chi: int, n_sweeps: int) -> float:
    return state.apply_layer_dmrg(layer, chi, n_sweeps)


def apply_layers_dmrg(state: MPS, layers, chi: int, n_sweeps: int, update: str = "two-site") -> float:
    return state.apply_layers_dmrg(layers, chi, n_sweeps, update)


def apply_layer_dmrg_batched(states: Sequence[MPS], layers, chis: Sequence[int], n_sweeps: int) -> np.ndarray:
    """One layer per instance, run concurrently (each state should own a stream)."""
    lib = load_library()
    b = len(states)
    recs = [np.ascontiguousarray(layer if isinstance(layer, np.ndarray) else circuits.pack_layer(layer),
                                 dtype=circuits.GATE_DTYPE) for layer in layers]
    hs = (ctypes.c_void_p * b)(*[s._h.value for s in states])
    gp = (ctypes.c_void_p * b)(*[r.ctypes.data if len(r) else None for r in recs])
    ng = np.ascontiguousarray([len(r) for r in recs], dtype=np.int32)
    ch = np.ascontiguousarray(chis, dtype=np.int32)
    f = np.zeros(b)
    _check(lib.apply_layer_dmrg_batched(hs, b, gp, _iptr(ng), _iptr(ch), n_sweeps, _dptr(f)))
    return f


def batch_stats():
    """(shared tridiagonal-reduction launches, reductions they carried) of the batched calls."""
    lib = load_library()
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(lib.mps_batch_stats(ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def fidelity(state: MPS):
    return state.fidelity()


def sample(state: MPS, n_samples: int, seed: int) -> np.ndarray:
    return state.sample(n_samples, seed)


def mps_destroy(state: MPS) -> None:
    state.close()


class Statevector:
    """Handle of an exact on-GPU statevector (owns an ``sv_state*``): the perfect state
    against which an MPS is measured (F of eq:F-sup, F_B of eq:FB-sup)."""

    def __init__(self, n: int, bits: Optional[Sequence[int]] = None, stream: Optional[int] = None):
        lib = load_library()
        self.n = n
        self._h = ctypes.c_void_p()
        bits_arr = None if bits is None else np.ascontiguousarray(bits, dtype=np.uint8)
        if stream is None:
            stream = current_stream()
        _check(lib.sv_create(n, None if bits_arr is None else bits_arr.ctypes.data, stream, ctypes.byref(self._h)))
        _live.add(self)

    def close(self) -> None:
        if self._h:
            _lib.sv_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply_layer(self, layer) -> None:
        rec = np.ascontiguousarray(layer if isinstance(layer, np.ndarray) else circuits.pack_layer(layer),
                                   dtype=circuits.GATE_DTYPE)
        _check(_lib.sv_apply_layer(self._h, rec.ctypes.data if len(rec) else None, len(rec)))

    def amplitudes_at(self, indices) -> np.ndarray:
        idx = np.ascontiguousarray(indices, dtype=np.int64)
        out = np.zeros(2 * len(idx))
        _check(_lib.sv_amplitudes(self._h, len(idx), idx.ctypes.data if len(idx) else None, _dptr(out)))
        return out[0::2] + 1j * out[1::2]

    def compare(self, state: "MPS") -> dict:
        """<phi|psi>, F, F_B and both norms of an MPS phi against this exact state psi."""
        ov, F, FB, nrm = np.zeros(2), ctypes.c_double(), ctypes.c_double(), np.zeros(2)
        _check(_lib.sv_compare_mps(self._h, state._h, _dptr(ov), ctypes.byref(F), ctypes.byref(FB), _dptr(nrm)))
        return {"overlap": complex(ov[0], ov[1]), "F": F.value, "F_B": FB.value,
                "norm_mps": nrm[0], "norm_exact": nrm[1]}

    def schmidt(self, cut: int, chi: int):
        """(kept weight of the chi largest S^2, total weight, all S^2 largest first) at `cut`."""
        dim = 2 ** min(cut, self.n - cut)
        kept, total, s2 = ctypes.c_double(), ctypes.c_double(), np.zeros(dim)
        _check(_lib.sv_schmidt_weights(self._h, cut, chi, ctypes.byref(kept), ctypes.byref(total), _dptr(s2)))
        return kept.value, total.value, s2
