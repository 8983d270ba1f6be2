"""FP64 oracle of the DMRG compression step -- TEST INFRASTRUCTURE ONLY.

Plain NumPy complex128 implementation of one compression step of the paper
(Sec. IV.B, the compression step), in its two-site variant (mentioned in the
same section), with K >= 1 layers per step and one qubit per MPS tensor
(Sec. IV.A with r_tau = 1) or r_tau consecutive qubits per tensor.

Steps, in the paper's order:
  * the layer's gates become an MPO: one-qubit gates are absorbed into the
    neighbouring tensors (the "trivial contractions" of Sec. IV.B.2) and every
    two-qubit gate is split by an SVD into a sum of products (eq:SVD, App. A.1);
  * the initial guess is a TEBD-like "zip-up" of the MPO into the MPS
    (the TEBD initialisation of Sec. V.D.1);
  * sweeps optimise two neighbouring tensors at a time: the local tensor F
    (eq:scalarproduct) is obtained by contracting the environments in the
    "vertical" order of Sec. IV.B.2, the optimum is F/sqrt(f)
    (eq:optimization), split back by an SVD that keeps the chi largest
    singular values (Sec. VI.A);
  * the partial fidelity of the step is f_delta = the f of the last local
    update (eq:fa-sup), and F~ = prod f_delta (eq:Ftilde-sup).

Readings where the paper is silent (each one is listed in the design notes):
  * truncation keeps chi' = min(chi, #{i : S_i^2 > 1e-12 * sum S^2}) values;
  * one sweep is one directional pass over the n-1 neighbouring pairs;
    directions alternate, the first sweep running against the zip-up;
  * the zip-up starts at the end of the chain that holds the orthogonality
    centre of the input MPS, so no re-canonicalisation pass is needed between
    layers;
  * a two-qubit gate's operator-Schmidt terms with sigma_a <= 1e-14 sigma_0
    are dropped;
  * composite MPO bonds order the open gates by their left chain site, the
    leftmost gate being the most significant digit.

Groupings (Sec. IV.A with r_tau > 1): r_tau consecutive qubits per tensor, physical
dimension 2^r_tau (group_state, group_mpo); the zip-up, the sweeps and the truncation run
unchanged on the grouped sites (apply_layers with sizes).

K > 1 layers per step (Sec. IV.B, the contraction of Sec. IV.B.2 with K layers
between the two MPS): the MPO of the step is the site-by-site product of the K
layer MPOs (step_mpo); everything else is unchanged, with one f_delta for the
K layers.

Single-site variant (the paper's production rule, Sec. IV.B, eq:optimization
with one free tensor): the same zip-up, then sweeps that optimise one tensor
at a time, F = L A W R, M = F / sqrt(f) with f = |F|^2, and move the
orthogonality centre by a QR (left-to-right) or LQ (right-to-left) of M.  The
bond dimensions are those of the zip-up (they can only shrink, when the QR of
a site has fewer rows than columns).  Readings: one single-site sweep visits
all n sites; f_delta is the f of the last site of the last sweep.

Everything here is plain and slow on purpose: dense MPO tensors, einsum, and
LAPACK's SVD and QR.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import philox

EPS_TRUNC = 1e-12
GATE_RANK_CUTOFF = 1e-14


# ------------------------------------------------------------------ MPO ----
@dataclasses.dataclass
class SplitGate:
    i: int            # left chain site
    j: int            # right chain site
    x: np.ndarray     # (r, 2, 2) operators on site i, [a, s, t]
    y: np.ndarray     # (r, 2, 2) operators on site j


def split_two_qubit(q0: int, q1: int, u: np.ndarray) -> SplitGate:
    """Operator-Schmidt split U = sum_a X_a (x) Y_a (eq:SVD; App. A.1).

    U's row/column index is 2*s_q0 + s_q1.  The split is the SVD of U
    regrouped as the matrix [(s_i t_i), (s_j t_j)] with i = min(q0, q1).
    """
    u4 = np.asarray(u, dtype=np.complex128).reshape(2, 2, 2, 2)   # [s0, s1, t0, t1]
    if q0 < q1:
        i, j = q0, q1
        ui = u4
    else:
        i, j = q1, q0
        ui = u4.transpose(1, 0, 3, 2)
    mat = ui.transpose(0, 2, 1, 3).reshape(4, 4)                 # [(s_i t_i), (s_j t_j)]
    uu, ss, vh = np.linalg.svd(mat)
    r = int(np.count_nonzero(ss > GATE_RANK_CUTOFF * ss[0]))
    x = np.stack([np.sqrt(ss[a]) * uu[:, a].reshape(2, 2) for a in range(r)])
    y = np.stack([np.sqrt(ss[a]) * vh[a, :].reshape(2, 2) for a in range(r)])
    return SplitGate(i=i, j=j, x=x, y=y)


def fuse_one_qubit(n: int, layer) -> List[np.ndarray]:
    """Product of the one-qubit gates of each site, in list order."""
    g = [np.eye(2, dtype=np.complex128) for _ in range(n)]
    for q0, q1, u in layer:
        if q1 < 0:
            g[q0] = np.asarray(u, dtype=np.complex128) @ g[q0]
    return g


def layer_mpo(n: int, layer) -> Tuple[List[np.ndarray], List[SplitGate]]:
    """Dense MPO tensors W_k[b, s, t, b'] of one layer (shape (w_k, 2, 2, w_{k+1})).

    Bond k lies left of site k; w_0 = w_n = 1.  The gates open at bond k are
    the two-qubit gates with i < k <= j, ordered by i; the bond index is the
    mixed-radix number of their operator-Schmidt indices, the gate with the
    smallest i being the most significant digit.
    """
    g1 = fuse_one_qubit(n, layer)
    gates = []
    used = set()
    for q0, q1, u in layer:
        if q1 < 0:
            continue
        if q0 == q1 or not (0 <= q0 < n and 0 <= q1 < n):
            raise ValueError("bad two-qubit gate sites")
        if q0 in used or q1 in used:
            raise ValueError("two-qubit gates of one layer must be disjoint")
        used.update((q0, q1))
        gates.append(split_two_qubit(q0, q1, u))
    gates.sort(key=lambda gt: gt.i)
    # the one-qubit gates act first: absorb them on the input leg t
    for gt in gates:
        gt.x = np.einsum("ast,tu->asu", gt.x, g1[gt.i])
        gt.y = np.einsum("ast,tu->asu", gt.y, g1[gt.j])
    open_at = [[gi for gi, gt in enumerate(gates) if gt.i < k <= gt.j] for k in range(n + 1)]
    starts = {gt.i: gi for gi, gt in enumerate(gates)}
    ends = {gt.j: gi for gi, gt in enumerate(gates)}

    def tuples(k):
        return list(itertools.product(*[range(gates[gi].x.shape[0]) for gi in open_at[k]]))

    mpo = []
    for k in range(n):
        left, right = open_at[k], open_at[k + 1]
        lt, rt = tuples(k), tuples(k + 1)
        rindex = {t: idx for idx, t in enumerate(rt)}
        w = np.zeros((len(lt), 2, 2, len(rt)), dtype=np.complex128)
        for bi, tup in enumerate(lt):
            labels = dict(zip(left, tup))
            if k in starts:
                gi = starts[k]
                for a in range(gates[gi].x.shape[0]):
                    lab = dict(labels)
                    lab[gi] = a
                    bo = rindex[tuple(lab[x] for x in right)]
                    w[bi, :, :, bo] += gates[gi].x[a]
            elif k in ends:
                gi = ends[k]
                a = labels[gi]
                bo = rindex[tuple(labels[x] for x in right)]
                w[bi, :, :, bo] += gates[gi].y[a]
            else:
                bo = rindex[tuple(labels[x] for x in right)]
                w[bi, :, :, bo] += g1[k]
        mpo.append(w)
    return mpo, gates


def step_mpo(n: int, layers) -> List[np.ndarray]:
    """Dense MPO of K consecutive layers U_K ... U_1 (Sec. IV.B with K > 1 layers per step).

    Site by site, the later layer acts on the output leg of the earlier one:
    W_k[(b_1 .. b_K), s, t, (b_1' .. b_K')] = sum over the inner physical indices
    of the product of the K layer tensors, the bond of layer 1 being the most
    significant part of the composite index."""
    layers = list(layers)
    if not layers:
        raise ValueError("a step needs at least one layer")
    mpo = layer_mpo(n, layers[0])[0]
    for layer in layers[1:]:
        nxt = layer_mpo(n, layer)[0]
        out = []
        for w1, w2 in zip(mpo, nxt):
            c = np.einsum("asub,cutd->acstbd", w2, w1)   # w2 after w1 on the physical leg
            out.append(c.reshape(w1.shape[0] * w2.shape[0], 2, 2, w1.shape[3] * w2.shape[3]))
        mpo = out
    return mpo


def mpo_bond_dims(mpo: Sequence[np.ndarray]) -> List[int]:
    return [mpo[0].shape[0]] + [w.shape[3] for w in mpo]


# ------------------------------------------------------------------ MPS ----
@dataclasses.dataclass
class StepRecord:
    kind: str          # "zip", "l2r" or "r2l"
    bond: int          # bond whose dimension the step decided (zip: -1)
    f: float           # partial fidelity after the step
    sum_s2: float      # sum of all squared singular values of the local tensor
    chi_kept: int
    gap: float = math.inf   # S_k / S_{k+1} - 1 at the cut (k kept); inf when nothing non-zero is cut
    kappa: float = 0.0      # first-order sensitivity of the state to the cut (truncated_svd_gap)


@dataclasses.dataclass
class OracleMPS:
    tensors: List[np.ndarray]      # A_k[a, s, b], shape (D_k, d_k, D_{k+1}); d_k = 2 per qubit of the site
    center: int                    # 0 or n-1: site holding the norm
    log_f: float = 0.0
    n_layers: int = 0
    n_2q: int = 0
    step_log: List[StepRecord] = dataclasses.field(default_factory=list)
    layer_f: List[float] = dataclasses.field(default_factory=list)

    @property
    def n(self) -> int:
        return len(self.tensors)

    def bond_dims(self) -> List[int]:
        return [self.tensors[0].shape[0]] + [a.shape[2] for a in self.tensors]


def product_state(n: int, bits: Optional[Sequence[int]] = None) -> OracleMPS:
    """|x> as an MPS of bond dimension 1 (Sec. IV.A: chi = 1 product state)."""
    bits = [0] * n if bits is None else list(bits)
    ts = []
    for k in range(n):
        a = np.zeros((1, 2, 1), dtype=np.complex128)
        a[0, int(bits[k]), 0] = 1.0
        ts.append(a)
    return OracleMPS(tensors=ts, center=0)


# ------------------------------------------------------------ truncation ---
def chi_at(chi, bond: int) -> int:
    """The cap of a bond: chi itself, or entry `bond` of a per-bond sequence."""
    return int(chi) if np.isscalar(chi) else int(chi[bond])


def _svd(m: np.ndarray):
    """Thin SVD by LAPACK: the divide-and-conquer driver, or the QR-iteration driver
    when divide and conquer does not converge (it can fail on exactly degenerate
    spectra, e.g. the states of SWAP networks); both compute the same factorisation."""
    try:
        return np.linalg.svd(m, full_matrices=False)
    except np.linalg.LinAlgError:
        import scipy.linalg
        return scipy.linalg.svd(m, full_matrices=False, lapack_driver="gesvd")


def truncated_svd_gap(m: np.ndarray, chi: int):
    """SVD keeping chi' = min(chi, #{S_i^2 > EPS_TRUNC * sum S^2}) values (Sec. VI.A).

    Also returns the conditioning of the cut, (gap, kappa):
      gap   = S_k / S_{k+1} - 1, the relative gap between the smallest kept and the
              largest discarded singular value (k kept; inf when nothing non-zero is
              discarded).  The kept subspace is unique only when it is non-zero.
      kappa = (S_1^2 / T) (S_k / sqrt(T)) / ((S_k^2 - S_{k+1}^2) / T), T = sum S^2:
              first-order perturbation theory (Davis-Kahan for the Gram matrix m m^H)
              turns a perturbation of relative size u of m m^H into a rotation of
              the kept subspace of at most u lambda_1 / (lambda_k - lambda_{k+1}),
              which moves the normalised state by that angle times the weight
              S_k / sqrt(T) of the mixed singular vector; with the same on the right
              (m^H m), 2 kappa u bounds the state's change at this cut to first
              order (kappa = 0 when nothing is discarded)."""
    u, s, vh = _svd(m)
    total = float(np.sum(s ** 2))
    if not total > 0.0 or not np.isfinite(total):
        raise FloatingPointError("local tensor has zero or non-finite norm")
    keep = int(np.count_nonzero(s ** 2 > EPS_TRUNC * total))
    k = max(1, min(chi, keep))
    gap, kappa = math.inf, 0.0
    if k < len(s) and s[k] > 0.0:
        gap = float(s[k - 1] / s[k] - 1.0)
        dl = float(s[k - 1] ** 2 - s[k] ** 2)
        kappa = math.inf if dl <= 0.0 else float(s[0] ** 2 * s[k - 1] / (dl * math.sqrt(total)))
    return u[:, :k], s[:k], vh[:k], total, (gap, kappa)


def truncated_svd(m: np.ndarray, chi: int):
    """truncated_svd_gap without the gap."""
    u, s, vh, total, _ = truncated_svd_gap(m, chi)
    return u, s, vh, total


# ---------------------------------------------------------- contractions ---
def _ein(spec, *ops):
    return np.einsum(spec, *ops, optimize=True)


def env_left_step(lenv, a, w, b):
    """L_{k+1}[q, c, x] = sum conj(B[p,s,q]) L_k[p,b,a] A[a,t,x] W[b,s,t,c]."""
    x = _ein("pba,atx->pbtx", lenv, a)
    x = _ein("pbtx,bstc->pscx", x, w)
    return _ein("pscx,psq->qcx", x, b.conj())


def env_right_step(renv, a, w, b):
    """R_k[p, b, y] = sum conj(B[p,s,q]) W[b,s,t,c] A[y,t,z] R_{k+1}[q,c,z]."""
    x = _ein("ytz,qcz->ytqc", a, renv)
    x = _ein("ytqc,bstc->ybsq", x, w)
    return _ein("ybsq,psq->pby", x, b.conj())


def two_site_tensor(lenv, a1, w1, a2, w2, renv):
    """Local tensor F of the pair (k, k+1): Theta[p, s, v, q] (eq:scalarproduct).

    Vertical order of Sec. IV.B.2: the top part (L, A_k, W_k, A_{k+1},
    W_{k+1}) is contracted downwards, then merged with R.
    """
    x = _ein("pba,atx->pbtx", lenv, a1)
    x = _ein("pbtx,bstc->pscx", x, w1)
    x = _ein("pscx,xuy->pscuy", x, a2)
    x = _ein("pscuy,cvue->psvey", x, w2)
    return _ein("psvey,qey->psvq", x, renv)


# ----------------------------------------------------------- zip-up -------
def zipup_left_to_right(a, w, chi, envs, log):
    n = len(a)
    b = [None] * n
    conds = []
    c = np.ones((1, 1, 1), dtype=np.complex128)
    envs[0] = c
    for k in range(n - 1):
        t = _ein("pba,atx,bstc->pscx", c, a[k], w[k])
        cl, ds, wk, dk = t.shape
        u, s, vh, total, cond = truncated_svd_gap(t.reshape(cl * ds, wk * dk), chi_at(chi, k + 1))
        b[k] = u.reshape(cl, ds, len(s))
        c = (s[:, None] * vh).reshape(len(s), wk, dk)
        envs[k + 1] = c
        conds.append(cond)
    t = _ein("pba,atx,bstc->pscx", c, a[n - 1], w[n - 1])
    f0 = float(np.sum(np.abs(t) ** 2))
    if not f0 > 0.0:
        raise FloatingPointError("zip-up produced a zero state")
    b[n - 1] = t.reshape(t.shape[0], t.shape[1], 1) / math.sqrt(f0)
    log.append(StepRecord("zip", -1, f0, f0, b[n - 1].shape[0], min((c[0] for c in conds), default=math.inf),
                         max((c[1] for c in conds), default=0.0)))
    return b, f0


def zipup_right_to_left(a, w, chi, envs, log):
    n = len(a)
    b = [None] * n
    conds = []
    c = np.ones((1, 1, 1), dtype=np.complex128)
    envs[n] = c
    for k in range(n - 1, 0, -1):
        t = _ein("qez,ytz,bste->ybsq", c, a[k], w[k])
        dk, wk, ds, cr = t.shape
        u, s, vh, total, cond = truncated_svd_gap(t.reshape(dk * wk, ds * cr), chi_at(chi, k))
        b[k] = vh.reshape(len(s), ds, cr)
        c = (u * s[None, :]).reshape(dk, wk, len(s)).transpose(2, 1, 0)
        envs[k] = c
        conds.append(cond)
    t = _ein("qez,ytz,bste->ybsq", c, a[0], w[0])
    f0 = float(np.sum(np.abs(t) ** 2))
    if not f0 > 0.0:
        raise FloatingPointError("zip-up produced a zero state")
    b[0] = t.reshape(1, t.shape[2], t.shape[3]) / math.sqrt(f0)
    log.append(StepRecord("zip", -1, f0, f0, b[0].shape[2], min((c[0] for c in conds), default=math.inf),
                         max((c[1] for c in conds), default=0.0)))
    return b, f0


# ----------------------------------------------------------- sweeps -------
def sweep_left_to_right(a, w, b, chi, envs, log):
    n = len(a)
    envs[0] = np.ones((1, 1, 1), dtype=np.complex128)
    f = None
    for k in range(n - 1):
        th = two_site_tensor(envs[k], a[k], w[k], a[k + 1], w[k + 1], envs[k + 2])
        cl, d1, d2, cr = th.shape
        u, s, vh, total, cond = truncated_svd_gap(th.reshape(cl * d1, d2 * cr), chi_at(chi, k + 1))
        f = float(np.sum(s ** 2))
        b[k] = u.reshape(cl, d1, len(s))
        b[k + 1] = (s[:, None] * vh / math.sqrt(f)).reshape(len(s), d2, cr)
        envs[k + 1] = env_left_step(envs[k], a[k], w[k], b[k])
        log.append(StepRecord("l2r", k + 1, f, total, len(s), *cond))
    return f


def sweep_right_to_left(a, w, b, chi, envs, log):
    n = len(a)
    envs[n] = np.ones((1, 1, 1), dtype=np.complex128)
    f = None
    for k in range(n - 2, -1, -1):
        th = two_site_tensor(envs[k], a[k], w[k], a[k + 1], w[k + 1], envs[k + 2])
        cl, d1, d2, cr = th.shape
        u, s, vh, total, cond = truncated_svd_gap(th.reshape(cl * d1, d2 * cr), chi_at(chi, k + 1))
        f = float(np.sum(s ** 2))
        b[k + 1] = vh.reshape(len(s), d2, cr)
        b[k] = (u * (s / math.sqrt(f))[None, :]).reshape(cl, d1, len(s))
        envs[k + 1] = env_right_step(envs[k + 2], a[k + 1], w[k + 1], b[k + 1])
        log.append(StepRecord("r2l", k + 1, f, total, len(s), *cond))
    return f


# ------------------------------------------------ single-site sweeps ------
def single_site_tensor(lenv, a, w, renv):
    """Local tensor of one site, F[p, s, q] = sum L[p,b,x] A[x,t,y] W[b,s,t,c] R[q,c,y]
    (eq:scalarproduct with one free tensor)."""
    x = _ein("pbx,xty->pbty", lenv, a)
    x = _ein("pbty,bstc->pscy", x, w)
    return _ein("pscy,qcy->psq", x, renv)


def sweep_single_left_to_right(a, w, b, envs, log):
    n = len(a)
    envs[0] = np.ones((1, 1, 1), dtype=np.complex128)
    f = None
    for k in range(n):
        m = single_site_tensor(envs[k], a[k], w[k], envs[k + 1])
        f = float(np.sum(np.abs(m) ** 2))
        if not f > 0.0:
            raise FloatingPointError("local tensor has zero norm")
        cl, ds, cr = m.shape
        if k == n - 1:
            b[k] = m / math.sqrt(f)
            log.append(StepRecord("l2r1", k + 1, f, f, cr))
            break
        q, _ = np.linalg.qr(m.reshape(cl * ds, cr))         # M = Q R, Q left-isometric
        b[k] = q.reshape(cl, ds, q.shape[1])
        envs[k + 1] = env_left_step(envs[k], a[k], w[k], b[k])
        log.append(StepRecord("l2r1", k + 1, f, f, q.shape[1]))
    return f


def sweep_single_right_to_left(a, w, b, envs, log):
    n = len(a)
    envs[n] = np.ones((1, 1, 1), dtype=np.complex128)
    f = None
    for k in range(n - 1, -1, -1):
        m = single_site_tensor(envs[k], a[k], w[k], envs[k + 1])
        f = float(np.sum(np.abs(m) ** 2))
        if not f > 0.0:
            raise FloatingPointError("local tensor has zero norm")
        cl, ds, cr = m.shape
        if k == 0:
            b[k] = m / math.sqrt(f)
            log.append(StepRecord("r2l1", k, f, f, cl))
            break
        # M = L Q with Q right-isometric: QR of M^H
        q, _ = np.linalg.qr(m.reshape(cl, ds * cr).conj().T)
        b[k] = q.conj().T.reshape(q.shape[1], ds, cr)
        envs[k] = env_right_step(envs[k + 1], a[k], w[k], b[k])
        log.append(StepRecord("r2l1", k, f, f, q.shape[1]))
    return f


# ------------------------------------------------------------ groupings ---
def _group(ts, sizes, join):
    sizes = [int(r) for r in sizes]
    if min(sizes, default=1) < 1 or sum(sizes) != len(ts):
        raise ValueError("group sizes must be >= 1 and add up to the number of qubits")
    out, k = [], 0
    for r in sizes:
        g = ts[k]
        for t in ts[k + 1:k + r]:
            g = join(g, t)
        out.append(g)
        k += r
    return out


def group_tensors(tensors: Sequence[np.ndarray], sizes: Sequence[int]) -> List[np.ndarray]:
    """Sites of r consecutive qubits (Sec. IV.A, r_tau qubits per tensor, physical dimension
    2^r_tau): A_g[a, (s_1 .. s_r), b] = sum over the inner bonds of A_1[a, s_1, .] ... A_r[., s_r, b],
    the group's first qubit the most significant digit of its index (so the state's amplitudes keep
    their order)."""
    return _group(list(tensors), sizes, lambda g, a: np.einsum("asb,btc->astc", g, a).reshape(
        g.shape[0], g.shape[1] * a.shape[1], a.shape[2]))


def group_mpo(mpo: Sequence[np.ndarray], sizes: Sequence[int]) -> List[np.ndarray]:
    """The MPO on the same sites: W_g[b, (s_1 .. s_r), (t_1 .. t_r), c] = sum over the inner MPO
    bonds of W_1 ... W_r, with the digit order of group_tensors on the output (s) and input (t)
    legs."""
    return _group(list(mpo), sizes, lambda g, w: np.einsum("bstc,cuvd->bsutvd", g, w).reshape(
        g.shape[0], g.shape[1] * w.shape[1], g.shape[2] * w.shape[2], w.shape[3]))


def group_state(state: OracleMPS, sizes: Sequence[int]) -> OracleMPS:
    """The same state with r_tau consecutive qubits per tensor; the norm stays at the chain end
    that held it."""
    ts = group_tensors(state.tensors, sizes)
    return OracleMPS(tensors=ts, center=0 if state.center == 0 else len(ts) - 1, log_f=state.log_f,
                     n_layers=state.n_layers, n_2q=state.n_2q)


# ------------------------------------------------------ compression step ---
def apply_layer(state: OracleMPS, layer, chi: int, n_sweeps: int, update: str = "two-site") -> float:
    """One compression step (K = 1): fit a bond-chi MPS to W|psi>, return f_delta.

    update = "two-site" (SVD split of each pair, bond dimensions up to chi) or
    "single-site" (bond dimensions of the zip-up, QR moves of the centre)."""
    return apply_layers(state, [layer], chi, n_sweeps, update)


def apply_layers(state: OracleMPS, layers, chi: int, n_sweeps: int, update: str = "two-site",
                 sizes: Optional[Sequence[int]] = None) -> float:
    """One compression step over K consecutive layers: fit a bond-chi MPS to
    U_K ... U_1 |psi> with the MPO of step_mpo; return f_delta (one f for the K layers).

    chi is one cap for every bond or a sequence of n + 1 caps, entry c for the bond
    between sites c - 1 and c (a grouping of the qubits into tensors leaves the bonds
    inside a group uncapped).

    sizes (Sec. IV.A, r_tau qubits per tensor): the number of consecutive qubits in each
    site of the state (made by group_state), default one each; the step's MPO is grouped
    the same way (group_mpo) and everything else is unchanged, with n the number of
    sites."""
    if np.isscalar(chi):
        if chi < 1:
            raise ValueError("chi >= 1 required")
    elif len(chi) != state.n + 1 or min(list(chi)[1:state.n] or [1]) < 1:
        raise ValueError("a per-bond chi needs n + 1 entries >= 1")
    if n_sweeps < 0:
        raise ValueError("n_sweeps >= 0 required")
    if update not in ("two-site", "single-site"):
        raise ValueError("update must be 'two-site' or 'single-site'")
    layers = list(layers)
    single = update == "single-site"
    n = state.n
    if sizes is None:
        w = step_mpo(n, layers)
    else:
        sizes = [int(r) for r in sizes]
        if len(sizes) != n or min(sizes) < 1:
            raise ValueError("sizes needs one entry >= 1 per site of the state")
        if any(a.shape[1] != 2 ** r for a, r in zip(state.tensors, sizes)):
            raise ValueError("the state's physical dimensions are not 2^sizes")
        w = group_mpo(step_mpo(sum(sizes), layers), sizes)
    a = state.tensors
    envs: Dict[int, np.ndarray] = {}
    log: List[StepRecord] = []
    if state.center == 0:
        b, f = zipup_left_to_right(a, w, chi, envs, log)
        direction = "r2l"
        center = n - 1
    else:
        b, f = zipup_right_to_left(a, w, chi, envs, log)
        direction = "l2r"
        center = 0
    if n >= 2:
        for _ in range(n_sweeps):
            if direction == "r2l":
                f = (sweep_single_right_to_left(a, w, b, envs, log) if single
                     else sweep_right_to_left(a, w, b, chi, envs, log))
                center, direction = 0, "l2r"
            else:
                f = (sweep_single_left_to_right(a, w, b, envs, log) if single
                     else sweep_left_to_right(a, w, b, chi, envs, log))
                center, direction = n - 1, "r2l"
    state.tensors = b
    state.center = center
    state.log_f += math.log(f)
    state.n_layers += len(layers)
    state.n_2q += sum(1 for layer in layers for g in layer if g[1] >= 0)
    state.step_log.extend(log)
    state.layer_f.append(f)
    return f


def fidelity(state: OracleMPS):
    """F~ = prod f_delta (eq:Ftilde-sup) and eps~ = 1 - F~^{1/N_2g}."""
    f_tilde = math.exp(state.log_f)
    eps = 1.0 - f_tilde ** (1.0 / state.n_2q) if state.n_2q > 0 else 0.0
    return f_tilde, state.log_f, eps


def run_circuit(circuit, chi: int, n_sweeps: int, depth: Optional[int] = None,
                bits=None) -> OracleMPS:
    st = product_state(circuit.n, bits)
    layers = circuit.layers if depth is None else circuit.layers[:depth]
    for layer in layers:
        apply_layer(st, layer, chi, n_sweeps)
    return st


# ------------------------------------------------------ amplitudes, etc. ---
def amplitude(state: OracleMPS, bits: Sequence[int]) -> complex:
    v = np.ones((1,), dtype=np.complex128)
    for k, a in enumerate(state.tensors):
        v = v @ a[:, int(bits[k]), :]
    return complex(v[0])


def to_statevector(state: OracleMPS) -> np.ndarray:
    v = np.ones((1, 1), dtype=np.complex128)                 # [x, bond]
    for a in state.tensors:
        v = np.einsum("xa,asb->xsb", v, a).reshape(-1, a.shape[2])
    return v.reshape(-1)


def overlap(bra: OracleMPS, ket: OracleMPS) -> complex:
    """<bra|ket>."""
    e = np.ones((1, 1), dtype=np.complex128)
    for a, b in zip(bra.tensors, ket.tensors):
        e = np.einsum("pq,psr,qst->rt", e, a.conj(), b)
    return complex(e[0, 0])


def sample(state: OracleMPS, n_samples: int, seed: int) -> np.ndarray:
    """Exact sequential sampling of |phi(x)|^2, starting at the centre site.

    Bits are returned as an (n_samples, n) uint8 array.  The uniform number for
    sample j at site k is ``philox.uniform(seed, j, k)``; site k takes value 0
    when that number is below p(0 | earlier sites).
    """
    n = state.n
    order = range(n) if state.center == 0 else range(n - 1, -1, -1)
    out = np.zeros((n_samples, n), dtype=np.uint8)
    for j in range(n_samples):
        v = np.ones((1,), dtype=np.complex128)
        for k in order:
            a = state.tensors[k]
            if state.center == 0:
                u0, u1 = v @ a[:, 0, :], v @ a[:, 1, :]
            else:
                u0, u1 = a[:, 0, :] @ v, a[:, 1, :] @ v
            p0 = float(np.vdot(u0, u0).real)
            p1 = float(np.vdot(u1, u1).real)
            r = philox.uniform(seed, j, k)
            if r < p0 / (p0 + p1):
                out[j, k], v = 0, u0 / math.sqrt(p0)
            else:
                out[j, k], v = 1, u1 / math.sqrt(p1)
    return out


def expectation_zz(state: OracleMPS, i: int, j: int) -> float:
    """<phi| Z_i Z_j |phi> by a transfer-matrix contraction (Z_i alone when i == j)."""
    z = np.array([1.0, -1.0])
    e = np.ones((1, 1), dtype=np.complex128)
    for k, a in enumerate(state.tensors):
        if k == i or k == j:
            op = z if i != j else z
            a_op = a * op[None, :, None]
        else:
            a_op = a
        e = np.einsum("pq,psr,qst->rt", e, a.conj(), a_op)
    return float(e[0, 0].real)
