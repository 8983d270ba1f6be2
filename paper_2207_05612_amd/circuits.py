"""Seeded synthetic random-circuit generators.

This module produces *inputs* only: gate matrices, the qubit -> chain-site map
and the per-layer gate lists.  It holds none of the compression method's
arithmetic and is shared by the FP64 oracle (``oracle/``) and by the GPU path,
so both see bit-identical gates for a given seed.

Workloads follow the paper's random-circuit construction (Sec. V.A, "Three
quantum circuits"): every cycle applies a random one-qubit gate on every qubit,
drawn from {sqrt(X), sqrt(Y), sqrt(W)}, followed by two-qubit gates on the
pairs of one coupler pattern, patterns cycling ABCD-CDAB.  The paper's
Sycamore lattice is replaced by a rectangular grid read in snake order along
its short side (one qubit per MPS site, Sec. IV.A with r_tau = 1).

Conventions shared with the C ABI:
  * a gate is ``(q0, q1, U)``; ``q1 = -1`` for one-qubit gates;
  * one-qubit ``U`` is 2x2 with ``U[out, in]``;
  * two-qubit ``U`` is 4x4 with row/column index ``2*s_q0 + s_q1``;
  * inside one layer every one-qubit gate acts before every two-qubit gate,
    and the two-qubit gates act on disjoint sites.

Draw order of cycle d (``numpy.random.default_rng(seed)``, PCG64):
  1. ``integers(0, 3, size=n)`` one-qubit choices, qubits in row-major grid
     order;
  2. for each pair of pattern ``SEQUENCE[d % 8]``, sorted by chain site, its
     two-qubit gate: Haar = 32 ``standard_normal`` draws, fSim = theta then phi.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

# ---------------------------------------------------------------- gate set --
I2 = np.eye(2, dtype=np.complex128)
PAULI_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PAULI_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PAULI_W = (PAULI_X + PAULI_Y) / np.sqrt(2.0)


def sqrt_pauli(g: np.ndarray) -> np.ndarray:
    """Square root of a Pauli-like involution G (G @ G = I): (I - iG)/sqrt(2).

    Its square is -iG, i.e. G up to a global phase.
    """
    return (I2 - 1j * g) / np.sqrt(2.0)


SQRT_X = sqrt_pauli(PAULI_X)
SQRT_Y = sqrt_pauli(PAULI_Y)
SQRT_W = sqrt_pauli(PAULI_W)
ONE_QUBIT_SET = (SQRT_X, SQRT_Y, SQRT_W)


def fsim(theta: float, phi: float) -> np.ndarray:
    """fSim(theta, phi) in the basis |00>,|01>,|10>,|11> (index 2*s0 + s1)."""
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[1, 0, 0, 0],
                     [0, c, -1j * s, 0],
                     [0, -1j * s, c, 0],
                     [0, 0, 0, np.exp(-1j * phi)]], dtype=np.complex128)


def haar_unitary_from_normals(z: np.ndarray, dim: int = 4) -> np.ndarray:
    """Haar-distributed U(dim) from 2*dim*dim standard normal draws.

    QR of a complex Ginibre matrix with the phases of diag(R) moved into Q
    (Mezzadri, Notices AMS 54 (2007) 592).
    """
    z = np.asarray(z, dtype=np.float64).reshape(2, dim, dim)
    g = (z[0] + 1j * z[1]) / np.sqrt(2.0)
    q, r = np.linalg.qr(g)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def zz_phase(gamma: float) -> np.ndarray:
    """exp(-i gamma Z x Z), diagonal in the computational basis."""
    z = np.array([1, -1, -1, 1], dtype=np.float64)
    return np.diag(np.exp(-1j * gamma * z)).astype(np.complex128)


def rx(beta2: float) -> np.ndarray:
    """RX(beta2) = exp(-i beta2/2 X); the QAOA mixer exp(-i beta X) is RX(2 beta)."""
    c, s = np.cos(beta2 / 2), np.sin(beta2 / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]],
                dtype=np.complex128)

# ------------------------------------------------------------ geometry -----
@dataclasses.dataclass(frozen=True)
class Grid:
    """Rectangular grid of ``n`` qubits, ``width`` columns, rows filled in order.

    The last row may be partial.  Qubit (r, c) sits on chain site
    ``r*width + c`` on even rows and ``r*width + (m_r - 1 - c)`` on odd rows,
    m_r being the number of qubits in row r (snake order).
    """
    n: int
    width: int

    @property
    def rows(self) -> int:
        return -(-self.n // self.width)

    def row_len(self, r: int) -> int:
        return min(self.width, self.n - r * self.width)

    def coords(self) -> List[Tuple[int, int]]:
        return [(r, c) for r in range(self.rows) for c in range(self.row_len(r))]

    def site(self, r: int, c: int) -> int:
        m = self.row_len(r)
        if not (0 <= c < m):
            raise ValueError("no qubit at (%d, %d)" % (r, c))
        return r * self.width + (c if r % 2 == 0 else m - 1 - c)

    def pattern_pairs(self, letter: str) -> List[Tuple[int, int]]:
        """Chain-site pairs of coupler pattern A/B (along a row) or C/D (between rows).

        A: (r,c)-(r,c+1), r+c even.  B: same, r+c odd.
        C: (r,c)-(r+1,c), r+c even.  D: same, r+c odd.
        Pairs are sorted by (site_i, site_j) with site_i < site_j.
        """
        parity = 0 if letter in "AC" else 1
        pairs = []
        for r, c in self.coords():
            if (r + c) % 2 != parity:
                continue
            if letter in "AB":
                if c + 1 < self.row_len(r):
                    pairs.append((self.site(r, c), self.site(r, c + 1)))
            else:
                if r + 1 < self.rows and c < self.row_len(r + 1):
                    pairs.append((self.site(r, c), self.site(r + 1, c)))
        pairs = [(min(a, b), max(a, b)) for a, b in pairs]
        return sorted(pairs)


def grid_from_shape(rows: int, cols: int) -> Grid:
    """A full rows x cols grid, read in snake order along its short side."""
    return Grid(n=rows * cols, width=min(rows, cols))


SEQUENCE = "ABCDCDAB"

Gate = Tuple[int, int, np.ndarray]


@dataclasses.dataclass
class Circuit:
    n: int
    layers: List[List[Gate]]
    label: str = ""

    @property
    def n_2q(self) -> int:
        return sum(1 for layer in self.layers for g in layer if g[1] >= 0)

    def layer_n_2q(self, d: int) -> int:
        return sum(1 for g in self.layers[d] if g[1] >= 0)


def random_circuit(grid: Grid, depth: int, seed: int, two_qubit: str = "haar",
                   sequence: str = SEQUENCE) -> Circuit:
    """Random circuit on ``grid``: per cycle, 1q layer then one coupler pattern.

    ``two_qubit`` is ``"haar"`` (Haar U(4)) or ``"fsim"`` (fSim with
    theta ~ U(0, pi/2), phi ~ U(0, pi), drawn per gate instance).
    """
    rng = np.random.default_rng(seed)
    coords = grid.coords()
    layers: List[List[Gate]] = []
    for d in range(depth):
        choice = rng.integers(0, 3, size=grid.n)
        layer: List[Gate] = []
        one_q = {}
        for (r, c), ch in zip(coords, choice):
            one_q[grid.site(r, c)] = ONE_QUBIT_SET[int(ch)]
        for s in sorted(one_q):
            layer.append((s, -1, one_q[s]))
        for (i, j) in grid.pattern_pairs(sequence[d % len(sequence)]):
            if two_qubit == "haar":
                u = haar_unitary_from_normals(rng.standard_normal(32))
            elif two_qubit == "fsim":
                theta = rng.uniform(0.0, np.pi / 2)
                phi = rng.uniform(0.0, np.pi)
                u = fsim(theta, phi)
            else:
                raise ValueError(two_qubit)
            layer.append((i, j, u))
        layers.append(layer)
    return Circuit(n=grid.n, layers=layers,
                   label="grid%dx%d_d%d_%s_s%d" % (grid.rows, grid.width, depth,
                                                  two_qubit, seed))


# ------------------------------------------------------ Sycamore layout ----
@dataclasses.dataclass
class SycamoreLayout:
    """The processor topology of the paper's Fig. 1: n_c columns holding n_b and n_b - 1
    qubits alternately (column 0 holds n_b).  Qubit (c, y) has column c and height y:
    y = 0, 2, .., 2(n_b - 1) in even columns and y = 1, 3, .., 2n_b - 3 in odd ones, so
    nearest neighbours are the diagonal pairs (c, y)-(c + 1, y +- 1).  Chain order is
    column by column, bottom to top (the order of the vertical groupings).

    Coupler classes, each a matching:
      A: (c, y)-(c+1, y+1), c even     B: (c, y)-(c+1, y+1), c odd
      C: (c, y)-(c+1, y-1), c even     D: (c, y)-(c+1, y-1), c odd
    A quarter turn of the lattice maps A -> C -> B -> D -> A, the letter map that takes
    the paper's Sequence I string to its Sequence II string.
    """
    n_b: int
    n_c: int

    def column_len(self, c: int) -> int:
        return self.n_b if c % 2 == 0 else self.n_b - 1

    @property
    def n(self) -> int:
        return sum(self.column_len(c) for c in range(self.n_c))

    def coords(self) -> List[Tuple[int, int]]:
        return [(c, 2 * r + (c % 2)) for c in range(self.n_c) for r in range(self.column_len(c))]

    def site(self, c: int, y: int) -> int:
        if not (0 <= c < self.n_c) or (y - c) % 2 != 0 or not (0 <= (y - c % 2) // 2 < self.column_len(c)):
            raise ValueError("no qubit at (%d, %d)" % (c, y))
        return sum(self.column_len(k) for k in range(c)) + (y - c % 2) // 2

    def has(self, c: int, y: int) -> bool:
        try:
            self.site(c, y)
            return True
        except ValueError:
            return False

    def pattern_pairs(self, letter: str) -> List[Tuple[int, int]]:
        """Chain-site pairs (i < j) of coupler class A, B, C or D."""
        parity = 0 if letter in "AC" else 1
        dy = 1 if letter in "AB" else -1
        pairs = []
        for c, y in self.coords():
            if c % 2 == parity and self.has(c + 1, y + dy):
                a, b = self.site(c, y), self.site(c + 1, y + dy)
                pairs.append((min(a, b), max(a, b)))
        return sorted(pairs)


def group_bond_profile(group_sizes: Sequence[int], chi: int) -> List[int]:
    """Per-bond caps of a grouping of consecutive chain sites into tensors (Sec. IV.A with
    r_tau > 1): chi on the bonds between groups, and on a bond inside a group the largest
    Schmidt rank any state can have there, 2^min(c, n - c), so that nothing inside a group is
    truncated.  Entry c is the bond between sites c - 1 and c (n + 1 entries)."""
    n = int(sum(group_sizes))
    if min(group_sizes) < 1:
        raise ValueError("groups must be non-empty")
    cuts = set(np.cumsum(group_sizes)[:-1].tolist())
    return [1] + [chi if c in cuts else 2 ** min(c, n - c) for c in range(1, n)] + [1]


def sycamore_column_groups(layout: "SycamoreLayout", columns: Sequence[int]) -> List[int]:
    """Group sizes (in chain order) of a vertical grouping of the Sycamore layout: group g
    holds columns[g] consecutive columns (the V groupings of Sec. V.C)."""
    if sum(columns) != layout.n_c:
        raise ValueError("the groups must cover every column")
    sizes, c = [], 0
    for k in columns:
        sizes.append(sum(layout.column_len(c + i) for i in range(k)))
        c += k
    return sizes


def sycamore_row_groups(layout: "SycamoreLayout", offset: int = 0):
    """A horizontal grouping of the Sycamore layout (the H groupings of Sec. V.C): qubits grouped
    by pairs of heights {2m + offset, 2m + 1 + offset} (offset 0 or 1; a lone height at an
    edge forms its own group).  Returns (order, sizes): order lists the column-major chain
    sites in the new chain order (group by group, each group by column then height), sizes the
    group sizes in that order."""
    if offset not in (0, 1):
        raise ValueError("offset must be 0 or 1")
    groups = {}
    for c, y in layout.coords():
        groups.setdefault((y + offset) // 2, []).append((c, y))
    order, sizes = [], []
    for key in sorted(groups):
        members = sorted(groups[key])
        order += [layout.site(c, y) for c, y in members]
        sizes.append(len(members))
    return order, sizes


def sycamore_diagonal_groups(layout: "SycamoreLayout", direction: str = "up"):
    """A diagonal grouping of the Sycamore layout (the D groupings of Sec. V.C): one group per
    diagonal line of qubits, y - c constant for direction "up" (the lines that couplers A and B
    follow, so the A and B layers stay inside the groups) and y + c constant for "down" (C and
    D).  Returns (order, sizes) as sycamore_row_groups: the column-major chain sites in the new
    chain order (group by group, each group by column) and the group sizes in that order."""
    if direction not in ("up", "down"):
        raise ValueError("direction must be 'up' or 'down'")
    groups = {}
    for c, y in layout.coords():
        groups.setdefault(y - c if direction == "up" else y + c, []).append((c, y))
    order, sizes = [], []
    for key in sorted(groups):
        members = sorted(groups[key])
        order += [layout.site(c, y) for c, y in members]
        sizes.append(len(members))
    return order, sizes


def relabel_circuit(circuit: Circuit, order: Sequence[int]) -> Circuit:
    """The same circuit on a new chain: site order[k] of the old chain becomes site k."""
    pos = {old: new for new, old in enumerate(order)}
    if sorted(pos) != list(range(circuit.n)):
        raise ValueError("order must be a permutation of the chain sites")
    layers = [[(pos[q0], pos[q1] if q1 >= 0 else -1, u) for q0, q1, u in layer] for layer in circuit.layers]
    return Circuit(n=circuit.n, layers=layers, label=circuit.label + "_relabelled")


# Sequence I is the supremacy pattern ABCD-CDAB; Sequence II is the same pattern turned by a
# quarter (CDBA-BACD).
SEQUENCE_I = "ABCDCDAB"
SEQUENCE_II = "CDBABACD"
FSIM_THETA, FSIM_PHI = 1.0, np.pi / 2     # the fixed fSim of the paper's Sequences I and II


def sycamore_circuit(layout: SycamoreLayout, depth: int, seed: int, sequence: str = "I",
                     two_qubit: str = "fsim") -> Circuit:
    """Sequence I or II on the Sycamore layout: per layer a random one-qubit gate from
    {sqrt X, sqrt Y, sqrt W} on every qubit, then a two-qubit gate on every coupler of the
    layer's class: fSim(1, pi/2) (``two_qubit="fsim"``, the paper's choice) or a Haar U(4)
    per coupler (``"haar"``, whose Schmidt spectra have no structural ties)."""
    pattern = {"I": SEQUENCE_I, "II": SEQUENCE_II}[sequence]
    if two_qubit not in ("fsim", "haar"):
        raise ValueError(two_qubit)
    rng = np.random.default_rng(seed)
    u2 = fsim(FSIM_THETA, FSIM_PHI)
    layers: List[List[Gate]] = []
    for d in range(depth):
        choice = rng.integers(0, 3, size=layout.n)
        layer: List[Gate] = [(s, -1, ONE_QUBIT_SET[int(choice[s])]) for s in range(layout.n)]
        for i, j in layout.pattern_pairs(pattern[d % len(pattern)]):
            layer.append((i, j, u2 if two_qubit == "fsim" else haar_unitary_from_normals(rng.standard_normal(32))))
        layers.append(layer)
    return Circuit(n=layout.n, layers=layers,
                   label="sycamore_nb%d_nc%d_seq%s_d%d_%s_s%d" % (layout.n_b, layout.n_c, sequence, depth,
                                                                 two_qubit, seed))


def random_brickwork(n: int, depth: int, seed: int) -> Circuit:
    """Nearest-neighbour chain brickwork of Haar gates with random 1q gates.

    Small-n helper (bond growth is slow and regular), used by the tests.
    """
    rng = np.random.default_rng(seed)
    layers = []
    for d in range(depth):
        choice = rng.integers(0, 3, size=n)
        layer: List[Gate] = [(s, -1, ONE_QUBIT_SET[int(choice[s])]) for s in range(n)]
        for i in range(d % 2, n - 1, 2):
            layer.append((i, i + 1, haar_unitary_from_normals(rng.standard_normal(32))))
        layers.append(layer)
    return Circuit(n=n, layers=layers, label="brick_n%d_d%d_s%d" % (n, depth, seed))


# ------------------------------------------------------------ workloads ----
def plain_fp64_workload(seed: int = 0) -> Circuit:
    """12 qubits on a 3x4 grid, depth 8, Haar 2q gates (chi = 64 is exact)."""
    return random_circuit(grid_from_shape(3, 4), 8, seed, "haar")


def grid36_workload(seed: int) -> Circuit:
    """36 qubits on a 6x6 grid, depth 14, Haar 2q gates."""
    return random_circuit(grid_from_shape(6, 6), 14, seed, "haar")


def sycamore_like_54_workload(seed: int = 0, depth: int = 20) -> Circuit:
    """54 qubits on a 6x9 grid (snake over width 6), fSim(theta, phi) 2q gates."""
    return random_circuit(grid_from_shape(9, 6), depth, seed, "fsim")


def sycamore_54_workload(seed: int = 0, depth: int = 20, sequence: str = "I") -> Circuit:
    """The paper's 54-qubit processor (n_b = 5, n_c = 12), Sequence I or II, depth 20."""
    return sycamore_circuit(SycamoreLayout(5, 12), depth, seed, sequence)


def batched_instances(count: int = 64, seed: int = 0):
    """Ragged instances: n ~ U{20..40}, depth ~ U{8..20}, chi from {32..512}, width ~ U{4,5,6}.

    Returns a list of ``(circuit, chi)``; instance i draws its gates from seed 1000+i.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(20, 41))
        depth = int(rng.integers(8, 21))
        chi = int(rng.choice([32, 64, 128, 256, 512]))
        width = int(rng.integers(4, 7))
        out.append((random_circuit(Grid(n, width), depth, 1000 + i, "haar"), chi))
    return out


# -------------------------------------------------------------- packing ----
GATE_DTYPE = np.dtype([("q0", "<i4"), ("q1", "<i4"), ("m", "<f8", (32,))], align=False)


def pack_layer(layer: Sequence[Gate]) -> np.ndarray:
    """Pack a layer into the C ABI gate record array (interleaved complex128)."""
    arr = np.zeros(len(layer), dtype=GATE_DTYPE)
    for idx, (q0, q1, u) in enumerate(layer):
        arr[idx]["q0"] = q0
        arr[idx]["q1"] = q1
        flat = np.asarray(u, dtype=np.complex128).reshape(-1)
        m = np.zeros(32)
        m[0:2 * flat.size:2] = flat.real
        m[1:2 * flat.size:2] = flat.imag
        arr[idx]["m"] = m
    return arr


def save_npz(path: str, circuit: Circuit) -> None:
    recs = [pack_layer(layer) for layer in circuit.layers]
    np.savez(path, n=circuit.n, n_layers=len(recs), label=circuit.label,
             **{"layer%d" % i: r for i, r in enumerate(recs)})


def load_npz(path: str) -> Circuit:
    z = np.load(path, allow_pickle=False)
    layers = []
    for i in range(int(z["n_layers"])):
        rec = z["layer%d" % i]
        layer = []
        for g in rec:
            m = g["m"][0::2] + 1j * g["m"][1::2]
            q0, q1 = int(g["q0"]), int(g["q1"])
            u = m[:4].reshape(2, 2) if q1 < 0 else m[:16].reshape(4, 4)
            layer.append((q0, q1, u))
        layers.append(layer)
    return Circuit(n=int(z["n"]), layers=layers, label=str(z["label"]))


def bits_to_index(bits: Sequence[int]) -> int:
    """Statevector index of a bitstring: site 0 is the most significant bit."""
    x = 0
    for b in bits:
        x = (x << 1) | int(b)
    return x


# ----------------------------------------------------------------- QAOA ----
HADAMARD = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)


def random_regular_graph(n: int, degree: int, seed: int, max_tries: int = 10000):
    """Random d-regular simple graph by the pairing (configuration) model with rejection."""
    if (n * degree) % 2:
        raise ValueError("n * degree must be even")
    rng = np.random.default_rng(seed)
    for _ in range(max_tries):
        stubs = np.repeat(np.arange(n), degree)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        edges = set()
        ok = True
        for a, b in pairs:
            a, b = int(a), int(b)
            if a == b or (min(a, b), max(a, b)) in edges:
                ok = False
                break
            edges.add((min(a, b), max(a, b)))
        if ok:
            return sorted(edges)
    raise RuntimeError("no simple regular graph found")


@dataclasses.dataclass
class QaoaCircuit:
    circuit: Circuit
    edges: List[Tuple[int, int]]
    final_position: List[int]      # chain site holding logical qubit q at the end


def qaoa_maxcut_swap_network(n: int, edges, gammas: Sequence[float], betas: Sequence[float]) -> QaoaCircuit:
    """QAOA MaxCut U = prod_k U_B(beta_k) U_C(gamma_k) on a chain (Sec. V.A, sequence III).

    U_C(gamma) = prod_E exp(-i gamma Z_u Z_v) is routed by a full odd-even
    transposition (SWAP) network of n brick layers: every pair of logical
    qubits is adjacent exactly once, and where the pair is a graph edge the
    SWAP is fused with exp(-i gamma ZZ).  The network reverses the logical
    order; the next cost layer runs on the reversed order.  U_B(beta) =
    prod exp(-i beta X) = RX(2 beta) on every qubit, placed as one-qubit gates
    of the next brick layer (or of a final one-qubit layer).  The initial
    |+>^n is prepared by Hadamards in the first layer.
    """
    edge_set = {(min(a, b), max(a, b)) for a, b in edges}
    pos_of = list(range(n))        # logical -> site
    at = list(range(n))            # site -> logical
    layers: List[List[Gate]] = []
    pending_1q = {s: HADAMARD for s in range(n)}
    for gamma, beta in zip(gammas, betas):
        zz_swap = SWAP @ zz_phase(gamma)
        for d in range(n):
            layer: List[Gate] = [(s, -1, u) for s, u in sorted(pending_1q.items())]
            pending_1q = {}
            for i in range(d % 2, n - 1, 2):
                a, b = at[i], at[i + 1]
                u = zz_swap if (min(a, b), max(a, b)) in edge_set else SWAP
                layer.append((i, i + 1, u))
                at[i], at[i + 1] = b, a
                pos_of[a], pos_of[b] = i + 1, i
            layers.append(layer)
        mixer = rx(2.0 * beta)
        pending_1q = {s: mixer for s in range(n)}
    layers.append([(s, -1, u) for s, u in sorted(pending_1q.items())])
    return QaoaCircuit(circuit=Circuit(n=n, layers=layers, label="qaoa_n%d_p%d" % (n, len(gammas))),
                       edges=sorted(edge_set), final_position=pos_of)


def qaoa_parameter_sets(count: int, p: int, seed: int = 0):
    """(gamma, beta) sets: gamma ~ U[0, pi], beta ~ U[0, pi/2], one pair per QAOA layer."""
    rng = np.random.default_rng(seed)
    return [(rng.uniform(0, np.pi, p), rng.uniform(0, np.pi / 2, p)) for _ in range(count)]


def maxcut_expectation_from_zz(edges, final_position, zz) -> float:
    """<C> = sum_E (1 - <Z_u Z_v>)/2, zz(i, j) giving <Z_i Z_j> on chain sites."""
    return float(sum(0.5 * (1.0 - zz(final_position[u], final_position[v])) for u, v in edges))


def metropolis_draws(n: int, n_steps: int, seed: int):
    """Seeded random inputs of a Metropolis chain over bitstrings: per step a uniformly random
    proposed bitstring (n bits, site order) and one uniform number in [0, 1) for the acceptance.
    Both the oracle and the library's sampler take these as inputs."""
    rng = np.random.default_rng(seed)
    proposals = rng.integers(0, 2, size=(n_steps, n)).astype(np.uint8)
    uniforms = rng.random(n_steps)
    return proposals, uniforms
