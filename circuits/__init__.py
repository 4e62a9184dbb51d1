"""Seeded synthetic qudit circuits: the input data shared by the oracle and the HIP path.

This module only *describes* circuits. It draws random numbers (wire orders, gate choices,
Haar-random unitaries, random initial superpositions) and writes them down as plain data; it applies
no gate and evaluates nothing the simulator computes. Named gates of the paper's gate set
(Sec. 2.1: generalized NOT X_{+a}, phase-shift Z_d, generalized Hadamard F_d and the controlled
INCREMENT) are emitted *symbolically* (a kind plus parameters) so that each consumer builds their
matrices on its own. Unitaries that are not in the paper's gate set (Haar-random gates, the qudit
QFT's controlled phases and qudit swaps) are emitted as explicit complex128 matrices.

Conventions shared by every consumer:
  * flat index is big-endian mixed radix: qudit 0 is the most significant digit;
  * a multi-qudit unitary's row/column index takes its first listed target as the most
    significant digit.

Workload shapes follow the paper's benchmark mix (qubit-qutrit registers, controlled shifts,
many small circuits, a 20-qutrit register) without reproducing any benchmark circuit.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Gate", "Circuit", "haar_unitary", "random_basis_superposition",
    "config0", "config1", "config1_shrink", "config2", "config3", "config4",
    "random_gate", "random_circuit", "permutation_circuit", "diagonal_circuit", "seeded_rng",
    "qubit_hadamard_on_qutrit", "ToffoliNetwork", "toffoli_network",
]


def seeded_rng(seed: int) -> np.random.Generator:
    """NumPy PCG64 generator; every workload is seeded as 1000 + config number."""
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Gate:
    """One gate as data.

    kind: "X" (shift by ``a``), "Z", "F" (named, single target) or "U" (explicit ``U``).
    A named "X" with controls is the paper's generalized CNOT / multi-controlled Toffoli.
    ``U`` (kind "U" only) is a complex128 (d_T, d_T) array over the targets in listed order.
    """
    kind: str
    targets: tuple
    controls: tuple = ()
    cvals: tuple = ()
    a: int = 0
    U: Optional[np.ndarray] = None
    tag: str = ""

    def qudits(self):
        return tuple(self.targets) + tuple(self.controls)


@dataclass
class Circuit:
    dims: tuple
    gates: List[Gate] = field(default_factory=list)
    init_basis: Optional[tuple] = None        # digits of the initial basis state, default |0...0>
    init_amps: Optional[np.ndarray] = None    # explicit complex128 initial state (overrides basis)
    name: str = ""

    @property
    def D(self) -> int:
        return int(np.prod(np.asarray(self.dims, dtype=np.int64)))


# --------------------------------------------------------------------------------------------
# random unitaries and states (inputs, not method arithmetic)
# --------------------------------------------------------------------------------------------
def haar_unitary(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random U(d): QR of a complex Ginibre matrix with the phases of R's diagonal divided
    out (Mezzadri, "How to generate random matrices from the classical compact groups", 2007)."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    diag = np.diagonal(r)
    ph = diag / np.abs(diag)
    return np.ascontiguousarray(q * ph[np.newaxis, :]).astype(np.complex128)


def random_basis_superposition(D: int, K: int, rng: np.random.Generator) -> np.ndarray:
    """K distinct basis indices drawn uniformly, i.i.d. complex Gaussian weights, normalised."""
    idx = rng.choice(D, size=min(K, D), replace=False)
    w = rng.standard_normal(len(idx)) + 1j * rng.standard_normal(len(idx))
    w /= math.sqrt(float(np.sum(np.abs(w) ** 2)))
    psi = np.zeros(D, dtype=np.complex128)
    psi[idx] = w
    return psi


# --------------------------------------------------------------------------------------------
# gate samplers
# --------------------------------------------------------------------------------------------
def random_gate(dims: Sequence[int], rng: np.random.Generator, kinds=("X", "Z", "F", "CX", "H1"),
                cval_top: bool = True) -> Gate:
    """One gate from the paper's set, generalised to each wire's dimension.

    kinds: "X" = X_{+1}; "Z"; "F"; "CX" = generalized CNOT with shift +1 and control value
    d_c - 1 (or a uniform control value if ``cval_top`` is False); "H1" = Haar d x d.
    """
    n = len(dims)
    kind = kinds[int(rng.integers(len(kinds)))]
    if kind == "CX" and n < 2:
        kind = "X"
    if kind == "CX":
        t = int(rng.integers(n))
        c = int(rng.integers(n - 1))
        c = c + 1 if c >= t else c
        v = dims[c] - 1 if cval_top else int(rng.integers(dims[c]))
        return Gate("X", (t,), (c,), (v,), a=1)
    t = int(rng.integers(n))
    if kind == "X":
        return Gate("X", (t,), a=1)
    if kind in ("Z", "F"):
        return Gate(kind, (t,))
    if kind == "H1":
        return Gate("U", (t,), U=haar_unitary(dims[t], rng), tag="haar")
    raise ValueError(kind)


def random_circuit(dims: Sequence[int], ngates: int, rng: np.random.Generator,
                   max_targets: int = 2, max_controls: int = 2, max_dT: int = 16) -> Circuit:
    """General random circuit for parity tests: named gates, controlled named gates and Haar
    unitaries on 1..max_targets distinct (not necessarily adjacent) targets with 0..max_controls
    controls carrying uniform control values."""
    n = len(dims)
    gates = []
    for _ in range(ngates):
        r = rng.random()
        perm = rng.permutation(n)
        if r < 0.45:
            k = int(rng.integers(1, max_targets + 1))
            k = min(k, n)
            tg = [int(q) for q in perm[:k]]
            while int(np.prod([dims[q] for q in tg])) > max_dT and len(tg) > 1:
                tg.pop()
            rest = [int(q) for q in perm[len(tg):]]
            m = int(rng.integers(0, min(max_controls, len(rest)) + 1))
            cs = rest[:m]
            cv = [int(rng.integers(dims[c])) for c in cs]
            dT = int(np.prod([dims[q] for q in tg]))
            gates.append(Gate("U", tuple(tg), tuple(cs), tuple(cv), U=haar_unitary(dT, rng), tag="haar"))
        else:
            t = int(perm[0])
            kind = ("X", "Z", "F")[int(rng.integers(3))]
            rest = [int(q) for q in perm[1:]]
            m = int(rng.integers(0, min(max_controls, len(rest)) + 1))
            cs = rest[:m]
            cv = [int(rng.integers(dims[c])) for c in cs]
            a = int(rng.integers(1, dims[t])) if kind == "X" else 0
            gates.append(Gate(kind, (t,), tuple(cs), tuple(cv), a=a))
    return Circuit(tuple(int(d) for d in dims), gates, name="random")


def permutation_circuit(dims: Sequence[int], ngates: int, rng: np.random.Generator) -> Circuit:
    """Only X_{+a} / controlled X_{+a}: maps a basis state to one basis state."""
    n = len(dims)
    gates = []
    for _ in range(ngates):
        perm = rng.permutation(n)
        t = int(perm[0])
        m = int(rng.integers(0, min(2, n - 1) + 1))
        cs = [int(q) for q in perm[1:1 + m]]
        cv = [int(rng.integers(dims[c])) for c in cs]
        gates.append(Gate("X", (t,), tuple(cs), tuple(cv), a=int(rng.integers(1, dims[t]))))
    return Circuit(tuple(int(d) for d in dims), gates, name="permutation")


def diagonal_circuit(dims: Sequence[int], ngates: int, rng: np.random.Generator) -> Circuit:
    """Only Z_d and controlled Z_d gates."""
    n = len(dims)
    gates = []
    for _ in range(ngates):
        perm = rng.permutation(n)
        t = int(perm[0])
        m = int(rng.integers(0, min(2, n - 1) + 1))
        cs = [int(q) for q in perm[1:1 + m]]
        cv = [int(rng.integers(dims[c])) for c in cs]
        gates.append(Gate("Z", (t,), tuple(cs), tuple(cv)))
    return Circuit(tuple(int(d) for d in dims), gates, name="diagonal")


# --------------------------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------------------------
def config0() -> Circuit:
    """6 qutrits (D = 729), |0..0>, 40 gates uniform over {X+1, Z_3, F_3, CX(+1, control value 2)}."""
    rng = seeded_rng(1000)
    dims = (3,) * 6
    gates = [random_gate(dims, rng, kinds=("X", "Z", "F", "CX")) for _ in range(40)]
    return Circuit(dims, gates, name="cfg0-6qutrits")


def _hybrid_gates(dims, ngates, rng):
    n = len(dims)
    gates = []
    for _ in range(ngates):
        if rng.random() < 0.5:
            t = int(rng.integers(n))
            gates.append(Gate("U", (t,), U=haar_unitary(dims[t], rng), tag="haar"))
        else:
            t = int(rng.integers(n))
            c = int(rng.integers(n - 1))
            c = c + 1 if c >= t else c
            v = int(rng.integers(dims[c]))
            a = int(rng.integers(1, dims[t]))        # a ~ U[1, d_t - 1]
            gates.append(Gate("X", (t,), (c,), (v,), a=a))
    return gates


def config1(ngates: int = 500) -> Circuit:
    """Hybrid register: seeded shuffle of 10 qubits + 8 qutrits + 2 ququarts
    (D = 2^10 * 3^8 * 4^2 = 107,495,424), 500 gates: Haar d x d on a uniform qudit (p = 1/2) or a
    controlled shift on a uniform ordered pair with a uniform control value."""
    rng = seeded_rng(1001)
    dims = [2] * 10 + [3] * 8 + [4] * 2
    dims = tuple(int(d) for d in rng.permutation(dims))
    return Circuit(dims, _hybrid_gates(dims, ngates, rng), name="cfg1-hybrid-20q")


def config1_shrink(ngates: int = 500) -> Circuit:
    """10-qudit shrink of the same mix: 5 qubits + 4 qutrits + 1 ququart (D = 10,368)."""
    rng = seeded_rng(1001)
    dims = [2] * 5 + [3] * 4 + [4] * 1
    dims = tuple(int(d) for d in rng.permutation(dims))
    return Circuit(dims, _hybrid_gates(dims, ngates, rng), name="cfg1-shrink-10q")


def qudit_qft_gates(d: int, n: int) -> List[Gate]:
    """Qudit QFT on n qudits of dimension d (big-endian): for j = 0..n-1 apply F_d on qudit j,
    then for every k > j the controlled phase diag exp(2 pi i x_j x_k / d^(k-j+1)) on (j, k);
    finish with the qudit reversal as floor(n/2) swaps (d^2 x d^2 permutations)."""
    gates: List[Gate] = []
    dd = d * d
    for j in range(n):
        gates.append(Gate("F", (j,)))
        for k in range(j + 1, n):
            den = float(d) ** (k - j + 1)
            ph = np.empty(dd, dtype=np.complex128)
            for xj in range(d):
                for xk in range(d):
                    ang = 2.0 * math.pi * (xj * xk) / den
                    ph[xj * d + xk] = complex(math.cos(ang), math.sin(ang))
            gates.append(Gate("U", (j, k), U=np.diag(ph), tag="cphase"))
    sw = np.zeros((dd, dd), dtype=np.complex128)
    for x in range(d):
        for y in range(d):
            sw[y * d + x, x * d + y] = 1.0
    for j in range(n // 2):
        gates.append(Gate("U", (j, n - 1 - j), U=sw.copy(), tag="swap"))
    return gates


def config2(n: int = 14, K: int = 256) -> Circuit:
    """Qudit QFT on n ququarts (n = 14: D = 268,435,456) from a seeded random superposition of
    K = 256 basis states."""
    rng = seeded_rng(1002)
    dims = (4,) * n
    D = 4 ** n
    psi = random_basis_superposition(D, K, rng)
    return Circuit(dims, qudit_qft_gates(4, n), init_amps=psi, name=f"cfg2-qft-{n}ququarts")


def config3(n: int = 20, layers: int = 30) -> Circuit:
    """n qutrits (n = 20: D = 3,486,784,401), `layers` brickwork layers of Haar 9x9 gates:
    even layers on (0,1),(2,3),..., odd layers on (1,2),(3,4),..."""
    rng = seeded_rng(1003)
    dims = (3,) * n
    gates = []
    for l in range(layers):
        start = 0 if l % 2 == 0 else 1
        for q in range(start, n - 1, 2):
            gates.append(Gate("U", (q, q + 1), U=haar_unitary(9, rng), tag="haar"))
    return Circuit(dims, gates, name=f"cfg3-brickwork-{n}qutrits")


def _batch_dims(rng, lo=1e3, hi=1e6):
    logD = rng.uniform(math.log(lo), math.log(hi))
    w = rng.dirichlet((1.0, 1.0, 1.0))
    a = int(round(w[0] * logD / math.log(2)))
    b = int(round(w[1] * logD / math.log(3)))
    c = int(round(w[2] * logD / math.log(4)))
    dims = [2] * a + [3] * b + [4] * c
    D = lambda ds: int(np.prod(ds)) if ds else 1
    while D(dims) < lo:
        dims.append(2)
    while D(dims) > hi:                      # drop the largest radix present
        dims.remove(max(dims))
    while D(dims) < lo:                      # cannot overshoot: D < lo here and 2 * lo < hi
        dims.append(2)
    order = rng.permutation(len(dims))
    return tuple(int(dims[i]) for i in order)


def config4(nc: int = 4096, ngates: int = 100, seed: int = 1004) -> List[Circuit]:
    """nc independent circuits over uneven registers 2^a 3^b 4^c, total dimension log-uniform in
    [1e3, 1e6]; each has `ngates` gates from {X+1, Z, F, CX(+1, v = d_c - 1), Haar d x d}."""
    rng = seeded_rng(seed)
    out = []
    for i in range(nc):
        dims = _batch_dims(rng)
        gates = [random_gate(dims, rng, kinds=("X", "Z", "F", "CX", "H1")) for _ in range(ngates)]
        out.append(Circuit(dims, gates, name=f"cfg4-{i}"))
    return out


# --------------------------------------------------------------------------------------------
# permutation-heavy workload for the sparse state
# --------------------------------------------------------------------------------------------
def qubit_hadamard_on_qutrit() -> np.ndarray:
    """3x3 unitary acting as the Hadamard on levels {0, 1} of a qutrit and fixing level 2 (an
    explicit gate, so each consumer applies it as given)."""
    c = 1.0 / math.sqrt(2.0)
    return np.array([[c, c, 0.0], [c, -c, 0.0], [0.0, 0.0, 1.0]], dtype=np.complex128)


@dataclass
class ToffoliNetwork:
    """A reversible Toffoli network on qubit wires plus qutrit wires that carry logical bits and
    serve as the intermediate-level control of each Toffoli (the paper's multiplier and RevLib
    circuits, Sec. 3.4 and 6, decomposed through intermediate qutrits).

    dims: qubits first, then qutrits. inputs: the superposition-preparing layer (F on the first
    n_in qubits, the embedded Hadamard on every qutrit), so 2^(n_in + n_qutrits) basis states are
    present. network: named X gates with 0, 1 or 2 controls, all control values 1 and every target
    a qubit; a 2-control gate has a qutrit as its second control (so it has a free level)."""
    dims: tuple
    inputs: List[Gate]
    network: List[Gate]


def toffoli_network(n_qubits: int, n_qutrits: int, n_in: int, ngates: int, rng: np.random.Generator,
                    p_toffoli: float = 0.5, p_cx: float = 0.3) -> ToffoliNetwork:
    dims = (2,) * n_qubits + (3,) * n_qutrits
    qubits = list(range(n_qubits))
    qutrits = list(range(n_qubits, n_qubits + n_qutrits))
    h3 = qubit_hadamard_on_qutrit()
    inputs = [Gate("F", (q,)) for q in range(n_in)] + [Gate("U", (q,), U=h3, tag="h01") for q in qutrits]
    net = []
    for _ in range(ngates):
        r = rng.random()
        t = int(rng.choice(qubits))
        if r < p_toffoli and qutrits:
            c2 = int(rng.choice(qutrits))
            c1 = int(rng.choice([q for q in range(len(dims)) if q not in (t, c2)]))
            net.append(Gate("X", (t,), (c1, c2), (1, 1), a=1))
        elif r < p_toffoli + p_cx:
            c = int(rng.choice([q for q in range(len(dims)) if q != t]))
            net.append(Gate("X", (t,), (c,), (1,), a=1))
        else:
            net.append(Gate("X", (t,), a=1))
    return ToffoliNetwork(dims, inputs, net)
