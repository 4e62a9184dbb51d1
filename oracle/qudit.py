"""NumPy complex128 oracle for generalized qudit gates on a mixed-radix register.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's CPU-baseline
leg; never by the product library.

Conventions (readings of the paper, each stated once here):
  * Register (Sec. 2.2 and Sec. 3.3, Eq. (3)): the state of qudits with dimensions d_0..d_{n-1} is
    the Kronecker product |psi_0> (x) ... (x) |psi_{n-1}>, so it has D = prod d_i entries and, in the
    Kronecker order of Eq. (3), qudit 0 is the most significant digit of the flat index
    (stride s_i = prod_{j>i} d_j). The example output of Sec. 3.9 labels q0 = 1, q1 = 2 as |120>,
    which agrees. (Sec. 3.2 calls the first qudit the LSB; the equation and the example win.)
  * A gate on targets (t_0, ..., t_{k-1}) has a (d_T x d_T) unitary, d_T = prod d_{t_j}, whose
    row/column index takes t_0 as its most significant digit; this is the block layout of the
    generalized CNOT of Sec. 2.1, whose blocks are indexed by the control listed first.
  * Controls: a gate acts only on basis states whose control digits equal the given control values
    (Sec. 2.1: the INCREMENT and multi-controlled Toffoli act when every control is d-1; here the
    value is explicit, defaulting to d_c - 1 in the helpers).
  * omega = exp(2 pi i / d) (Sec. 2.1, phase-shift gate). omega^m is evaluated with m reduced mod d
    first; quarter turns (4 m / d integral) take their exact values.
  * F_d carries the factor 1 / sqrt(d) computed as 1.0 / sqrt(d) (Sec. 2.1, generalized Hadamard).
"""
from __future__ import annotations

import math
from typing import Iterable, Sequence

import numpy as np

__all__ = [
    "register_size", "strides", "digits_of", "index_of",
    "omega_power", "x_gate", "z_gate", "f_gate", "identity_gate", "gate_unitary",
    "basis_state", "initial_state",
    "apply_gate", "apply_gate_at", "gate_operator", "kron_operator",
    "run_circuit", "run_circuit_operator",
    "probabilities", "norm2", "compare", "fused_block",
]


# ----------------------------------------------------------------------------- register (Sec. 2.2)
def register_size(dims: Sequence[int]) -> int:
    """D = product of the qudit dimensions (Sec. 2.2: dims (2, 3, 4) give 24 entries)."""
    D = 1
    for d in dims:
        D *= int(d)
    return D


def strides(dims: Sequence[int]) -> list:
    """Big-endian mixed-radix strides: s_i = prod_{j > i} d_j, s_{n-1} = 1."""
    s = [1] * len(dims)
    for i in range(len(dims) - 2, -1, -1):
        s[i] = s[i + 1] * int(dims[i + 1])
    return s


def digits_of(x: int, dims: Sequence[int]) -> list:
    """Digits of flat index x, qudit 0 first."""
    out = [0] * len(dims)
    for i in range(len(dims) - 1, -1, -1):
        out[i] = x % dims[i]
        x //= dims[i]
    return out


def index_of(digs: Sequence[int], dims: Sequence[int]) -> int:
    x = 0
    for dgt, d in zip(digs, dims):
        x = x * d + dgt
    return x


# ----------------------------------------------------------------------------- gates (Sec. 2.1)
def omega_power(m: int, d: int) -> complex:
    """omega^m with omega = exp(2 pi i / d); exponent reduced mod d, exact quarter turns."""
    m %= d
    if (4 * m) % d == 0:
        return (1 + 0j, 1j, -1 + 0j, -1j)[(4 * m) // d]
    ang = 2.0 * math.pi * m / d
    return complex(math.cos(ang), math.sin(ang))


def x_gate(d: int, a: int = 1) -> np.ndarray:
    """Generalized NOT X^d_{+a}: |x> -> |(x + a) mod d>, 1 <= a <= d - 1 (Sec. 2.1)."""
    if not 1 <= a <= d - 1:
        raise ValueError("shift must satisfy 1 <= a <= d-1")
    U = np.zeros((d, d), dtype=np.complex128)
    for x in range(d):
        U[(x + a) % d, x] = 1.0
    return U


def z_gate(d: int) -> np.ndarray:
    """Generalized phase-shift Z_d = diag(1, omega, ..., omega^{d-1}) (Sec. 2.1)."""
    return np.diag([omega_power(x, d) for x in range(d)]).astype(np.complex128)


def f_gate(d: int) -> np.ndarray:
    """Generalized Hadamard F_d = (1 / sqrt d) [omega^{jk}] (Sec. 2.1)."""
    s = 1.0 / math.sqrt(d)
    U = np.empty((d, d), dtype=np.complex128)
    for j in range(d):
        for k in range(d):
            w = omega_power(j * k, d)
            U[j, k] = complex(w.real * s, w.imag * s)
    return U


def identity_gate(d: int) -> np.ndarray:
    return np.eye(d, dtype=np.complex128)


def gate_unitary(gate, dims: Sequence[int]) -> np.ndarray:
    """Unitary of a gate record (attributes kind, targets, a, U) on a register with dims.

    The unitary is built from the dimension of the acting wire (Sec. 3.4)."""
    if gate.kind == "U":
        return np.asarray(gate.U, dtype=np.complex128)
    if len(gate.targets) != 1:
        raise ValueError("named gates act on one target")
    d = int(dims[gate.targets[0]])
    if gate.kind == "X":
        return x_gate(d, gate.a)
    if gate.kind == "Z":
        return z_gate(d)
    if gate.kind == "F":
        return f_gate(d)
    raise ValueError(f"unknown gate kind {gate.kind!r}")


# ----------------------------------------------------------------------------- states (Sec. 3.3)
def basis_state(dims: Sequence[int], values: Iterable[int] | None = None) -> np.ndarray:
    """Kronecker product of one basis vector per wire (Sec. 3.2 init_states, Sec. 3.3 Eq. (3))."""
    vals = [0] * len(dims) if values is None else list(values)
    psi = np.ones(1, dtype=np.complex128)
    for v, d in zip(vals, dims):
        e = np.zeros(int(d), dtype=np.complex128)
        e[int(v)] = 1.0
        psi = np.kron(psi, e)
    return psi


def initial_state(circuit) -> np.ndarray:
    if getattr(circuit, "init_amps", None) is not None:
        return np.array(circuit.init_amps, dtype=np.complex128, copy=True)
    return basis_state(circuit.dims, getattr(circuit, "init_basis", None))


# ----------------------------------------------------------------------------- O1: contraction
def _check_gate(dims, targets, controls, cvals, U):
    n = len(dims)
    T, C = list(targets), list(controls)
    if len(set(T)) != len(T) or len(set(C)) != len(C) or set(T) & set(C):
        raise ValueError("targets must be distinct and disjoint from controls")
    if any(not 0 <= q < n for q in T + C):
        raise ValueError("qudit index out of range")
    if len(cvals) != len(C) or any(not 0 <= v < dims[c] for c, v in zip(C, cvals)):
        raise ValueError("bad control value")
    dT = 1
    for t in T:
        dT *= int(dims[t])
    U = np.asarray(U, dtype=np.complex128)
    if U.shape != (dT, dT):
        raise ValueError(f"U must be {dT}x{dT}")
    return T, C, dT, U


def apply_gate(psi: np.ndarray, dims: Sequence[int], targets, controls, cvals, U) -> np.ndarray:
    """O1: apply one (controlled) k-qudit gate by tensor contraction; returns a new array.

    Computes psi_out = (I (x) U (x) I) psi restricted to the control-matching block, i.e. the
    Moment's Kronecker product applied to the state (Sec. 3.5-3.6) without forming it."""
    dims = tuple(int(d) for d in dims)
    T, C, dT, U = _check_gate(dims, targets, controls, cvals, U)
    out = np.array(psi, dtype=np.complex128, copy=True)
    view = out.reshape(dims)                          # axis i <-> qudit i, C order: big-endian
    sel = [slice(None)] * len(dims)
    for c, v in zip(C, cvals):
        sel[c] = int(v)
    sub = view[tuple(sel)]                            # control axes fixed: a view
    remaining = [q for q in range(len(dims)) if q not in C]
    ax = [remaining.index(t) for t in T]
    front = list(range(len(T)))
    moved = np.moveaxis(sub, ax, front)               # targets first, in listed order
    shape = moved.shape
    mixed = U @ moved.reshape(dT, -1)                 # rows: target digits, t_0 most significant
    view[tuple(sel)] = np.moveaxis(mixed.reshape(shape), front, ax)
    return out


def apply_gate_at(psi_in: np.ndarray, dims: Sequence[int], targets, controls, cvals, U,
                  indices: Iterable[int]) -> np.ndarray:
    """Output amplitudes of one gate at the given flat indices, computed one by one from psi_in."""
    dims = tuple(int(d) for d in dims)
    T, C, dT, U = _check_gate(dims, targets, controls, cvals, U)
    tdims = [dims[t] for t in T]
    res = []
    for i in indices:
        dg = digits_of(int(i), dims)
        if any(dg[c] != v for c, v in zip(C, cvals)):
            res.append(complex(psi_in[int(i)]))
            continue
        row = index_of([dg[t] for t in T], tdims)
        acc = 0j
        for col in range(dT):
            cd = digits_of(col, tdims)
            src = list(dg)
            for t, v in zip(T, cd):
                src[t] = v
            acc += U[row, col] * complex(psi_in[index_of(src, dims)])
        res.append(acc)
    return np.array(res, dtype=np.complex128)


# ----------------------------------------------------------------------------- O2: brute force
def gate_operator(dims: Sequence[int], targets, controls, cvals, U) -> np.ndarray:
    """O2: the full D x D operator of one gate, built by enumerating basis states:
    <y|G|x> = U[loc(y_T), loc(x_T)] delta(y_rest, x_rest) if x_C = v, else delta(y, x)."""
    dims = tuple(int(d) for d in dims)
    T, C, dT, U = _check_gate(dims, targets, controls, cvals, U)
    D = register_size(dims)
    tdims = [dims[t] for t in T]
    M = np.zeros((D, D), dtype=np.complex128)
    for x in range(D):
        xd = digits_of(x, dims)
        if any(xd[c] != v for c, v in zip(C, cvals)):
            M[x, x] = 1.0
            continue
        col = index_of([xd[t] for t in T], tdims)
        for row in range(dT):
            yd = list(xd)
            for t, v in zip(T, digits_of(row, tdims)):
                yd[t] = v
            M[index_of(yd, dims), x] = U[row, col]
    return M


def kron_operator(dims: Sequence[int], target: int, U) -> np.ndarray:
    """The paper's Moment operator for one single-qudit gate: the Kronecker product of the slots,
    identities everywhere except the acting wire (Sec. 3.5, Eq. (3) order)."""
    M = np.ones((1, 1), dtype=np.complex128)
    for i, d in enumerate(dims):
        M = np.kron(M, np.asarray(U, dtype=np.complex128) if i == target else identity_gate(int(d)))
    return M


def run_circuit(circuit, psi0: np.ndarray | None = None) -> np.ndarray:
    """O1 over a whole circuit, gates in order."""
    dims = tuple(circuit.dims)
    psi = initial_state(circuit) if psi0 is None else np.array(psi0, dtype=np.complex128, copy=True)
    for g in circuit.gates:
        psi = apply_gate(psi, dims, g.targets, g.controls, g.cvals, gate_unitary(g, dims))
    return psi


def run_circuit_operator(circuit, psi0: np.ndarray | None = None) -> np.ndarray:
    """O2 over a whole circuit, as the paper executes (Sec. 3.6): the Moments are popped in
    reverse, each Moment's operator is formed, the operators are multiplied together and one
    matrix-vector product with the initial state finishes. Tiny registers only (D <= ~3000)."""
    dims = tuple(circuit.dims)
    psi = initial_state(circuit) if psi0 is None else np.array(psi0, dtype=np.complex128, copy=True)

    def op(g):
        U = gate_unitary(g, dims)
        if len(g.targets) == 1 and not g.controls:
            return kron_operator(dims, g.targets[0], U)
        return gate_operator(dims, g.targets, g.controls, g.cvals, U)

    if not circuit.gates:
        return psi
    acc = op(circuit.gates[-1])
    for g in reversed(circuit.gates[:-1]):
        acc = acc @ op(g)
    return acc @ psi


# ----------------------------------------------------------------------------- output (Sec. 3.8)
def probabilities(psi: np.ndarray) -> np.ndarray:
    """|alpha_x|^2 per basis state in FP64 (Sec. 3.8 OutputMethod probability; Eq. (1) norm)."""
    p = np.asarray(psi, dtype=np.complex128)
    return p.real * p.real + p.imag * p.imag


def norm2(psi: np.ndarray) -> float:
    return float(np.sum(probabilities(psi)))


def compare(psi_ref: np.ndarray, psi: np.ndarray):
    """(max |psi - psi_ref|, 1 - |<psi_ref|psi>|^2, | ||psi||^2 - 1 |) in FP64."""
    a = np.asarray(psi_ref, dtype=np.complex128)
    b = np.asarray(psi, dtype=np.complex128)
    max_abs = float(np.max(np.abs(b - a))) if a.size else 0.0
    inner = complex(np.vdot(a, b))
    fid_loss = 1.0 - (inner.real * inner.real + inner.imag * inner.imag)
    drift = abs(norm2(b) - 1.0)
    return max_abs, fid_loss, drift


# ----------------------------------------------------------------------------- fusion check
def fused_block(dims: Sequence[int], window: Sequence[int], gates) -> np.ndarray:
    """Product (later gates on the left) of the gates' operators over the sub-register `window`
    (qudit indices of the full register, the first most significant). Every gate's targets and
    controls must lie inside the window. The bounded-width counterpart of the paper's operator
    products (Sec. 3.6)."""
    window = list(window)
    wdims = [int(dims[q]) for q in window]
    pos = {q: i for i, q in enumerate(window)}
    B = register_size(wdims)
    M = np.eye(B, dtype=np.complex128)
    for g in gates:
        U = gate_unitary(g, dims)
        E = gate_operator(wdims, [pos[t] for t in g.targets], [pos[c] for c in g.controls],
                          list(g.cvals), U)
        M = E @ M
    return M
