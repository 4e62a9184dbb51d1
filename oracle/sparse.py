"""Oracle for the sparse state: the list of a state's non-zero amplitudes, updated gate by gate.
TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU-baseline leg).

What the paper fixes (Sec. 3.3 and the SparseBackend of Sec. 3.7): a state is stored in a
compressed sparse column, i.e. only its non-zero amplitudes and their flat indices are kept, and
the operator products skip zero elements. The state reached is the same vector as the dense
simulation's (oracle.qudit), so the definition of every gate is the one written there:
<y|G|x> = U[loc(y_T), loc(x_T)] when the control digits of x hold the control values and the other
digits agree, identity on the rest.

Readings (each shared with the library and stated in its header):
  * an index is present exactly when its amplitude is not exactly zero: a gate output whose real
    and imaginary parts are both exactly 0.0 is dropped (sparse matrix products store no exact
    zeros). Entries moved by a monomial gate are never dropped;
  * a gate is *monomial* when every column and every row of U holds exactly one entry that is not
    exactly zero (shifts, generalized CNOTs, Z_d, controlled phases, qudit swaps), so that distinct
    indices stay distinct; it maps each matching entry
    to one entry: column loc goes to the row r holding that column's entry and the amplitude is
    multiplied by U[r, loc], except that a multiplier of exactly 1 leaves it untouched. Any other
    gate is *dense*: the matching entries that share every non-target digit form a slice, and the
    slice's d_T outputs are U times the slice's d_T inputs (absent inputs are zero);
  * arithmetic: a complex product u*x is formed as (ur*xr - ui*xi, ur*xi + ui*xr), each real
    operation rounded on its own (no fused multiply-add), and a dense output is the sum over
    columns j = 0, 1, .., d_T - 1 in that order starting from +0.0. This fixes every bit of the
    result, and so every drop decision.

The state is a pair of arrays: flat indices (int64, distinct) and amplitudes (complex128), in
increasing index, the order of a compressed sparse column (Sec. 3.3). A library may keep its list
in another order; the entries themselves are unique.
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np

from .qudit import gate_unitary, initial_state, register_size, strides

__all__ = ["from_dense", "to_dense", "basis", "gate_class", "apply_gate", "run_circuit", "norm2"]


def from_dense(psi: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Non-zero entries of a dense state, in increasing index (the compressed column's order)."""
    psi = np.asarray(psi, dtype=np.complex128)
    idx = np.flatnonzero((psi.real != 0) | (psi.imag != 0)).astype(np.int64)
    return idx, psi[idx].copy()


def to_dense(dims: Sequence[int], idx: np.ndarray, amp: np.ndarray) -> np.ndarray:
    psi = np.zeros(register_size(dims), dtype=np.complex128)
    psi[np.asarray(idx, dtype=np.int64)] = amp
    return psi


def basis(dims: Sequence[int], values: Sequence[int] | None = None):
    """One entry of amplitude exactly 1 at the basis state with the given digits (|0..0> default)."""
    st = strides(dims)
    x = 0 if values is None else sum(int(v) * int(s) for v, s in zip(values, st))
    return np.array([x], dtype=np.int64), np.array([1.0 + 0.0j])


def gate_class(U) -> Tuple[str, np.ndarray, np.ndarray]:
    """("monomial", rows, values) when every column and every row has exactly one entry that is
    not exactly zero, else ("dense", None, None)."""
    U = np.asarray(U, dtype=np.complex128)
    nz = (U.real != 0) | (U.imag != 0)
    if np.all(nz.sum(axis=0) == 1) and np.all(nz.sum(axis=1) == 1):
        rows = np.argmax(nz, axis=0)
        return "monomial", rows, U[rows, np.arange(U.shape[1])]
    return "dense", None, None


def _cmul(ur, ui, xr, xi):
    """(ur + i ui)(xr + i xi), each real operation rounded separately."""
    a = ur * xr
    b = ui * xi
    c = ur * xi
    e = ui * xr
    return a - b, c + e


def apply_gate(dims: Sequence[int], idx: np.ndarray, amp: np.ndarray, targets, controls, cvals, U):
    """One (controlled) k-qudit gate on the entry list; returns the new (idx, amp)."""
    dims = [int(d) for d in dims]
    st = strides(dims)
    T, C = [int(t) for t in targets], [int(c) for c in controls]
    U = np.asarray(U, dtype=np.complex128)
    tdims = [dims[t] for t in T]
    dT = int(np.prod(tdims)) if T else 1
    if U.shape != (dT, dT):
        raise ValueError(f"U must be {dT}x{dT}")
    idx = np.asarray(idx, dtype=np.int64)
    amp = np.asarray(amp, dtype=np.complex128)

    match = np.ones(idx.shape, dtype=bool)
    for c, v in zip(C, cvals):
        match &= (idx // st[c]) % dims[c] == int(v)
    # local column index of each entry: the target digits, first target most significant
    tdig = [(idx // st[t]) % dims[t] for t in T]
    loc = np.zeros(idx.shape, dtype=np.int64)
    for dg, d in zip(tdig, tdims):
        loc = loc * d + dg
    base = idx.copy()                         # the index with every target digit set to 0
    for dg, t in zip(tdig, T):
        base -= dg * st[t]

    def offset(local):                        # flat offset of local row indices
        off = np.zeros(np.shape(local), dtype=np.int64)
        rest = np.asarray(local, dtype=np.int64)
        for t, d in zip(reversed(T), reversed(tdims)):
            off += (rest % d) * st[t]
            rest = rest // d
        return off

    kind, rows, vals = gate_class(U)
    if kind == "monomial":
        out_idx = idx.copy()
        out_amp = amp.copy()
        m = np.flatnonzero(match)
        r = rows[loc[m]]
        out_idx[m] = base[m] + offset(r)
        u = vals[loc[m]]
        scale = ~((u.real == 1.0) & (u.imag == 0.0))
        ms = m[scale]
        re, im = _cmul(u.real[scale], u.imag[scale], amp.real[ms], amp.imag[ms])
        out_amp.real[ms] = re                          # the parts are stored as computed
        out_amp.imag[ms] = im
        return _ascending(out_idx, out_amp)

    # dense gate: one slice per distinct base among the matching entries
    m = np.flatnonzero(match)
    slice_key, sid = np.unique(base[m], return_inverse=True)
    sid = sid.reshape(-1)
    ns = slice_key.size
    Xr = np.zeros((ns, dT))
    Xi = np.zeros((ns, dT))
    Xr[sid, loc[m]] = amp.real[m]
    Xi[sid, loc[m]] = amp.imag[m]
    Yr = np.zeros((ns, dT))
    Yi = np.zeros((ns, dT))
    for i in range(dT):
        acc_r = np.zeros(ns)
        acc_i = np.zeros(ns)
        for j in range(dT):
            pr, pi = _cmul(U[i, j].real, U[i, j].imag, Xr[:, j], Xi[:, j])
            acc_r = acc_r + pr
            acc_i = acc_i + pi
        Yr[:, i] = acc_r
        Yi[:, i] = acc_i
    keep = (Yr != 0) | (Yi != 0)                      # exact zeros are not stored
    s_of, i_of = np.nonzero(keep)
    new_idx = slice_key[s_of] + offset(i_of)
    new_amp = np.empty(s_of.size, dtype=np.complex128)
    new_amp.real = Yr[s_of, i_of]
    new_amp.imag = Yi[s_of, i_of]
    p = np.flatnonzero(~match)                        # entries the gate leaves as they are
    return _ascending(np.concatenate([idx[p], new_idx]), np.concatenate([amp[p], new_amp]))


def _ascending(idx: np.ndarray, amp: np.ndarray):
    """The entries in increasing index (indices are distinct)."""
    order = np.argsort(idx, kind="stable")
    return idx[order], amp[order]


def run_circuit(circuit, idx=None, amp=None):
    """Every gate of the circuit in order, from (idx, amp) or the circuit's initial state."""
    dims = circuit.dims
    if idx is None:
        if getattr(circuit, "init_amps", None) is not None:
            idx, amp = from_dense(initial_state(circuit))
        else:
            idx, amp = basis(dims, getattr(circuit, "init_basis", None))
    idx, amp = _ascending(np.asarray(idx, dtype=np.int64), np.asarray(amp, dtype=np.complex128))
    for g in circuit.gates:
        idx, amp = apply_gate(dims, idx, amp, g.targets, g.controls, g.cvals, gate_unitary(g, dims))
    return idx, amp


def norm2(amp: np.ndarray) -> float:
    """Sum over the entries of re^2 + im^2: each square rounded, the sum of those rounded exactly."""
    a = np.asarray(amp, dtype=np.complex128)
    return math.fsum(np.concatenate([a.real * a.real, a.imag * a.imag]).tolist())
