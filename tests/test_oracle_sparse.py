"""Pins of the sparse-state oracle (oracle/sparse.py).

* Against the dense definition: the two independent dense oracles (per-gate contraction and the
  paper's operator-product execution of Sec. 3.6) give the same vector on random circuits.
* Closed forms: permutation circuits send a basis state to one basis state predicted by an integer
  simulation of the digits (Sec. 2.1 shifts and generalized CNOTs), on registers far beyond any
  dense state; the generalized GHZ state has d entries of exactly 1/sqrt(d); Hadamards on k qubits
  of a 40-qubit register give 2^k entries of equal magnitude; a Hadamard applied twice returns to
  one entry (the cancelled output is exactly zero and is dropped).
* Entries come in increasing index (the compressed column's order), on a hand-derived example.
"""
import itertools
import math

import numpy as np
import pytest

import circuits as C
import oracle as O
from oracle import sparse as S


def _check_valid(idx, amp):
    assert idx.dtype == np.int64 and amp.dtype == np.complex128
    assert np.all(np.diff(idx) > 0), "indices distinct and increasing"
    assert np.all((amp.real != 0) | (amp.imag != 0)), "no stored zero"


@pytest.mark.parametrize("seed", range(8))
def test_random_circuits_match_the_dense_contraction(seed):
    rng = np.random.default_rng(100 + seed)
    dims = [int(x) for x in rng.integers(2, 5, size=int(rng.integers(3, 8)))]
    circ = C.random_circuit(dims, 30, rng, max_targets=2, max_controls=2)
    idx, amp = S.run_circuit(circ)
    _check_valid(idx, amp)
    dense = O.run_circuit(circ)
    got = S.to_dense(dims, idx, amp)
    assert np.max(np.abs(got - dense)) <= 1e-13
    big = np.flatnonzero(np.abs(dense) > 1e-12)
    assert set(big.tolist()) <= set(idx.tolist())


def test_tiny_circuit_matches_the_operator_products():
    circ = C.config0()
    idx, amp = S.run_circuit(circ)
    _check_valid(idx, amp)
    ref = O.run_circuit_operator(circ)
    assert np.max(np.abs(S.to_dense(circ.dims, idx, amp) - ref)) <= 1e-13


def test_superposed_start_and_three_target_gates():
    rng = np.random.default_rng(7)
    dims = (2, 3, 2, 4, 3)
    psi0 = C.random_basis_superposition(int(np.prod(dims)), 40, rng)
    gates = [C.Gate("U", (4, 0, 2), (1,), (2,), U=C.haar_unitary(12, rng)),
             C.Gate("U", (3,), (0, 2), (1, 0), U=C.haar_unitary(4, rng)),
             C.Gate("X", (1,), (3,), (2,), a=2), C.Gate("Z", (3,), (1,), (1,))]
    circ = C.Circuit(dims, gates, init_amps=psi0)
    idx, amp = S.run_circuit(circ)
    _check_valid(idx, amp)
    assert np.max(np.abs(S.to_dense(dims, idx, amp) - O.run_circuit(circ))) <= 1e-13


def _digit_walk(dims, gates, start):
    """Integer simulation of shifts and generalized CNOTs on a digit list (Sec. 2.1)."""
    dg = list(start)
    for g in gates:
        if all(dg[c] == v for c, v in zip(g.controls, g.cvals)):
            t = g.targets[0]
            dg[t] = (dg[t] + g.a) % dims[t]
    return dg


def _flat(dims, dg):
    x = 0
    for d, v in zip(dims, dg):
        x = x * d + v
    return x


@pytest.mark.parametrize("seed", range(4))
def test_permutation_circuit_on_39_qutrits_is_one_basis_state(seed):
    rng = np.random.default_rng(200 + seed)
    dims = (3,) * 39                                   # D = 3^39, about 4.05e18
    circ = C.permutation_circuit(dims, 300, rng)
    start = [int(v) for v in rng.integers(0, 3, size=39)]
    circ.init_basis = tuple(start)
    idx, amp = S.run_circuit(circ)
    assert idx.tolist() == [_flat(dims, _digit_walk(dims, circ.gates, start))]
    assert amp[0] == 1.0 + 0.0j


def test_permutations_move_a_superposition_without_touching_amplitudes():
    rng = np.random.default_rng(5)
    dims = tuple(int(x) for x in rng.choice([2, 3, 4], size=24))
    k = 6
    had = [C.Gate("F", (q,)) for q in range(k) if dims[q] >= 2]
    perm = C.permutation_circuit(dims, 200, rng)
    idx0, amp0 = S.run_circuit(C.Circuit(dims, had))
    idx, amp = S.run_circuit(C.Circuit(dims, perm.gates), idx0, amp0)
    _check_valid(idx, amp)
    # each entry lands where the digit walk sends its index, with the same bits
    moved = {_flat(dims, _digit_walk(dims, perm.gates, O.digits_of(x0, dims))): a for x0, a in zip(idx0.tolist(), amp0)}
    assert sorted(moved) == idx.tolist()
    assert all(moved[x] == a for x, a in zip(idx.tolist(), amp))


@pytest.mark.parametrize("d,n", [(2, 5), (3, 4), (4, 3), (5, 3)])
def test_generalized_ghz(d, n):
    dims = (d,) * n
    gates = [C.Gate("F", (0,))]
    for k in range(1, n):
        for v in range(1, d):
            gates.append(C.Gate("X", (k,), (0,), (v,), a=v))
    idx, amp = S.run_circuit(C.Circuit(dims, gates))
    step = sum(d ** (n - 1 - q) for q in range(n))
    assert idx.tolist() == [j * step for j in range(d)]
    assert np.all(amp == complex(1.0 / math.sqrt(d), 0.0))


def test_hadamards_on_a_40_qubit_register():
    dims = (2,) * 40
    qs = (3, 17, 29, 39)
    idx, amp = S.run_circuit(C.Circuit(dims, [C.Gate("F", (q,)) for q in qs]))
    want = sorted(sum(b << (39 - q) for b, q in zip(bits, qs)) for bits in itertools.product((0, 1), repeat=4))
    assert sorted(idx.tolist()) == want
    assert np.all(amp == amp[0]) and abs(amp[0].real - 0.25) < 1e-15 and amp[0].imag == 0.0
    assert abs(S.norm2(amp) - 1.0) < 1e-15


def test_cancelled_output_is_dropped():
    dims = (2, 3)
    idx, amp = S.run_circuit(C.Circuit(dims, [C.Gate("F", (0,)), C.Gate("F", (0,))]))
    assert idx.tolist() == [0] and abs(amp[0] - 1.0) < 1e-15


def test_entries_in_increasing_index():
    # dims (2, 3): flat index 3*q0 + q1. Entries (4, a), (0, b), (3, b) given out of order; F_2 on
    # qudit 0 forms the slice q1 = 1 (inputs x = (0, a): outputs at 1 and 4) and the slice q1 = 0
    # (x = (b, b), whose row-1 output b/sqrt2 - b/sqrt2 is exactly zero and dropped: output at 0).
    dims = (2, 3)
    a, b = 0.6 - 0.2j, 0.5 + 0.3j
    idx0 = np.array([4, 0, 3], dtype=np.int64)
    amp0 = np.array([a, b, b])
    idx, amp = S.apply_gate(dims, idx0, amp0, (0,), (), (), O.f_gate(2))
    assert idx.tolist() == [0, 1, 4]
    dense = O.apply_gate(S.to_dense(dims, idx0, amp0), dims, (0,), (), (), O.f_gate(2))
    assert np.max(np.abs(amp - dense[idx])) < 1e-15
    # F_3 on qudit 1 controlled by q0 = 1: entries 4 and 3 form one slice with outputs 3, 4, 5;
    # the non-matching entry 0 is kept
    idx2, amp2 = S.apply_gate(dims, idx0, amp0, (1,), (0,), (1,), O.f_gate(3))
    assert idx2.tolist() == [0, 3, 4, 5] and amp2[0] == b
    # a monomial gate that sends the largest index to the smallest: X_{+1} on qudit 0
    idx3, amp3 = S.apply_gate(dims, np.array([4, 0]), np.array([a, b]), (0,), (), (), O.x_gate(2, 1))
    assert idx3.tolist() == [1, 3] and amp3.tolist() == [a, b]


def test_gate_classes():
    assert S.gate_class(O.x_gate(5, 2))[0] == "monomial"
    assert S.gate_class(O.z_gate(3))[0] == "monomial"
    swap = np.zeros((9, 9), dtype=np.complex128)
    for i, j in itertools.product(range(3), range(3)):
        swap[3 * j + i, 3 * i + j] = 1.0
    kind, rows, vals = S.gate_class(swap)
    assert kind == "monomial" and np.all(vals == 1.0)
    assert S.gate_class(O.f_gate(3))[0] == "dense"
    assert S.gate_class(C.haar_unitary(4, np.random.default_rng(0)))[0] == "dense"
    # one entry per column but two in a row (not unitary): would merge two indices, so dense
    assert S.gate_class(np.array([[1, 1], [0, 0]], dtype=np.complex128))[0] == "dense"


def test_swap_exchanges_digits_and_phases_multiply():
    dims = (3, 2, 3)
    swap = np.zeros((9, 9), dtype=np.complex128)
    for i, j in itertools.product(range(3), range(3)):
        swap[3 * j + i, 3 * i + j] = 1.0
    idx, amp = S.basis(dims, (1, 1, 2))
    idx, amp = S.apply_gate(dims, idx, amp, (0, 2), (), (), swap)
    assert idx.tolist() == [_flat(dims, (2, 1, 1))] and amp[0] == 1.0
    idx, amp = S.apply_gate(dims, idx, amp, (0,), (), (), O.z_gate(3))
    assert abs(amp[0] - np.exp(2j * np.pi * 2 / 3)) < 1e-15


def test_from_dense_round_trip():
    rng = np.random.default_rng(3)
    psi = C.random_basis_superposition(500, 30, rng)
    idx, amp = S.from_dense(psi)
    assert np.all(np.diff(idx) > 0) and len(idx) == 30
    assert np.array_equal(S.to_dense((500,), idx, amp), psi)
