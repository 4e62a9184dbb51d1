"""Pins for the oracle against what the paper prints and what the mathematics fixes (CPU only).

Each check is independent of the oracle's own formulas: values printed in the paper, library
routines (numpy.fft, scipy block_diag), algebraic identities of the Weyl-Heisenberg group, integer
digit simulation and brute force over basis states.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import circuits as C
import oracle as O

GD = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------------ P1: worked example
def test_worked_example_sec39():
    """Sec. 3.9: dims (2,3,3), H on q0, CX((0,1), +2) -> |000> and |120> with 0.7071067811865475."""
    g = json.load(open(os.path.join(GD, "worked_example.json")))
    dims = g["dims"]
    circ = C.Circuit(tuple(dims), [], init_basis=tuple(g["init_states"]))
    for r in g["gates"]:
        circ.gates.append(C.Gate(r["kind"], tuple(r["targets"]), tuple(r.get("controls", ())),
                                 tuple(r.get("control_values", ())), a=r.get("a", 0)))
    psi = O.run_circuit(circ)
    expected = np.zeros(O.register_size(dims), dtype=np.complex128)
    for ket, amp in g["expected_amplitudes"].items():
        expected[O.index_of([int(ch) for ch in ket], dims)] = float(amp)
    # bit-exact: the printed decimal is the shortest repr of fl(1/sqrt 2)
    assert np.array_equal(psi, expected)
    assert O.index_of([1, 2, 0], dims) == 15
    # the paper's own scheme (operator products, then one GEMV) gives the same state
    assert np.array_equal(O.run_circuit_operator(circ), expected)


def test_hadamard_d2_printed_sec39():
    g = json.load(open(os.path.join(GD, "worked_example.json")))
    H = np.array([[float(x) for x in row] for row in g["expected_hadamard_d2"]])
    assert np.array_equal(O.f_gate(2), H.astype(np.complex128))


# ------------------------------------------------------------------------ P3: gate identities
@pytest.mark.parametrize("d", [2, 3, 4, 5, 6, 7, 9])
def test_weyl_heisenberg_identities(d):
    X, Z, F = O.x_gate(d, 1), O.z_gate(d), O.f_gate(d)
    I = np.eye(d)
    w = np.exp(2j * np.pi / d)
    Fh = F.conj().T
    assert np.allclose(np.linalg.matrix_power(X, d), I, atol=1e-14)
    assert np.allclose(np.linalg.matrix_power(Z, d), I, atol=1e-13)
    assert np.allclose(Z @ X, w * (X @ Z), atol=1e-14)            # ZX = omega XZ
    assert np.allclose(F @ X @ Fh, Z, atol=1e-14)                  # F X F^dag = Z
    assert np.allclose(F @ Z @ Fh, np.linalg.inv(X), atol=1e-14)  # F Z F^dag = X^{-1}
    assert np.allclose(np.linalg.matrix_power(F, 4), I, atol=1e-13)
    assert np.allclose(F @ Fh, I, atol=1e-14)
    e0 = np.zeros(d); e0[0] = 1
    assert np.allclose(F @ e0, np.full(d, 1 / math.sqrt(d)), atol=1e-15)  # DFT|0> uniform
    # F is the unitary inverse DFT matrix of numpy.fft
    assert np.allclose(F, np.sqrt(d) * np.fft.ifft(np.eye(d), axis=0), atol=1e-14)
    for a in range(1, d):
        assert np.array_equal(O.x_gate(d, a), np.linalg.matrix_power(X, a))


def test_exact_quarter_turns():
    assert np.array_equal(O.z_gate(4), np.diag([1, 1j, -1, -1j]))
    assert np.array_equal(O.z_gate(2), np.diag([1, -1]).astype(np.complex128))


def test_shift_range():
    with pytest.raises(ValueError):
        O.x_gate(3, 0)
    with pytest.raises(ValueError):
        O.x_gate(3, 3)


# ------------------------------------------------------------------------ P4: C_{X,d} matrix
@pytest.mark.parametrize("d,a", [(2, 1), (3, 1), (3, 2), (4, 3), (5, 2)])
def test_generalized_cnot_block_matrix(d, a):
    """Sec. 2.1: C_{X,d} = blockdiag(I_d, ..., I_d, X^d_{+a}) with the control listed first."""
    M = O.gate_operator((d, d), [1], [0], [d - 1], O.x_gate(d, a))
    blocks = [np.eye(d)] * (d - 1) + [O.x_gate(d, a)]
    assert np.array_equal(M, scipy.linalg.block_diag(*blocks).astype(np.complex128))


@pytest.mark.parametrize("d,n", [(2, 3), (3, 3), (2, 4)])
def test_multi_controlled_toffoli_block_matrix(d, n):
    """Sec. 2.1: C^n_{X,d} = blockdiag(I_d, ..., X^d_{+a}): all n-1 controls at d-1."""
    dims = (d,) * n
    M = O.gate_operator(dims, [n - 1], list(range(n - 1)), [d - 1] * (n - 1), O.x_gate(d, 1))
    blocks = [np.eye(d)] * (d ** (n - 1) - 1) + [O.x_gate(d, 1)]
    assert np.array_equal(M, scipy.linalg.block_diag(*blocks).astype(np.complex128))


def test_mixed_dimension_cx():
    """CX with a qubit control and a qutrit target (the CX^3_{+2} of Sec. 3.1)."""
    M = O.gate_operator((2, 3), [1], [0], [1], O.x_gate(3, 2))
    assert np.array_equal(M, scipy.linalg.block_diag(np.eye(3), O.x_gate(3, 2)).astype(np.complex128))


# ------------------------------------------------------------------------ P5: Toffoli decomposition
def test_toffoli_decomposition_with_intermediate_qutrit():
    """Sec. 3.4: Toffoli((0,1,2), +1) = cx((0,1),+1), cx((1,2),+1), cx((0,1),+2) with the middle
    wire a qutrit (controls activate on d_c - 1). On qubit inputs it equals the Toffoli."""
    dims = (2, 3, 2)
    circ = C.Circuit(dims, [C.Gate("X", (1,), (0,), (1,), a=1),
                            C.Gate("X", (2,), (1,), (2,), a=1),
                            C.Gate("X", (1,), (0,), (1,), a=2)])
    for x0 in range(2):
        for x1 in range(2):
            for x2 in range(2):
                psi = O.run_circuit(circ, O.basis_state(dims, (x0, x1, x2)))
                want = O.basis_state(dims, (x0, x1, x2 ^ (x0 & x1)))
                assert np.array_equal(psi, want), (x0, x1, x2)


# ------------------------------------------------------------------------ P6: O1 == O2
def test_o1_equals_bruteforce_config0():
    c = C.config0()
    a = O.run_circuit(c)
    b = O.run_circuit_operator(c)
    assert np.max(np.abs(a - b)) <= 1e-13
    assert abs(O.norm2(a) - 1) <= 1e-13


@pytest.mark.parametrize("seed,dims", [(1, (2, 3, 4)), (2, (3, 2, 2, 3)), (3, (4, 4, 3)),
                                       (4, (2, 2, 2, 2, 2, 2)), (5, (5, 3, 2, 2)), (6, (7,)),
                                       (7, (3, 3, 3, 3, 3, 3, 3))])
def test_o1_equals_bruteforce_random(seed, dims):
    rng = C.seeded_rng(seed)
    c = C.random_circuit(dims, 30, rng, max_targets=3, max_controls=2, max_dT=27)
    c.init_amps = C.random_basis_superposition(O.register_size(dims), 7, rng)
    a = O.run_circuit(c)
    b = O.run_circuit_operator(c)
    assert np.max(np.abs(a - b)) <= 1e-13


def test_kron_equals_enumeration():
    rng = C.seeded_rng(11)
    dims = (2, 3, 4, 3)
    for t in range(4):
        U = C.haar_unitary(dims[t], rng)
        assert np.allclose(O.kron_operator(dims, t, U), O.gate_operator(dims, [t], [], [], U),
                           atol=0, rtol=0)


def test_apply_gate_at_matches_contraction():
    rng = C.seeded_rng(12)
    dims = (3, 2, 4, 3, 2)
    D = O.register_size(dims)
    psi = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    U = C.haar_unitary(12, rng)
    out = O.apply_gate(psi, dims, [2, 0], [4], [1], U)
    idx = rng.choice(D, 50, replace=False)
    assert np.allclose(O.apply_gate_at(psi, dims, [2, 0], [4], [1], U, idx), out[idx],
                       atol=1e-13, rtol=0)


# ------------------------------------------------------------------------ P7: generalized GHZ
@pytest.mark.parametrize("d,n", [(2, 5), (3, 4), (4, 4), (5, 3)])
def test_generalized_ghz(d, n):
    dims = (d,) * n
    gates = [C.Gate("F", (0,))]
    for k in range(1, n):
        for v in range(1, d):
            gates.append(C.Gate("X", (k,), (0,), (v,), a=v))
    psi = O.run_circuit(C.Circuit(dims, gates))
    want = np.zeros(d ** n, dtype=np.complex128)
    for j in range(d):
        want[O.index_of([j] * n, dims)] = 1 / math.sqrt(d)
    assert np.max(np.abs(psi - want)) <= 1e-15


# ------------------------------------------------------------------------ P8: qudit QFT
@pytest.mark.parametrize("d,n", [(3, 3), (4, 3), (2, 4), (3, 4), (4, 6), (2, 9), (3, 7)])
def test_qudit_qft_equals_inverse_fft(d, n):
    D = d ** n
    rng = C.seeded_rng(100 + d * n)
    psi0 = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    psi0 /= np.linalg.norm(psi0)
    c = C.Circuit((d,) * n, C.qudit_qft_gates(d, n), init_amps=psi0)
    assert np.max(np.abs(O.run_circuit(c) - math.sqrt(D) * np.fft.ifft(psi0))) <= 1e-12


# ------------------------------------------------------------------------ P9: permutation circuits
def _digit_sim(dims, gates, digs):
    digs = list(digs)
    for g in gates:
        if all(digs[c] == v for c, v in zip(g.controls, g.cvals)):
            t = g.targets[0]
            digs[t] = (digs[t] + g.a) % dims[t]
    return digs


@pytest.mark.parametrize("seed,dims", [(21, (2, 3, 4, 2, 3)), (22, (3,) * 7), (23, (4, 2, 5, 2))])
def test_permutation_circuits_track_basis(seed, dims):
    rng = C.seeded_rng(seed)
    c = C.permutation_circuit(dims, 60, rng)
    start = [int(rng.integers(d)) for d in dims]
    psi = O.run_circuit(c, O.basis_state(dims, start))
    end = _digit_sim(dims, c.gates, start)
    want = np.zeros_like(psi)
    want[O.index_of(end, dims)] = 1.0
    assert np.array_equal(psi, want)


# ------------------------------------------------------------------------ P10: diagonal circuits
@pytest.mark.parametrize("seed,dims", [(31, (2, 3, 4, 3)), (32, (5, 3, 2))])
def test_diagonal_circuits_closed_form(seed, dims):
    rng = C.seeded_rng(seed)
    c = C.diagonal_circuit(dims, 40, rng)
    D = O.register_size(dims)
    psi0 = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    out = O.run_circuit(c, psi0)
    # closed form: each basis state x picks up prod over active gates of exp(2 pi i x_t / d_t)
    want = np.empty(D, dtype=np.complex128)
    for x in range(D):
        dg = O.digits_of(x, dims)
        ang = 0.0
        for g in c.gates:
            if all(dg[cc] == v for cc, v in zip(g.controls, g.cvals)):
                t = g.targets[0]
                ang += dg[t] / dims[t]
        want[x] = psi0[x] * np.exp(2j * np.pi * ang)
    assert np.max(np.abs(out - want)) <= 1e-12


# ------------------------------------------------------------------------ P11: norm, compare
def test_norm_preserved_config1_shrink():
    c = C.config1_shrink(200)
    psi = O.run_circuit(c)
    assert abs(O.norm2(psi) - 1.0) <= 1e-13


def test_compare_closed_forms():
    rng = C.seeded_rng(41)
    psi = rng.standard_normal(64) + 1j * rng.standard_normal(64)
    psi /= np.linalg.norm(psi)
    th = 0.3
    ma, fl, dr = O.compare(psi, np.exp(1j * th) * psi)
    assert abs(fl) <= 1e-15 and dr <= 1e-15
    assert abs(ma - abs(np.exp(1j * th) - 1) * np.max(np.abs(psi))) <= 1e-15
    eps = 1e-3
    ma, fl, dr = O.compare(psi, (1 + eps) * psi)
    assert abs(dr - ((1 + eps) ** 2 - 1)) <= 1e-14
    assert abs(fl - (1 - (1 + eps) ** 2)) <= 1e-14
    # orthogonal states: fidelity loss 1
    e = np.zeros(4, complex); e[0] = 1
    f = np.zeros(4, complex); f[1] = 1
    assert O.compare(e, f)[1] == 1.0


def test_probabilities_match_modulus():
    rng = C.seeded_rng(42)
    psi = rng.standard_normal(100) + 1j * rng.standard_normal(100)
    assert np.allclose(O.probabilities(psi), np.abs(psi) ** 2, rtol=1e-15, atol=0)


# ------------------------------------------------------------------------ fused blocks
def test_fused_block_equals_sequential_application():
    rng = C.seeded_rng(51)
    dims = (2, 3, 4, 3, 2)
    window = [3, 0, 2]
    gates = [C.Gate("U", (0, 3), U=C.haar_unitary(6, rng)), C.Gate("F", (2,)),
             C.Gate("X", (3,), (0,), (1,), a=2), C.Gate("U", (2,), (3,), (2,), U=C.haar_unitary(4, rng))]
    M = O.fused_block(dims, window, gates)
    D = O.register_size(dims)
    psi = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    seq = O.run_circuit(C.Circuit(dims, gates), psi)
    fused = O.apply_gate(psi, dims, window, [], [], M)
    assert np.max(np.abs(seq - fused)) <= 1e-13
    assert np.allclose(M @ M.conj().T, np.eye(M.shape[0]), atol=1e-13)


# ------------------------------------------------------------------------ pins catch mistakes
def test_pins_detect_planted_mistakes(monkeypatch):
    """Plant plausible mistakes in the oracle and check a pin above fails for each."""
    # (a) conjugated omega in Z: breaks ZX = omega XZ
    good_z = O.z_gate
    monkeypatch.setattr(O, "z_gate", lambda d: good_z(d).conj())
    X, Z = O.x_gate(3), O.z_gate(3)
    assert not np.allclose(Z @ X, np.exp(2j * np.pi / 3) * (X @ Z))
    monkeypatch.undo()

    # (b) little-endian register: the worked example's |120> moves
    from oracle import qudit as Q
    good_apply = Q.apply_gate

    def little_endian_apply(psi, dims, targets, controls, cvals, U):
        # the flat array read with qudit n-1 as the most significant digit
        n = len(dims)
        rev = lambda q: n - 1 - q
        return good_apply(psi, tuple(reversed(dims)), [rev(t) for t in targets],
                          [rev(c) for c in controls], cvals, U)

    circ = C.Circuit((2, 3, 3), [C.Gate("F", (0,)), C.Gate("X", (1,), (0,), (1,), a=2)])
    monkeypatch.setattr(Q, "apply_gate", little_endian_apply)
    psi_bad = Q.run_circuit(circ)
    monkeypatch.undo()
    assert abs(psi_bad[15]) < 0.5  # |120> is not populated when the significance is flipped

    # (c) transposed U in the contraction: O1 != O2 on a Haar gate
    monkeypatch.setattr(Q, "apply_gate", lambda psi, dims, t, c, v, U: good_apply(psi, dims, t, c, v, np.asarray(U).T))
    rng = C.seeded_rng(61)
    c = C.random_circuit((2, 3, 4), 6, rng)
    a = Q.run_circuit(c)
    monkeypatch.undo()
    assert np.max(np.abs(a - O.run_circuit_operator(c))) > 1e-6

    # (d) controls ignored: the Toffoli decomposition pin fails
    monkeypatch.setattr(Q, "apply_gate", lambda psi, dims, t, c, v, U: good_apply(psi, dims, t, [], [], U))
    dims = (2, 3, 2)
    circ = C.Circuit(dims, [C.Gate("X", (1,), (0,), (1,), a=1), C.Gate("X", (2,), (1,), (2,), a=1),
                            C.Gate("X", (1,), (0,), (1,), a=2)])
    psi = Q.run_circuit(circ, O.basis_state(dims, (0, 0, 0)))
    monkeypatch.undo()
    assert not np.array_equal(psi, O.basis_state(dims, (0, 0, 0)))
