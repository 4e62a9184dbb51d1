"""Pins of the density-matrix oracle (oracle/density.py).

* Pure evolution: psi psi^dagger taken through gates equals the outer product of the state-vector
  oracle's result (per-gate contraction, an independent code path).
* Closed forms: the named channels are trace preserving (sum K^dagger K = I); full depolarizing of a
  one-qudit register gives I/d and, on one qudit of a larger register, tr_t(rho) (x) I/d (partial
  trace by reshaping); the d^2 Weyl operators twirl any rho to d tr(rho) I; dephasing scales every
  off-diagonal element by 1 - p d/(d-1); amplitude damping moves weight g from |j> to |j-1>.
* Random noisy circuits keep rho Hermitian, positive semidefinite and of unit trace; purity and
  fidelity take their closed values on pure states.
"""
import math

import numpy as np
import pytest

import circuits as C
import oracle as O
from oracle import density as Dm


def random_rho(D, rng, rank=3):
    A = rng.standard_normal((D, rank)) + 1j * rng.standard_normal((D, rank))
    rho = A @ A.conj().T
    return rho / np.trace(rho).real


@pytest.mark.parametrize("seed", range(4))
def test_pure_evolution_matches_the_state_vector_oracle(seed):
    rng = np.random.default_rng(seed)
    dims = [int(x) for x in rng.integers(2, 4, size=4)]
    circ = C.random_circuit(dims, 20, rng)
    rho = Dm.from_state(O.basis_state(dims))
    for g in circ.gates:
        rho = Dm.apply_unitary(rho, dims, g.targets, g.controls, g.cvals, O.gate_unitary(g, dims))
    psi = O.run_circuit(circ)
    assert np.max(np.abs(rho - np.outer(psi, psi.conj()))) <= 1e-13
    assert abs(Dm.purity(rho) - 1.0) <= 1e-13 and abs(Dm.fidelity(rho, psi) - 1.0) <= 1e-13


@pytest.mark.parametrize("d", [2, 3, 4, 5])
@pytest.mark.parametrize("make,p", [(Dm.depolarizing, 0.3), (Dm.dephasing, 0.2), (Dm.amplitude_damping, 0.4)])
def test_named_channels_are_trace_preserving(d, make, p):
    assert Dm.kraus_complete(make(d, p)) <= 1e-14


def test_depolarizing_closed_forms():
    rng = np.random.default_rng(1)
    for d in (2, 3, 4):
        rho = random_rho(d, rng)
        assert np.max(np.abs(Dm.apply_channel(rho, (d,), (0,), Dm.depolarizing(d, 1.0)) - np.eye(d) / d)) <= 1e-14
    dims = (2, 3, 2)
    rho = random_rho(12, rng)
    p = 0.35
    got = Dm.apply_channel(rho, dims, (1,), Dm.depolarizing(3, p))
    r = rho.reshape(2, 3, 2, 2, 3, 2)
    red = np.einsum("ajbcjd->abcd", r)                       # trace over qudit 1 (row and column)
    full = np.einsum("abcd,jk->ajbckd", red, np.eye(3) / 3).reshape(12, 12)
    assert np.max(np.abs(got - ((1 - p) * rho + p * full))) <= 1e-14


@pytest.mark.parametrize("d", [2, 3, 5])
def test_weyl_twirl(d):
    rho = random_rho(d, np.random.default_rng(d))
    X, Z = O.x_gate(d, 1), O.z_gate(d)
    s = sum(np.linalg.matrix_power(X, a) @ np.linalg.matrix_power(Z, b) @ rho
            @ (np.linalg.matrix_power(X, a) @ np.linalg.matrix_power(Z, b)).conj().T
            for a in range(d) for b in range(d))
    assert np.max(np.abs(s - d * np.trace(rho) * np.eye(d))) <= 1e-13


@pytest.mark.parametrize("d", [2, 3, 4])
def test_dephasing_scales_coherences(d):
    rho = random_rho(d, np.random.default_rng(10 + d))
    p = 0.3
    got = Dm.apply_channel(rho, (d,), (0,), Dm.dephasing(d, p))
    f = 1.0 - p * d / (d - 1)
    want = rho * f
    np.fill_diagonal(want, np.diagonal(rho))
    assert np.max(np.abs(got - want)) <= 1e-14


def test_amplitude_damping_moves_one_level():
    d, g = 4, 0.25
    for j in range(d):
        rho = np.zeros((d, d), dtype=np.complex128)
        rho[j, j] = 1.0
        got = Dm.apply_channel(rho, (d,), (0,), Dm.amplitude_damping(d, g))
        want = np.zeros((d, d))
        if j == 0:
            want[0, 0] = 1.0
        else:
            want[j, j] = 1.0 - g
            want[j - 1, j - 1] = g
        assert np.max(np.abs(got - want)) <= 1e-15


@pytest.mark.parametrize("seed", range(3))
def test_noisy_circuits_stay_physical(seed):
    rng = np.random.default_rng(40 + seed)
    dims = (2, 3, 2, 3)
    circ = C.random_circuit(dims, 15, rng)
    rho = Dm.from_state(O.basis_state(dims))
    makers = (Dm.depolarizing, Dm.dephasing, Dm.amplitude_damping)
    for g in circ.gates:
        rho = Dm.apply_unitary(rho, dims, g.targets, g.controls, g.cvals, O.gate_unitary(g, dims))
        q = g.targets[0]
        rho = Dm.apply_channel(rho, dims, (q,), makers[int(rng.integers(3))](dims[q], 0.1))
    assert abs(Dm.trace(rho) - 1.0) <= 1e-13
    assert np.max(np.abs(rho - rho.conj().T)) <= 1e-14
    assert np.min(np.linalg.eigvalsh(rho)) >= -1e-13
    assert 1.0 / np.prod(dims) - 1e-13 <= Dm.purity(rho) <= 1.0 + 1e-13
    assert abs(np.sum(Dm.probabilities(rho)) - 1.0) <= 1e-13


def test_two_qudit_channel_is_the_product_of_its_factors():
    """A channel given as the tensor products of two one-qudit Kraus sets equals applying them in
    turn (first target most significant in the joint Kraus matrices)."""
    rng = np.random.default_rng(3)
    dims = (3, 2, 2)
    rho = random_rho(12, rng)
    ka, kb = Dm.dephasing(3, 0.3), Dm.amplitude_damping(2, 0.4)
    joint = [np.kron(a, b) for a in ka for b in kb]
    got = Dm.apply_channel(rho, dims, (0, 2), joint)
    want = Dm.apply_channel(Dm.apply_channel(rho, dims, (0,), ka), dims, (2,), kb)
    assert np.max(np.abs(got - want)) <= 1e-14
