"""GPU runs of circuits from the front-end (qd_circuit_apply) against the oracle: the hand-derived
QASM program, a random program, and a Toffoli chain against the multi-controlled gate it
replaces (on inputs whose intermediate levels are free)."""
import numpy as np
import pytest

import circuits as C
import oracle as O
from oracle import frontend as F
import paper_2211_07918_amd as Q
from gpu_util import max_abs, torch_stream
from test_frontend_abi import random_program
from test_oracle_frontend import PROGRAM, to_circuit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stream():
    return torch_stream()


def run_lib(text_or_circuit, dims, stream, psi0=None):
    c = Q.qd_qasm_parse(text_or_circuit) if isinstance(text_or_circuit, str) else text_or_circuit
    s = Q.qd_state_init(dims, Q.QD_C128, stream)
    try:
        if psi0 is not None:
            Q.qd_state_upload(s, psi0)
        Q.qd_circuit_apply(s, c)
        return Q.qd_state_download(s)
    finally:
        Q.qd_state_free(s)
        if isinstance(text_or_circuit, str):
            Q.qd_circuit_free(c)


def test_program_state(stream):
    _, dims, gates = F.parse_qasm(PROGRAM)
    psi = run_lib(PROGRAM, dims, stream)
    assert max_abs(psi, O.run_circuit(to_circuit(dims, gates))) <= 1e-15
    assert abs(psi[3] - 0.7071067811865475) <= 1e-16 and abs(psi[20] + 0.7071067811865475) <= 1e-16


@pytest.mark.parametrize("seed", range(3))
def test_random_program(stream, seed):
    text = random_program(np.random.default_rng(seed), n_q=7, n_g=120)
    _, dims, gates = F.parse_qasm(text)
    psi = run_lib(text, dims, stream)
    assert max_abs(psi, O.run_circuit(to_circuit(dims, gates))) <= 1e-12


def test_toffoli_chain_on_the_gpu(stream):
    dims = [2, 3, 3, 2]
    mct = Q.qd_circuit_create(dims)
    Q.qd_circuit_add(mct, Q.QD_GATE_X, 3, 1, (0, 1, 2), (1, 1, 1))
    chain = Q.qd_circuit_decompose(mct)
    try:
        rng = np.random.default_rng(4)
        # superpositions over the logical subspace: the chained qutrits hold 0 or 1
        for _ in range(3):
            psi0 = np.zeros(36, dtype=np.complex128)
            for x in range(36):
                dg = O.digits_of(x, dims)
                if dg[1] < 2 and dg[2] < 2:
                    psi0[x] = rng.normal() + 1j * rng.normal()
            psi0 /= np.linalg.norm(psi0)
            a = run_lib(mct, dims, stream, psi0)
            b = run_lib(chain, dims, stream, psi0)
            assert max_abs(a, b) <= 1e-15
    finally:
        Q.qd_circuit_free(chain)
        Q.qd_circuit_free(mct)
