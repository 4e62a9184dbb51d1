"""Parity of the C-ABI circuit front-end (qd_qasm_parse, qd_circuit_moments, qd_circuit_decompose)
with the front-end oracle. Host-only calls: integer results, compared exactly."""
import numpy as np
import pytest

from oracle import frontend as F
import paper_2211_07918_amd as Q
from test_oracle_frontend import MALFORMED, PROGRAM, random_gates

KIND = {"X": Q.QD_GATE_X, "Z": Q.QD_GATE_Z, "F": Q.QD_GATE_F}


def lib_gates(c):
    return [(k, t, a, ctl, val) for k, t, a, ctl, val in Q.qd_circuit_gates(c)]


def oracle_gates(gates):
    return [(KIND[k], t, a, tuple(ctl), tuple(val)) for k, t, a, ctl, val in gates]


def random_program(rng, n_q=5, n_g=60):
    dims = [int(x) for x in rng.integers(2, 6, size=n_q)]
    names = [f"w{i}" for i in range(n_q)]
    lines = [f".qudit {n_q}"] + [f"qudit {nm.upper() if i % 2 else nm} ({d})" for i, (nm, d) in enumerate(zip(names, dims))]
    lines.append(".begin")
    for _ in range(n_g):
        kind = ["X", "H", "Z", "CX", "MCT"][int(rng.integers(5))]
        t = int(rng.integers(n_q))
        if kind in ("H", "Z"):
            lines.append(f"{kind.lower() if rng.random() < 0.5 else kind} {names[t]}")
        elif kind == "X":
            sh = f" {int(rng.integers(1, dims[t]))}" if rng.random() < 0.5 else ""
            lines.append(f"X {names[t]}{sh}")
        else:
            k = 1 if kind == "CX" else int(rng.integers(2, 4))
            ctl = [int(x) for x in rng.choice([q for q in range(n_q) if q != t], k, replace=False)]
            sh = f" {int(rng.integers(1, dims[t]))}" if rng.random() < 0.5 else ""
            lines.append(f"{kind} " + " ".join(names[q] for q in ctl) + f" {names[t]}{sh}  # gate")
    lines.append(".end")
    return "\n".join(lines)


def test_program_parses_like_the_oracle():
    c = Q.qd_qasm_parse(PROGRAM)
    try:
        names, dims, gates = F.parse_qasm(PROGRAM)
        assert Q.qd_circuit_dims(c) == dims
        assert [Q.qd_circuit_name(c, q) for q in range(len(dims))] == names
        assert lib_gates(c) == oracle_gates(gates)
    finally:
        Q.qd_circuit_free(c)


@pytest.mark.parametrize("seed", range(8))
def test_random_programs(seed):
    text = random_program(np.random.default_rng(seed))
    c = Q.qd_qasm_parse(text)
    try:
        _, dims, gates = F.parse_qasm(text)
        assert Q.qd_circuit_dims(c) == dims
        assert lib_gates(c) == oracle_gates(gates)
        mom, depth = Q.qd_circuit_moments(c)
        assert mom == F.moments(gates) and depth == max(mom) + 1
    finally:
        Q.qd_circuit_free(c)


def test_malformed_programs_rejected_by_both():
    for bad in MALFORMED:
        with pytest.raises(F.QasmError):
            F.parse_qasm(bad)
        with pytest.raises(Q.QDError) as e:
            Q.qd_qasm_parse(bad)
        assert e.value.code == Q.QD_EINVAL


@pytest.mark.parametrize("seed", range(6))
def test_moments_of_built_circuits(seed):
    rng = np.random.default_rng(100 + seed)
    dims = [int(x) for x in rng.integers(2, 5, size=6)]
    gates = random_gates(rng, dims, 80)
    c = Q.qd_circuit_create(dims)
    try:
        for k, t, a, ctl, val in gates:
            Q.qd_circuit_add(c, KIND[k], t, a, ctl, val)
        mom, depth = Q.qd_circuit_moments(c)
        assert mom == F.moments(gates) and depth == max(mom) + 1
    finally:
        Q.qd_circuit_free(c)


@pytest.mark.parametrize("seed", range(6))
def test_decomposition_like_the_oracle(seed):
    rng = np.random.default_rng(200 + seed)
    dims = [int(x) for x in rng.integers(3, 6, size=6)]
    gates = []
    for _ in range(30):
        t = int(rng.integers(6))
        k = int(rng.integers(0, 4))
        ctl = tuple(int(x) for x in rng.choice([q for q in range(6) if q != t], k, replace=False))
        # values that leave a free level on every chained control
        val = tuple(int(rng.integers(0, dims[q] - 1)) for q in ctl)
        gates.append(("X", t, int(rng.integers(1, dims[t])), ctl, val))
    c = Q.qd_circuit_create(dims)
    try:
        for k, t, a, ctl, val in gates:
            Q.qd_circuit_add(c, KIND[k], t, a, ctl, val)
        d = Q.qd_circuit_decompose(c)
        try:
            assert lib_gates(d) == oracle_gates(F.decompose_circuit(dims, gates))
            assert all(len(g[3]) <= 1 for g in lib_gates(d))
        finally:
            Q.qd_circuit_free(d)
    finally:
        Q.qd_circuit_free(c)


def test_builder_and_decomposition_errors():
    c = Q.qd_circuit_create([2, 3, 2])
    try:
        for args in ((Q.QD_GATE_X, 0, 2, (), ()), (Q.QD_GATE_X, 3, 1, (), ()), (Q.QD_GATE_X, 0, 1, (0,), (1,)),
                     (Q.QD_GATE_X, 0, 1, (1,), (3,)), (7, 0, 1, (), ())):
            with pytest.raises(Q.QDError):
                Q.qd_circuit_add(c, *args)
        assert Q.qd_circuit_size(c) == (3, 0)
        Q.qd_circuit_add(c, Q.QD_GATE_X, 2, 1, (0, 1), (1, 2))     # qudit 1 at 2 has no level 3
        with pytest.raises(Q.QDError) as e:
            Q.qd_circuit_decompose(c)
        assert e.value.code == Q.QD_EDIM
    finally:
        Q.qd_circuit_free(c)
