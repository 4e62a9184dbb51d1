"""GPU density matrices (qd_density_*) against the density oracle (full operators and matrix
products), and at benchmark size against the GPU state-vector path and properties that hold at any
size: trace, Hermiticity, purity and the fidelity of a noise-free evolution."""
import numpy as np
import pytest

import circuits as C
import oracle as O
from oracle import density as Dm
import paper_2211_07918_amd as Q
from gpu_util import torch_stream

pytestmark = pytest.mark.gpu

MAKERS = {Q.QD_CHANNEL_DEPOLARIZING: Dm.depolarizing, Q.QD_CHANNEL_DEPHASING: Dm.dephasing,
          Q.QD_CHANNEL_AMPLITUDE_DAMPING: Dm.amplitude_damping}


@pytest.fixture(scope="module")
def stream():
    return torch_stream()


def download_rho(rho, dims):
    D = int(np.prod(dims))
    return Q.qd_state_download(rho).reshape(D, D)


def noisy_program(dims, ngates, rng, p=0.08):
    """Gates from the random-circuit sampler, each followed by a named channel on its first target;
    every fifth step a joint two-qudit channel (products of one-qudit Kraus sets)."""
    circ = C.random_circuit(dims, ngates, rng, max_targets=2, max_controls=2)
    prog = []
    kinds = list(MAKERS)
    for i, g in enumerate(circ.gates):
        prog.append(("gate", g))
        q = g.targets[0]
        kind = kinds[int(rng.integers(3))]
        prog.append(("chan", (q,), kind, p))
        if i % 5 == 4 and len(dims) > 1:
            a, b = [int(x) for x in rng.choice(len(dims), 2, replace=False)]
            if dims[a] * dims[b] <= 32:
                prog.append(("joint", (a, b), p))
    return prog


def run_oracle(dims, prog, rho):
    for op in prog:
        if op[0] == "gate":
            g = op[1]
            rho = Dm.apply_unitary(rho, dims, g.targets, g.controls, g.cvals, O.gate_unitary(g, dims))
        elif op[0] == "chan":
            _, t, kind, p = op
            rho = Dm.apply_channel(rho, dims, t, MAKERS[kind](dims[t[0]], p))
        else:
            _, (a, b), p = op
            ks = [np.kron(x, y) for x in Dm.dephasing(dims[a], p) for y in Dm.depolarizing(dims[b], p)]
            rho = Dm.apply_channel(rho, dims, (a, b), ks)
    return rho


def run_gpu(dims, prog, rho_h):
    for op in prog:
        if op[0] == "gate":
            Q.apply_circuit_gate_density(rho_h, op[1], dims)
        elif op[0] == "chan":
            _, t, kind, p = op
            Q.qd_density_apply_channel(rho_h, t, Q.qd_channel_kraus(kind, dims[t[0]], p))
        else:
            _, (a, b), p = op
            ka = Q.qd_channel_kraus(Q.QD_CHANNEL_DEPHASING, dims[a], p)
            kb = Q.qd_channel_kraus(Q.QD_CHANNEL_DEPOLARIZING, dims[b], p)
            Q.qd_density_apply_channel(rho_h, (a, b), [np.kron(x, y) for x in ka for y in kb])


@pytest.mark.parametrize("seed", range(6))
def test_noisy_circuits_match_the_oracle(stream, seed):
    rng = np.random.default_rng(600 + seed)
    dims = tuple(int(x) for x in rng.integers(2, 5, size=int(rng.integers(2, 5))))
    prog = noisy_program(dims, 12, rng)
    want = run_oracle(dims, prog, Dm.from_state(O.basis_state(dims)))
    rho = Q.qd_density_init(dims, Q.QD_C128, stream)
    try:
        run_gpu(dims, prog, rho)
        got = download_rho(rho, dims)
        assert np.max(np.abs(got - want)) <= 1e-12
        assert abs(Q.qd_density_trace(rho) - Dm.trace(want)) <= 1e-13
        assert np.max(np.abs(Q.qd_density_probabilities(rho) - Dm.probabilities(want))) <= 1e-13
        assert abs(Q.qd_density_purity(rho) - Dm.purity(want)) <= 1e-12
    finally:
        Q.qd_state_free(rho)


def test_from_state_and_fidelity(stream):
    rng = np.random.default_rng(7)
    dims = (3, 2, 4, 2)
    D = int(np.prod(dims))
    psi0 = C.random_basis_superposition(D, 20, rng)
    circ = C.random_circuit(dims, 10, rng)
    psi = O.run_circuit(circ, psi0)
    s = Q.qd_state_init(dims, Q.QD_C128, stream)
    rho = Q.qd_density_init(dims, Q.QD_C128, stream)
    try:
        Q.qd_state_upload(s, psi0)
        Q.qd_density_from_state(rho, s)
        assert np.max(np.abs(download_rho(rho, dims) - Dm.from_state(psi0))) <= 1e-15
        for g in circ.gates:
            Q.apply_circuit_gate_density(rho, g, dims)
        Q.qd_state_upload(s, psi)
        assert abs(Q.qd_density_fidelity(rho, s) - 1.0) <= 1e-12
        Q.qd_density_apply_channel(rho, (1,), Q.qd_channel_kraus(Q.QD_CHANNEL_DEPOLARIZING, 2, 0.5))
        want = Dm.apply_channel(Dm.from_state(psi), dims, (1,), Dm.depolarizing(2, 0.5))
        assert abs(Q.qd_density_fidelity(rho, s) - Dm.fidelity(want, psi)) <= 1e-12
    finally:
        Q.qd_state_free(s)
        Q.qd_state_free(rho)


def test_complex64_density(stream):
    rng = np.random.default_rng(8)
    dims = (2, 3, 3)
    prog = noisy_program(dims, 10, rng)
    want = run_oracle(dims, prog, Dm.from_state(O.basis_state(dims)))
    rho = Q.qd_density_init(dims, Q.QD_C64, stream)
    try:
        run_gpu(dims, prog, rho)
        assert np.max(np.abs(download_rho(rho, dims) - want)) <= 1e-6
    finally:
        Q.qd_state_free(rho)


def test_errors(stream):
    dims = (2, 3)
    rho = Q.qd_density_init(dims, Q.QD_C128, stream)
    s = Q.qd_state_init((3, 2), Q.QD_C128, stream)
    try:
        bad = [0.5 * np.eye(2, dtype=np.complex128)]                 # not trace preserving
        with pytest.raises(Q.QDError) as e:
            Q.qd_density_apply_channel(rho, (0,), bad)
        assert e.value.code == Q.QD_ENOTUNITARY
        Q.qd_density_apply_channel(rho, (0,), bad, Q.QD_FLAG_SKIP_UNITARY_CHECK)   # allowed when asked
        assert abs(Q.qd_density_trace(rho) - 0.25) <= 1e-15
        with pytest.raises(Q.QDError) as e:
            Q.qd_density_from_state(rho, s)                            # other register
        assert e.value.code == Q.QD_EDIM
        with pytest.raises(Q.QDError):
            Q.qd_density_apply_channel(s, (0,), [np.eye(3)])           # not a density matrix
        with pytest.raises(Q.QDError):
            Q.qd_density_apply_gate(rho, (0,), (0,), (1,), O.x_gate(2))  # control repeats the target
    finally:
        Q.qd_state_free(rho)
        Q.qd_state_free(s)


def test_channel_dimension_limit(stream):
    dims = (4, 3, 3)
    rho = Q.qd_density_init(dims, Q.QD_C128, stream)
    try:
        ks = [np.eye(36, dtype=np.complex128)]
        with pytest.raises(Q.QDError) as e:             # d_T = 36 > 32
            Q.qd_density_apply_channel(rho, (0, 1, 2), ks)
        assert e.value.code == Q.QD_EDIM
    finally:
        Q.qd_state_free(rho)


def test_benchmark_size_pure_and_noisy(stream):
    """7 qubits + 4 qutrits (D = 10,368, 1.07e8 elements): a noise-free evolution of a random
    superposition must stay pure and give fidelity 1 with the GPU state-vector result; with
    depolarizing noise after every gate the trace stays 1 and the purity drops."""
    rng = C.seeded_rng(1007)
    dims = (2,) * 7 + (3,) * 4
    D = int(np.prod(dims))
    circ = C.random_circuit(dims, 30, rng, max_targets=1, max_controls=1)
    psi0 = C.random_basis_superposition(D, 64, rng)
    s = Q.qd_state_init(dims, Q.QD_C128, stream)
    rho = Q.qd_density_init(dims, Q.QD_C128, stream)
    try:
        Q.qd_state_upload(s, psi0)
        Q.qd_density_from_state(rho, s)
        for g in circ.gates:
            Q.apply_circuit_gate(s, g, dims)
            Q.apply_circuit_gate_density(rho, g, dims)
        assert abs(Q.qd_density_fidelity(rho, s) - 1.0) <= 1e-10
        assert abs(Q.qd_density_purity(rho) - 1.0) <= 1e-10
        for g in circ.gates[:10]:
            t = g.targets[0]
            Q.qd_density_apply_channel(rho, (t,), Q.qd_channel_kraus(Q.QD_CHANNEL_DEPOLARIZING, dims[t], 0.05))
        tr = Q.qd_density_trace(rho)
        assert abs(tr - 1.0) <= 1e-12
        pur = Q.qd_density_purity(rho)
        assert 1.0 / D <= pur < 1.0 - 1e-3
        p = Q.qd_density_probabilities(rho)
        assert np.min(p) >= -1e-15 and abs(np.sum(p) - 1.0) <= 1e-12
    finally:
        Q.qd_state_free(s)
        Q.qd_state_free(rho)


def test_operation_sequences_fuse_and_match(stream):
    """qd_density_apply_ops composes runs of uncontrolled operations on the same targets into one
    superoperator; the result matches the oracle and the one-by-one calls."""
    rng = np.random.default_rng(31)
    dims = (3, 2, 3, 2)
    circ = C.random_circuit(dims, 16, rng, max_targets=1, max_controls=1)
    ops = []
    for g in circ.gates:
        ops.append(("gate", g))
        t = g.targets[0]
        ops.append(("chan", (t,), Q.qd_channel_kraus(Q.QD_CHANNEL_DEPOLARIZING, dims[t], 0.1)))
        ops.append(("chan", (t,), Q.qd_channel_kraus(Q.QD_CHANNEL_AMPLITUDE_DAMPING, dims[t], 0.05)))
    want = Dm.from_state(O.basis_state(dims))
    for o in ops:
        if o[0] == "gate":
            g = o[1]
            want = Dm.apply_unitary(want, dims, g.targets, g.controls, g.cvals, O.gate_unitary(g, dims))
        else:
            want = Dm.apply_channel(want, dims, o[1], o[2])
    a = Q.qd_density_init(dims, Q.QD_C128, stream)
    b = Q.qd_density_init(dims, Q.QD_C128, stream)
    try:
        Q.qd_density_apply_ops(a, ops)
        for o in ops:
            if o[0] == "gate":
                Q.apply_circuit_gate_density(b, o[1], dims)
            else:
                Q.qd_density_apply_channel(b, o[1], o[2])
        ga, gb = download_rho(a, dims), download_rho(b, dims)
        assert np.max(np.abs(ga - want)) <= 1e-12 and np.max(np.abs(gb - want)) <= 1e-12
        bad = ops[:3] + [("chan", (0,), [0.5 * np.eye(3)])]              # rejected before any work
        with pytest.raises(Q.QDError) as e:
            Q.qd_density_apply_ops(a, bad)
        assert e.value.code == Q.QD_ENOTUNITARY
        assert np.array_equal(download_rho(a, dims), ga)
    finally:
        Q.qd_state_free(a)
        Q.qd_state_free(b)


@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
def test_runs_across_targets_compose_and_match(stream, prec):
    """Consecutive operations whose targets and controls together span qudits of dimension <= 4 (two
    qubits here) are one composed pass: controlled shifts, a controlled phase, a controlled dense
    gate, channels on either qubit and gates on the other, each run embedded on the pair. Against
    the oracle and against the same operations applied one call at a time. complex64: each pass
    rounds a superoperator of side <= 16 and the elements to 24 bits, so at most one pass per
    operation keeps the max-abs error below 4 x ops x 16 x 2^-24."""
    rng = np.random.default_rng(32)
    dims = (2, 3, 2, 2)
    G = C.Gate
    dep = lambda d, p: Q.qd_channel_kraus(Q.QD_CHANNEL_DEPOLARIZING, d, p)
    amp = lambda d, p: Q.qd_channel_kraus(Q.QD_CHANNEL_AMPLITUDE_DAMPING, d, p)
    ops = [("gate", G("U", (0,), U=C.haar_unitary(2, rng))), ("gate", G("U", (1,), U=C.haar_unitary(3, rng))),
           ("gate", G("U", (3,), U=C.haar_unitary(2, rng))),
           ("gate", G("X", (0,), (2,), (1,), a=1)), ("chan", (0,), dep(2, 0.1)),          # CX + its channel
           ("chan", (2,), amp(2, 0.2)), ("gate", G("U", (2,), U=C.haar_unitary(2, rng))),  # the other qubit
           ("gate", G("Z", (3,), (0,), (0,))), ("chan", (3,), dep(2, 0.05)),            # controlled phase
           ("gate", G("U", (2,), (3,), (1,), U=C.haar_unitary(2, rng))),                # controlled dense
           ("chan", (2,), amp(2, 0.3)), ("chan", (3,), dep(2, 0.2)),
           ("gate", G("X", (1,), (0,), (1,), a=2)), ("chan", (1,), dep(3, 0.1)),        # qubit-qutrit: span 6
           ("gate", G("U", (0, 3), U=C.haar_unitary(4, rng))), ("chan", (0,), amp(2, 0.1))]
    want = Dm.from_state(O.basis_state(dims))
    for o in ops:
        if o[0] == "gate":
            g = o[1]
            want = Dm.apply_unitary(want, dims, g.targets, g.controls, g.cvals, O.gate_unitary(g, dims))
        else:
            want = Dm.apply_channel(want, dims, o[1], o[2])
    tol = 1e-12 if prec == Q.QD_C128 else 4.0 * len(ops) * 16 * 2.0 ** -24
    a = Q.qd_density_init(dims, prec, stream)
    b = Q.qd_density_init(dims, prec, stream)
    try:
        Q.qd_density_apply_ops(a, ops)
        for o in ops:
            if o[0] == "gate":
                Q.apply_circuit_gate_density(b, o[1], dims)
            else:
                Q.qd_density_apply_channel(b, o[1], o[2])
        ga, gb = download_rho(a, dims), download_rho(b, dims)
        assert np.max(np.abs(ga - want)) <= tol and np.max(np.abs(gb - want)) <= tol
        assert abs(np.trace(ga) - 1.0) <= tol
        # the runs were composed: one pass per run of operations spanning dimension <= 4, against
        # one or two passes per operation when applied one call at a time
        composed, single = expected_passes(ops, dims)
        assert (composed, single) == (10, 19)
        assert Q.qd_state_gate_launches(a) == composed and Q.qd_state_gate_launches(b) == single
    finally:
        Q.qd_state_free(a)
        Q.qd_state_free(b)


def expected_passes(ops, dims):
    """Passes of qd_density_apply_ops and of one call per operation, by the documented rules: a
    run of two or more consecutive operations whose qudits span dimension <= 4 is one pass; alone,
    a channel is one pass, a gate one pass when diagonal with d_G <= 4 or uncontrolled with
    d_T <= 4, else two."""
    def qudits(o):
        return set(o[1].targets) | set(o[1].controls) if o[0] == "gate" else set(o[1])

    def span(qs):
        return int(np.prod([dims[q] for q in qs])) if qs else 1

    def alone(o):
        if o[0] != "gate":
            return 1
        g = o[1]
        dT = span(g.targets)
        dG = dT * span(g.controls)
        diag = Q.qd_gate_class(Q.gate_unitary(g, dims)) == Q.QD_CLASS_DIAGONAL
        return 1 if (diag and dG <= 4) or (not g.controls and dT <= 4) else 2

    composed, i = 0, 0
    while i < len(ops):
        qs, j = qudits(ops[i]), i + 1
        if span(qs) <= 4:
            while j < len(ops) and span(qs | qudits(ops[j])) <= 4:
                qs |= qudits(ops[j])
                j += 1
        composed += alone(ops[i]) if j - i == 1 else 1
        i = j
    return composed, sum(alone(o) for o in ops)
