"""GPU parity of the plain gate path (qd_apply_gate) against the oracle, through the C ABI.

Tolerances:
  * complex128: max-abs amplitude error <= 1e-12 (the bound the method is held to);
  * complex64: each gate adds at most ~ c d_T 2^-24 to the 2-norm error of a unit state (U and
    the state rounded to FP32, d_T products summed with fused multiply-adds), so G gates stay
    below 4 G d_T,max 2^-24 in the 2-norm and therefore in max-abs; fidelity loss <= 1e-6.
"""
import math

import numpy as np
import pytest

import circuits as C
import oracle as O
import paper_2211_07918_amd as Q
from gpu_util import fidelity_loss, max_abs, read_amplitudes, run_gpu, torch_stream

pytestmark = pytest.mark.gpu

U24 = 2.0 ** -24


def c64_tol(ngates, dmax):
    return 4.0 * ngates * dmax * U24


@pytest.fixture(scope="module")
def stream():
    return torch_stream()


# ------------------------------------------------------------------------------ paper example
def test_worked_example_bit_exact(stream):
    """Sec. 3.9 worked example: exactly 0.7071067811865475 at |000> and |120>."""
    circ = C.Circuit((2, 3, 3), [C.Gate("F", (0,)), C.Gate("X", (1,), (0,), (1,), a=2)])
    psi = run_gpu(circ, Q.QD_C128, stream)
    want = np.zeros(18, np.complex128)
    want[0] = want[15] = 0.7071067811865475
    assert np.array_equal(psi, want)


def test_config0_vs_bruteforce(stream):
    c = C.config0()
    psi = run_gpu(c, Q.QD_C128, stream)
    assert max_abs(psi, O.run_circuit_operator(c)) <= 1e-12
    assert max_abs(psi, O.run_circuit(c)) <= 1e-12
    p = Q.qd_probabilities(_state_of(c, stream))
    assert np.max(np.abs(p - O.probabilities(O.run_circuit(c)))) <= 1e-12


def _state_of(c, stream, prec=Q.QD_C128):
    """State handle after running c (caller frees via the module finalizer list)."""
    s = Q.qd_state_init(c.dims, prec, stream)
    _OPEN.append(s)
    for g in c.gates:
        Q.apply_circuit_gate(s, g, c.dims)
    return s


_OPEN = []


@pytest.fixture(autouse=True, scope="module")
def _free_states():
    yield
    for s in _OPEN:
        Q.qd_state_free(s)
    _OPEN.clear()


def test_config0_complex64(stream):
    c = C.config0()
    psi = run_gpu(c, Q.QD_C64, stream)
    ref = O.run_circuit(c)
    assert max_abs(psi, ref) <= c64_tol(len(c.gates), 3)
    assert fidelity_loss(ref, psi) <= 1e-6


def test_config1_shrink_500_gates(stream):
    c = C.config1_shrink()
    assert c.D == 10368 and len(c.gates) == 500
    assert max_abs(run_gpu(c, Q.QD_C128, stream), O.run_circuit(c)) <= 1e-12


@pytest.mark.parametrize("run_min", [1, 1024])
def test_config1_shrink_forced_routes(stream, run_min):
    """Same circuit with every gate forced to the direct kernel (run_min 1) or to the LDS tile
    kernel wherever a tile fits (run_min 1024)."""
    c = C.config1_shrink(200)
    Q.qd_tune_set(Q.QD_TUNE_RUN_MIN, run_min)
    try:
        psi = run_gpu(c, Q.QD_C128, stream)
    finally:
        Q.qd_tune_set(Q.QD_TUNE_RUN_MIN, 0)
    assert max_abs(psi, O.run_circuit(c)) <= 1e-12


RANDOM_REGS = [(2, 3, 4, 3, 2), (3, 3, 3, 3, 3, 3, 3), (4, 2, 5, 2, 3, 2), (2,) * 12, (7, 5, 3, 2, 11),
               (3, 2, 2, 4, 2, 3, 2, 2, 3), (5, 5, 5, 5)]


@pytest.mark.parametrize("dims", RANDOM_REGS)
@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
def test_random_circuits(stream, dims, prec):
    rng = C.seeded_rng(hash(dims) % 10000)
    c = C.random_circuit(dims, 60, rng, max_targets=2, max_controls=2, max_dT=16)
    c.init_amps = C.random_basis_superposition(O.register_size(dims), 9, rng)
    psi = run_gpu(c, prec, stream)
    ref = O.run_circuit(c)
    if prec == Q.QD_C128:
        assert max_abs(psi, ref) <= 1e-12
    else:
        assert max_abs(psi, ref) <= c64_tol(60, 16)
        assert fidelity_loss(ref, psi) <= 1e-6


def test_every_route_is_exercised(stream):
    """One gate per kernel family and precision, each checked against the oracle."""
    dims = (3, 2, 4, 3, 2, 2, 3, 2, 2, 2)
    rng = C.seeded_rng(5)
    D = O.register_size(dims)
    psi0 = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    psi0 /= np.linalg.norm(psi0)
    cases = [
        ([0], (), (), C.haar_unitary(3, rng), Q.QD_ROUTE_DIRECT),
        ([9], (), (), C.haar_unitary(2, rng), Q.QD_ROUTE_TILED),
        ([6, 9], (0,), (2,), C.haar_unitary(6, rng), Q.QD_ROUTE_TILED),
        ([2, 0], (9,), (1,), C.haar_unitary(12, rng), Q.QD_ROUTE_DIRECT),
        ([2, 6], (), (), C.haar_unitary(12, rng), Q.QD_ROUTE_GEMM),
        ([9], (3,), (1,), O.z_gate(2), Q.QD_ROUTE_DIAG),
        ([2, 3], (), (), np.diag(np.exp(2j * np.pi * rng.random(12))), Q.QD_ROUTE_DIAG),
        ([1], (0,), (2,), O.x_gate(2, 1), Q.QD_ROUTE_DIRECT),
        ([2, 0], (), (), np.eye(12)[rng.permutation(12)] * np.exp(1j * rng.random(12)), Q.QD_ROUTE_DIRECT),
        ([8, 9], (), (), np.eye(4)[rng.permutation(4)], Q.QD_ROUTE_TILED),
        ([0, 1, 2], (9,), (0,), C.haar_unitary(24, rng), Q.QD_ROUTE_GEMM),
        ([9, 3, 0], (), (), C.haar_unitary(18, rng), Q.QD_ROUTE_GEMM),
        ([2, 3, 6], (0,), (1,), C.haar_unitary(36, rng), Q.QD_ROUTE_GEMM),
        ([0, 1, 2, 3], (), (), C.haar_unitary(72, rng), Q.QD_ROUTE_GENERIC),
    ]
    for prec in (Q.QD_C128, Q.QD_C64):
        for t, c, v, U, route in cases:
            if prec == Q.QD_C128:
                assert Q.qd_gate_route(dims, prec, t, c, v, U) == route, (t, c, route)
            s = Q.qd_state_init(dims, prec, stream)
            try:
                Q.qd_state_upload(s, psi0)
                Q.qd_apply_gate(s, t, c, v, U)
                out = Q.qd_state_download(s)
            finally:
                Q.qd_state_free(s)
            ref = O.apply_gate(psi0, dims, t, c, v, U)
            tol = 1e-12 if prec == Q.QD_C128 else c64_tol(1, U.shape[0])
            assert max_abs(out, ref) <= tol, (t, c, route, prec)


@pytest.mark.parametrize("dims,targets", [((4, 4, 4, 2), [0, 1]), ((2, 2, 2, 2, 2, 2, 2), [6, 0, 3, 2, 5]),
                                          ((3, 3, 3, 2), [2, 1, 0]), ((256,), [0]), ((2, 128, 2), [1, 2]),
                                          ((4, 4, 4, 4, 4), [0, 1, 2, 3, 4])])
def test_large_gates_generic(stream, dims, targets):
    rng = C.seeded_rng(77)
    dT = int(np.prod([dims[t] for t in targets]))
    c = C.Circuit(dims, [C.Gate("U", tuple(targets), U=C.haar_unitary(dT, rng))],
                  init_amps=C.random_basis_superposition(O.register_size(dims), 5, rng))
    assert max_abs(run_gpu(c, Q.QD_C128, stream), O.run_circuit(c)) <= 1e-12


@pytest.mark.parametrize("dims", [(2,), (7,), (256,), (2, 2), (3, 5)])
def test_tiny_registers(stream, dims):
    rng = C.seeded_rng(9)
    gates = [C.Gate("F", (0,)), C.Gate("Z", (0,)), C.Gate("X", (0,), a=1),
             C.Gate("U", (0,), U=C.haar_unitary(dims[0], rng))]
    if len(dims) == 2:
        gates += [C.Gate("X", (1,), (0,), (1,), a=1), C.Gate("U", (0, 1), U=C.haar_unitary(dims[0] * dims[1], rng)),
                  C.Gate("U", (1,), (0,), (0,), U=C.haar_unitary(dims[1], rng))]
    c = C.Circuit(dims, gates)
    assert max_abs(run_gpu(c, Q.QD_C128, stream), O.run_circuit(c)) <= 1e-12


def test_all_qudits_targeted_or_controlled(stream):
    dims = (3, 2, 3)
    rng = C.seeded_rng(10)
    gates = [C.Gate("U", (0, 1, 2), U=C.haar_unitary(18, rng)),      # no free qudit
             C.Gate("U", (2,), (0, 1), (2, 1), U=C.haar_unitary(3, rng)),  # a single slice
             C.Gate("X", (1,), (0, 2), (0, 0), a=1), C.Gate("Z", (0,), (1, 2), (1, 2))]
    c = C.Circuit(dims, gates, init_amps=C.random_basis_superposition(18, 18, rng))
    assert max_abs(run_gpu(c, Q.QD_C128, stream), O.run_circuit(c)) <= 1e-12
    assert max_abs(run_gpu(c, Q.QD_C64, stream), O.run_circuit(c)) <= c64_tol(4, 18)


@pytest.mark.parametrize("param,values", [(Q.QD_TUNE_TILE_ELEMS, [256, 1024, 4096]),
                                          (Q.QD_TUNE_TILE_BLOCK, [64, 128]),
                                          (Q.QD_TUNE_DIRECT_BLOCK, [64, 192]),
                                          (Q.QD_TUNE_DIRECT_SPT, [1, 4]),
                                          (Q.QD_TUNE_DIAG_BLOCK, [64])])
def test_tuning_parameters_keep_results(stream, param, values):
    dims = (3, 2, 2, 4, 2, 3, 2, 2, 3)
    rng = C.seeded_rng(11)
    c = C.random_circuit(dims, 40, rng, max_dT=12)
    ref = O.run_circuit(c)
    for v in values:
        Q.qd_tune_set(param, v)
        try:
            assert max_abs(run_gpu(c, Q.QD_C128, stream), ref) <= 1e-12, (param, v)
        finally:
            Q.qd_tune_set(param, 0)


def test_wrap_torch_tensor(stream):
    import torch
    c = C.config0()
    t = torch.zeros(2 * c.D, dtype=torch.float64, device="cuda")
    s = Q.qd_state_wrap(c.dims, Q.QD_C128, t.data_ptr(), t.numel() * 8, stream)
    try:
        Q.qd_state_set_basis(s, [0] * 6)
        for g in c.gates:
            Q.apply_circuit_gate(s, g, c.dims)
        Q.qd_state_sync(s)
        host = t.cpu().numpy().view(np.complex128)
        assert max_abs(host, O.run_circuit(c)) <= 1e-12
        assert Q.qd_state_device_ptr(s) == t.data_ptr()
    finally:
        Q.qd_state_free(s)
    assert torch.count_nonzero(t).item() > 0      # the library did not free torch's memory
    with pytest.raises(Q.QDError) as e:
        Q.qd_state_wrap(c.dims, Q.QD_C128, t.data_ptr(), 100, stream)
    assert e.value.code == Q.QD_EDIM


def test_set_basis_upload_download(stream):
    dims = (2, 3, 4)
    s = Q.qd_state_init(dims, Q.QD_C128, stream)
    try:
        Q.qd_state_set_basis(s, [1, 2, 3])
        psi = Q.qd_state_download(s)
        assert np.array_equal(psi, O.basis_state(dims, [1, 2, 3]))
        v = np.arange(24) + 1j * np.arange(24)[::-1]
        Q.qd_state_upload(s, v)
        assert np.array_equal(Q.qd_state_download(s), v)
        with pytest.raises(Q.QDError) as e:
            Q.qd_state_set_basis(s, [2, 0, 0])
        assert e.value.code == Q.QD_EINVAL
    finally:
        Q.qd_state_free(s)


def test_readout_probabilities_norm_compare(stream):
    import torch
    rng = C.seeded_rng(12)
    dims = (3, 4, 2, 5, 3)
    c = C.random_circuit(dims, 30, rng)
    ref = O.run_circuit(c)
    s = _state_of(c, stream)
    p = Q.qd_probabilities(s)
    assert np.max(np.abs(p - O.probabilities(ref))) <= 1e-13
    dev = torch.empty(c.D, dtype=torch.float64, device="cuda")
    Q.qd_probabilities(s, dev.data_ptr())
    torch.cuda.synchronize()
    assert np.array_equal(dev.cpu().numpy(), p)
    n1, n2 = Q.qd_norm2(s), Q.qd_norm2(s)
    assert n1 == n2 and abs(n1 - O.norm2(ref)) <= 1e-13
    s32 = _state_of(c, stream, Q.QD_C64)
    ma, fl, dr = Q.qd_compare(s, s32)
    psi32 = Q.qd_state_download(s32)
    oma, ofl, odr = O.compare(Q.qd_state_download(s), psi32)
    assert abs(ma - oma) <= 1e-15 and abs(fl - ofl) <= 1e-13 and abs(dr - odr) <= 1e-13
    with pytest.raises(Q.QDError) as e:
        Q.qd_compare(s32, s)
    assert e.value.code == Q.QD_EDIM


@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
def test_one_pass_probabilities_and_norm(stream, prec):
    """qd_probabilities_norm2 against the two separate passes (probabilities bitwise those of
    qd_probabilities, the norm bitwise that of qd_norm2, into host and device memory) and against
    FP64 arithmetic on the downloaded state; complex128 also against the oracle. Registers smaller
    than one workgroup, ragged, and larger than one round of the reduction grid (2048 workgroups of
    256 threads, 524,288 amplitudes)."""
    import torch
    for dims, ngates, seed in (((3,), 2, 31), ((3, 4, 2, 5, 3), 30, 32), ((3,) * 12 + (2,), 40, 33)):
        c = C.random_circuit(dims, ngates, C.seeded_rng(seed))
        s = _state_of(c, stream, prec)
        p_sep, n_sep = Q.qd_probabilities(s), Q.qd_norm2(s)
        p_one, n_one = Q.qd_probabilities_norm2(s)
        assert np.array_equal(p_one, p_sep) and n_one == n_sep, dims
        dev = torch.empty(c.D, dtype=torch.float64, device="cuda")
        none, n_dev = Q.qd_probabilities_norm2(s, dev.data_ptr())
        assert none is None and n_dev == n_sep
        assert np.array_equal(dev.cpu().numpy(), p_sep)
        psi = Q.qd_state_download(s).astype(np.complex128)
        p_host = psi.real ** 2 + psi.imag ** 2
        assert np.max(np.abs(p_one - p_host)) <= 4e-16 * max(1.0, float(np.max(p_host))), dims
        assert abs(n_one - float(np.sum(p_host))) <= 1e-12, dims
        if prec == Q.QD_C128:
            ref = O.run_circuit(c)
            assert np.max(np.abs(p_one - O.probabilities(ref))) <= 1e-13
            assert abs(n_one - O.norm2(ref)) <= 1e-12


def test_validation_leaves_state_unchanged(stream):
    dims = (2, 3, 4)
    rng = C.seeded_rng(13)
    s = Q.qd_state_init(dims, Q.QD_C128, stream)
    try:
        v = C.random_basis_superposition(24, 24, rng)
        Q.qd_state_upload(s, v)
        bad = [([1], [1], [0], O.x_gate(3, 1), Q.QD_EINVAL), ([1], [0], [2], O.x_gate(3, 1), Q.QD_EINVAL),
               ([1], [], [], np.ones((3, 3)), Q.QD_ENOTUNITARY), ([2], [], [], O.x_gate(3, 1), Q.QD_EDIM),
               ([7], [], [], O.x_gate(3, 1), Q.QD_EINVAL)]
        for t, c, cv, U, code in bad:
            with pytest.raises(Q.QDError) as e:
                Q.qd_apply_gate(s, t, c, cv, U)
            assert e.value.code == code
        assert np.array_equal(Q.qd_state_download(s), v)
    finally:
        Q.qd_state_free(s)


# ------------------------------------------------------------------------------ full size
def _digit_sim(dims, gates, digs):
    digs = list(digs)
    for g in gates:
        if all(digs[c] == v for c, v in zip(g.controls, g.cvals)):
            t = g.targets[0]
            digs[t] = (digs[t] + g.a) % dims[t]
    return digs


def test_config1_full_size_samples_and_norm(stream):
    """D = 107,495,424: sampled outputs of single gates (every route the workload takes) against
    the oracle evaluated one amplitude at a time, and the norm after all 500 gates."""
    c = C.config1()
    s = Q.qd_state_init(c.dims, Q.QD_C128, stream)
    try:
        for g in c.gates[:25]:
            Q.apply_circuit_gate(s, g, c.dims)
        rng = C.seeded_rng(14)
        n = len(c.dims)
        mid = n // 2
        probes = [C.Gate("U", (n - 1,), U=C.haar_unitary(c.dims[n - 1], rng)),
                  C.Gate("U", (0,), U=C.haar_unitary(c.dims[0], rng)),
                  C.Gate("U", (mid,), U=C.haar_unitary(c.dims[mid], rng)),
                  C.Gate("X", (mid,), (n - 1,), (1,), a=1),
                  C.Gate("X", (n - 1,), (0,), (0,), a=1)]
        for g in probes:
            before = Q.qd_state_download(s)
            Q.apply_circuit_gate(s, g, c.dims)
            after = Q.qd_state_download(s)
            idx = rng.choice(c.D, 3000, replace=False)
            want = O.apply_gate_at(before, c.dims, g.targets, g.controls, g.cvals, O.gate_unitary(g, c.dims), idx)
            assert max_abs(after[idx], want) <= 1e-12, g
            del before, after
        for g in c.gates[25:]:
            Q.apply_circuit_gate(s, g, c.dims)
        assert abs(Q.qd_norm2(s) - 1.0) <= 1e-12
    finally:
        Q.qd_state_free(s)


def test_config1_full_size_permutation_circuit(stream):
    """Permutation-only circuit on the full hybrid register: the basis state lands exactly on the
    index an integer digit simulation predicts."""
    c = C.config1()
    rng = C.seeded_rng(15)
    pc = C.permutation_circuit(c.dims, 300, rng)
    start = [int(rng.integers(d)) for d in c.dims]
    s = Q.qd_state_init(c.dims, Q.QD_C128, stream)
    try:
        Q.qd_state_set_basis(s, start)
        for g in pc.gates:
            Q.apply_circuit_gate(s, g, c.dims)
        psi = Q.qd_state_download(s)
    finally:
        Q.qd_state_free(s)
    end = O.index_of(_digit_sim(c.dims, pc.gates, start), c.dims)
    nz = np.flatnonzero(psi)
    assert list(nz) == [end] and psi[end] == 1.0


def test_config1_full_size_diagonal_closed_form(stream):
    c = C.config1()
    rng = C.seeded_rng(16)
    dc = C.diagonal_circuit(c.dims, 60, rng)
    psi0 = C.random_basis_superposition(c.D, 4096, rng)
    s = Q.qd_state_init(c.dims, Q.QD_C128, stream)
    try:
        Q.qd_state_upload(s, psi0)
        for g in dc.gates:
            Q.apply_circuit_gate(s, g, c.dims)
        psi = Q.qd_state_download(s)
    finally:
        Q.qd_state_free(s)
    idx = np.flatnonzero(psi0)
    st = O.strides(c.dims)
    want = []
    for x in idx:
        dg = [(int(x) // st[i]) % c.dims[i] for i in range(len(c.dims))]
        ang = sum(dg[g.targets[0]] / c.dims[g.targets[0]] for g in dc.gates
                  if all(dg[cc] == v for cc, v in zip(g.controls, g.cvals)))
        want.append(psi0[x] * complex(math.cos(2 * math.pi * ang), math.sin(2 * math.pi * ang)))
    assert max_abs(psi[idx], np.array(want)) <= 1e-12
    assert np.count_nonzero(psi) == len(idx)


@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
def test_gemm_route_sizes(stream, prec):
    """Dense gates of 10 <= d_T <= 64 run as a small GEMM per tile of slices: padded and unpadded d_T
    (10, 15, 16, 18, 20, 24, 28, 32, 64), with and without a control, on a register whose slice
    count leaves a ragged last tile; each result against the oracle."""
    dims = (2, 5, 3, 4, 7, 2, 3, 4, 2)
    rng = C.seeded_rng(91)
    D = O.register_size(dims)
    psi0 = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    psi0 /= np.linalg.norm(psi0)
    cases = [((0, 1), (), ()), ((2, 1), (0,), (1,)), ((3, 1), (), ()), ((4, 3), (8,), (0,)),
             ((3, 7, 0), (), ()), ((8, 3, 6), (2,), (2,)), ((3, 7, 5, 0), (), ()), ((3, 7), (1,), (4,)),
             ((2, 6, 8), (), ())]
    for t, c, v in cases:
        dT = int(np.prod([dims[q] for q in t]))
        U = C.haar_unitary(dT, rng)
        assert Q.qd_gate_route(dims, prec, t, c, v, U) == (Q.QD_ROUTE_GEMM if 10 <= dT <= 64 else Q.QD_ROUTE_DIRECT), (t, dT)
        s = Q.qd_state_init(dims, prec, stream)
        try:
            Q.qd_state_upload(s, psi0)
            Q.qd_apply_gate(s, t, c, v, U)
            out = Q.qd_state_download(s)
        finally:
            Q.qd_state_free(s)
        ref = O.apply_gate(psi0, dims, t, c, v, U)
        tol = 1e-12 if prec == Q.QD_C128 else c64_tol(1, dT)
        assert max_abs(out, ref) <= tol, (t, c, dT, prec)


@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
def test_dense_12_16_one_slice_per_thread(stream, prec):
    """Dense gates of d_T = 12 and 16 whose targets all have large strides run one slice per thread
    with U in LDS (route DIRECT), with and without a control; each against the oracle."""
    dims = (4, 3, 4, 2, 3, 2, 2, 2, 3, 2)
    rng = C.seeded_rng(92)
    D = O.register_size(dims)
    psi0 = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    psi0 /= np.linalg.norm(psi0)
    for t, c, v in (((0, 1), (), ()), ((1, 2), (3,), (1,)), ((0, 2), (), ()), ((2, 0), (4,), (2,))):
        dT = int(np.prod([dims[q] for q in t]))
        U = C.haar_unitary(dT, rng)
        assert Q.qd_gate_route(dims, prec, t, c, v, U) == Q.QD_ROUTE_DIRECT, (t, dT)
        s = Q.qd_state_init(dims, prec, stream)
        try:
            Q.qd_state_upload(s, psi0)
            Q.qd_apply_gate(s, t, c, v, U)
            out = Q.qd_state_download(s)
        finally:
            Q.qd_state_free(s)
        ref = O.apply_gate(psi0, dims, t, c, v, U)
        tol = 1e-12 if prec == Q.QD_C128 else c64_tol(1, dT)
        assert max_abs(out, ref) <= tol, (t, c, dT, prec)


@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
@pytest.mark.parametrize("tile_elems", [256, 0, 4096])
def test_tiled_controls_inside_the_suffix(stream, prec, tile_elems):
    """Low-stride targets whose controls sit inside the LDS tile's contiguous suffix: controls of at
    least one 128-byte line of stride are left out of the tile (one or two of them, a third stays
    outside the tile), a control below one line stays inside it, each case against the oracle."""
    dims = (3, 2, 2, 4, 2, 3, 2, 2, 3, 2, 3)          # strides 6912 ... 18, 6, 3, 1
    rng = C.seeded_rng(93)
    D = O.register_size(dims)
    psi0 = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    psi0 /= np.linalg.norm(psi0)
    cases = [
        ((10,), (7,), (1,)),                 # control stride 18: not a whole number of lines
        ((10,), (6,), (0,)),                 # stride 36
        ((9,), (7, 5), (1, 2)),              # two controls inside the suffix
        ((10,), (7, 6, 5), (0, 1, 1)),       # three: the third stays above the tile
        ((10, 4), (7,), (1,)),               # a high target (two runs per tile) and a control inside
        ((8,), (4, 2), (1, 0)),              # controls of strides 216 and 1728
        ((10,), (8,), (2,)),                 # stride 6, inside a line
        ((9,), (8, 7), (0, 1)),              # stride 6 inside the tile and stride 18 left out
    ]
    dims9 = (2, 3, 2, 4, 2, 9, 3)                     # a 9-level target over a qutrit of stride 1
    D9 = O.register_size(dims9)
    psi9 = rng.standard_normal(D9) + 1j * rng.standard_normal(D9)
    psi9 /= np.linalg.norm(psi9)
    cases9 = [((5,), (6,), (2,)), ((5,), (6, 3), (1, 2)), ((5,), (3, 6), (0, 0))]
    Q.qd_tune_set(Q.QD_TUNE_TILE_ELEMS, tile_elems)
    try:
        for reg, x0, cs in ((dims, psi0, cases), (dims9, psi9, cases9)):
            for t, c, v in cs:
                dT = int(np.prod([reg[q] for q in t]))
                for U in (C.haar_unitary(dT, rng), O.x_gate(dT, 1) if len(t) == 1 else np.eye(dT)[::-1]):
                    assert Q.qd_gate_route(reg, prec, t, c, v, U) == Q.QD_ROUTE_TILED, (reg, t, c)
                    s = Q.qd_state_init(reg, prec, stream)
                    try:
                        Q.qd_state_upload(s, x0)
                        Q.qd_apply_gate(s, t, c, v, U)
                        out = Q.qd_state_download(s)
                    finally:
                        Q.qd_state_free(s)
                    ref = O.apply_gate(x0, reg, t, c, v, U)
                    tol = 1e-12 if prec == Q.QD_C128 else c64_tol(1, dT)
                    assert max_abs(out, ref) <= tol, (reg, t, c, prec, tile_elems)
    finally:
        Q.qd_tune_set(Q.QD_TUNE_TILE_ELEMS, 0)


@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
def test_tiled_kernel_walks_tiles_beyond_the_grid_cap(stream, prec):
    """A launch of more than 2^22 LDS tiles: the workgroups (at most 2^22) each walk two tiles. The
    register (23 qubits, a 200-level qudit, a qubit; D = 3,355,443,200, 54 GB per complex128 state)
    with a tile budget of 512 complex128 amplitudes (256 for complex64, whose budget is doubled)
    stages runs of 2 x 200 = 400 amplitudes for a gate on the last qubit, so the launch covers
    D / 400 = 8,388,608 tiles. The same gate through the direct kernel (run_min 1) on a complex128
    state prepared the same way is the reference: equal FP64 arithmetic for complex128, the
    complex64 bound of five gates otherwise; and the oracle at sampled outputs (the prepared state
    is a product state the oracle evaluates amplitude by amplitude)."""
    dims = (2,) * 23 + (200, 2)
    n = len(dims)
    D = O.register_size(dims)
    assert D == 3355443200 and D // 400 > 2 ** 22
    rng = C.seeded_rng(94)
    V = C.haar_unitary(2, rng)
    prep = [((0,), C.haar_unitary(2, rng)), ((11,), C.haar_unitary(2, rng)), ((22,), C.haar_unitary(2, rng)),
            ((n - 1,), C.haar_unitary(2, rng))]
    states = []
    try:
        for p in (prec, Q.QD_C128):
            s = Q.qd_state_init(dims, p, stream)
            states.append(s)
            Q.qd_state_set_basis(s, [0] * n)
        Q.qd_tune_set(Q.QD_TUNE_RUN_MIN, 1)
        try:
            for s in states:
                for t, U in prep:
                    Q.qd_apply_gate(s, t, (), (), U)
            Q.qd_apply_gate(states[1], (n - 1,), (), (), V)           # direct kernel
        finally:
            Q.qd_tune_set(Q.QD_TUNE_RUN_MIN, 0)
        Q.qd_tune_set(Q.QD_TUNE_TILE_ELEMS, 512 if prec == Q.QD_C128 else 256)
        try:
            assert Q.qd_gate_route(dims, prec, (n - 1,), (), (), V) == Q.QD_ROUTE_TILED
            Q.qd_apply_gate(states[0], (n - 1,), (), (), V)           # tile kernel, 8.4M tiles
        finally:
            Q.qd_tune_set(Q.QD_TUNE_TILE_ELEMS, 0)
        err, fid, drift = Q.qd_compare(states[1], states[0])
        tol = 1e-12 if prec == Q.QD_C128 else c64_tol(len(prep) + 1, 2)
        assert err <= tol and abs(fid) <= max(tol, 1e-12) and drift <= max(tol, 1e-12), (err, fid, drift)
        # The oracle at sampled outputs of the tile kernel: the prepared state is the product of
        # each prepared qubit's U|0> (|0> elsewhere), evaluated amplitude by amplitude; samples
        # include the ends of the state and of tiles in both rounds of the workgroups' walk.
        phi = {t[0]: U[:, 0] for t, U in prep}

        class Prepared:
            def __getitem__(self, i):
                dg = O.digits_of(int(i), dims)
                return complex(np.prod([phi[q][dg[q]] if q in phi else (1.0 if dg[q] == 0 else 0.0)
                                        for q in range(n)]))

        T = D // 400
        idx = list(rng.choice(D, 600, replace=False))
        for t in (0, 1, 2 ** 22 - 1, 2 ** 22, 2 ** 22 + 1, T - 1):
            idx += [t * 400, t * 400 + 1, t * 400 + 199, t * 400 + 200, t * 400 + 399]
        st = O.strides(dims)
        idx += [D - 1] + [a * st[0] + b * st[11] + c * st[22] + e
                          for a in (0, 1) for b in (0, 1) for c in (0, 1) for e in (0, 1)]
        want = O.apply_gate_at(Prepared(), dims, (n - 1,), (), (), V, idx)
        got = read_amplitudes(states[0], prec, idx)
        assert max_abs(got, want) <= tol, max_abs(got, want)
    finally:
        for s in states:
            Q.qd_state_free(s)


@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
def test_direct_controls_whole_lines(stream, prec):
    """Controlled gates on the slice-per-thread kernel where the control's active runs do not
    cover whole 128-byte lines: controls of stride below one line (tested per slice, every slice of a
    line holding an active amplitude written, lines with none left untouched: the stride-6 qutrit
    controls leave a third of the lines inactive), and a lowest control whose stride is not a whole
    number of lines (edge lanes rewrite
    the rest of the partly active lines): targets above and below the control, two controls, the
    last line of a register whose size is no multiple of a line, dense and monomial U, each
    against the oracle."""
    line = 8 if prec == Q.QD_C128 else 16
    regs = {
        # strides 4320, 2160, 540, 180, 90, 18, 6, 3, 1 (D = 12960)
        (3, 2, 4, 3, 2, 5, 3, 2, 3): [
            ((0,), (8,), (2,)), ((2,), (7,), (1,)), ((3,), (6, 8), (1, 0)), ((1,), (6, 4), (2, 1)),
            ((5,), (7,), (1,)), ((0,), (5,), (2,)), ((2,), (4,), (1,)), ((5,), (3,), (0,)),
            ((1, 4), (3,), (1,)), ((0,), (5, 3), (1, 2)), ((0,), (2,), (3,)), ((0,), (1,), (1,)),
            ((4, 1), (5,), (4,)), ((0,), (6,), (2,)), ((2,), (6, 7), (0, 1)),
        ],
        # strides 135, 45, 9, 3, 1 (D = 405: the last line is partial)
        (3, 3, 5, 3, 3): [((0,), (2,), (4,)), ((1,), (2,), (0,)), ((0,), (1,), (2,)), ((0, 1), (2,), (3,))],
    }
    rng = C.seeded_rng(97)
    seen = set()
    for dims, cases in regs.items():
        D = O.register_size(dims)
        st = O.strides(dims)
        psi0 = rng.standard_normal(D) + 1j * rng.standard_normal(D)
        psi0 /= np.linalg.norm(psi0)
        for t, c, v in cases:
            dT = int(np.prod([dims[q] for q in t]))
            low = min(st[q] for q in c)
            kind = "pred" if low < line else ("edge" if low % line else "aligned")
            seen.add(kind)
            mono = np.eye(dT)[np.roll(np.arange(dT), 1)] * np.exp(1j * rng.random(dT))
            for U in (C.haar_unitary(dT, rng), mono):
                assert Q.qd_gate_route(dims, prec, t, c, v, U) == Q.QD_ROUTE_DIRECT, (dims, t, c)
                s = Q.qd_state_init(dims, prec, stream)
                try:
                    Q.qd_state_upload(s, psi0)
                    Q.qd_apply_gate(s, t, c, v, U)
                    out = Q.qd_state_download(s)
                finally:
                    Q.qd_state_free(s)
                ref = O.apply_gate(psi0, dims, t, c, v, U)
                tol = 1e-12 if prec == Q.QD_C128 else c64_tol(1, dT)
                assert max_abs(out, ref) <= tol, (dims, t, c, kind, prec)
                # amplitudes outside the active slices are bit-identical (rewritten unchanged)
                act = np.ones(D, bool)
                idx = np.arange(D)
                for q, val in zip(c, v):
                    act &= (idx // st[q]) % dims[q] == val
                x0 = psi0.astype(out.dtype)
                assert np.array_equal(out[~act], x0[~act]), (dims, t, c, kind)
    assert seen == {"pred", "edge", "aligned"}


@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
def test_inline_controls_take_the_direct_route(stream, prec):
    """With the run threshold raised so that a target of stride 18 would be staged in LDS, a gate
    whose control of stride 6 (a qutrit, inside a line) leaves lines without a matching amplitude
    still runs on the direct kernel, which skips those lines; a control of stride 1 (every line
    matches somewhere) keeps the tile route, and so does every case in complex64, whose 16-amplitude
    lines all hold a matching amplitude here. Each against the oracle."""
    dims = (3, 2, 4, 3, 2, 5, 3, 2, 3)                # strides 4320, 2160, 540, 180, 90, 18, 6, 3, 1
    rng = C.seeded_rng(101)
    D = O.register_size(dims)
    psi0 = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    psi0 /= np.linalg.norm(psi0)
    line = 8 if prec == Q.QD_C128 else 16
    st = O.strides(dims)
    idx = np.arange(D)
    Q.qd_tune_set(Q.QD_TUNE_RUN_MIN, 64)
    try:
        seen = set()
        for t, c, v in (((5,), (6,), (2,)), ((5,), (6, 7), (0, 1)), ((5,), (8,), (1,))):
            act = np.ones(D, bool)
            for q, val in zip(c, v):
                act &= (idx // st[q]) % dims[q] == val
            full = D - D % line
            skips = not act[:full].reshape(-1, line).any(axis=1).all()
            route = Q.QD_ROUTE_DIRECT if skips else Q.QD_ROUTE_TILED
            seen.add(route)
            U = C.haar_unitary(5, rng)
            assert Q.qd_gate_route(dims, prec, t, c, v, U) == route, (t, c, prec)
            s = Q.qd_state_init(dims, prec, stream)
            try:
                Q.qd_state_upload(s, psi0)
                Q.qd_apply_gate(s, t, c, v, U)
                out = Q.qd_state_download(s)
            finally:
                Q.qd_state_free(s)
            ref = O.apply_gate(psi0, dims, t, c, v, U)
            tol = 1e-12 if prec == Q.QD_C128 else c64_tol(1, 5)
            assert max_abs(out, ref) <= tol, (t, c, prec)
        assert Q.QD_ROUTE_TILED in seen and (prec == Q.QD_C64 or Q.QD_ROUTE_DIRECT in seen)
    finally:
        Q.qd_tune_set(Q.QD_TUNE_RUN_MIN, 0)
