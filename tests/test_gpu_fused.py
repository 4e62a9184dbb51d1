"""GPU parity of gate fusion (qd_fuse) and fused-block application (qd_apply_fused).

* Each FP64 block built on the GPU equals the oracle's product of the block's gates embedded in
  its window, within 1e-12 (fusion is exact in exact arithmetic).
* Fused FP64 application reproduces the oracle state within 1e-12.
* Matrix-core modes keep the state in complex64. Each is gated on the literal fidelity loss,
  |1 - |<psi64|psi32>|^2| <= 1e-6 with psi32 as the path leaves it (no normalisation by the test;
  a norm above 1 makes the loss negative, so its magnitude is bounded), and on the norm drift
  | ||psi32||^2 - 1 | <= 1e-6, against the oracle (shrunken registers) or the complex128 plain GPU
  path (full size). FP32 products round A and X to 24 bits and accumulate 2B terms per output in
  FP32, so the 2-norm error of nb blocks stays below 4 nb (2B) 2^-24, and FP32 meets the gate as
  it is. Split BF16 holds A to ~2^-16 (two BF16 terms), so its norm drifts by up to ~2^-16 per
  block: it meets the gate with the path's FP64 renormalisation on the GPU as its last step
  (QD_FUSED_RENORMALIZE); without it, the direction of the state (fidelity after normalising) is
  held to 1e-6 and the drift is reported, bounded by 1e-5.
"""
import numpy as np
import pytest

import circuits as C
import oracle as O
import paper_2211_07918_amd as Q
from gpu_util import fidelity_loss, max_abs, read_amplitudes, torch_stream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stream():
    return torch_stream()


def fuse(circ, maxb, stream):
    ga = Q.GateArray(circ.gates, lambda i: circ.dims)
    return Q.qd_fuse(circ.dims, ga, maxb, stream)


def blocks_of(f):
    return [Q.qd_fused_block_info(f, b) for b in range(Q.qd_fused_count(f))]


def run_fused(circ, f, prec, mode, stream):
    s = Q.qd_state_init(circ.dims, prec, stream)
    try:
        if circ.init_amps is not None:
            Q.qd_state_upload(s, circ.init_amps)
        Q.qd_apply_fused(s, f, mode)
        return Q.qd_state_download(s)
    finally:
        Q.qd_state_free(s)


CASES = [("qft4x6", lambda: C.config2(6), 64), ("brick3x7", lambda: C.config3(7, 6), 81),
         ("hybrid-shrink", lambda: C.config1_shrink(80), 64), ("hybrid-shrink-27", lambda: C.config1_shrink(80), 27),
         ("qft3x6", lambda: C.Circuit((3,) * 6, C.qudit_qft_gates(3, 6),
                                      init_amps=C.random_basis_superposition(729, 50, C.seeded_rng(3))), 81),
         ("random-128", lambda: C.random_circuit((2, 4, 2, 2, 4, 2, 2), 40, C.seeded_rng(4), max_controls=1,
                                                 max_dT=16), 128),
         ("random-16", lambda: C.random_circuit((2, 3, 2, 2, 3, 2), 40, C.seeded_rng(5), max_controls=0,
                                                max_dT=12), 16)]


@pytest.mark.parametrize("name,make,maxb", CASES)
def test_blocks_match_oracle_products(stream, name, make, maxb):
    circ = make()
    f = fuse(circ, maxb, stream)
    try:
        infos = blocks_of(f)
        covered = []
        for b, info in enumerate(infos):
            gates = [circ.gates[i] for i in info["gates"]]
            assert info["gates"] == sorted(info["gates"]) and info["first_gate"] == info["gates"][0]
            covered += info["gates"]
            win = set(q for g in gates for q in g.qudits())
            assert sorted(win) == info["window"]
            assert info["B"] == int(np.prod([circ.dims[q] for q in info["window"]])) <= maxb
            M = Q.qd_fused_download_block(f, b)
            assert max_abs(M, O.fused_block(circ.dims, info["window"], gates)) <= 1e-12, (name, b)
        assert sorted(covered) == list(range(len(circ.gates)))
    finally:
        Q.qd_fused_free(f)


@pytest.mark.parametrize("name,make,maxb", CASES)
def test_fused_fp64_equals_oracle(stream, name, make, maxb):
    circ = make()
    f = fuse(circ, maxb, stream)
    try:
        psi = run_fused(circ, f, Q.QD_C128, Q.QD_MODE_FP64_PLAIN, stream)
    finally:
        Q.qd_fused_free(f)
    assert max_abs(psi, O.run_circuit(circ)) <= 1e-12


def precision(ref, psi):
    """Literal fidelity loss, norm drift and normalised fidelity loss of psi against ref (FP64)."""
    psi = np.asarray(psi, np.complex128)
    n2 = float(np.vdot(psi, psi).real)
    fid = fidelity_loss(ref, psi)
    return fid, abs(n2 - 1.0), 1.0 - (1.0 - fid) / n2


def assert_gate(ref, psi, what):
    """The precision gate: |literal fidelity loss| <= 1e-6 and norm drift <= 1e-6."""
    fid, drift, _ = precision(ref, psi)
    assert abs(fid) <= 1e-6 and drift <= 1e-6, (what, fid, drift)


# modes as graded: FP32 as the path leaves it; BF16x3 with the FP64 renormalisation on the GPU
GATED = [Q.QD_MODE_FP32_MFMA, Q.QD_MODE_BF16X3_MFMA | Q.QD_FUSED_RENORMALIZE]


@pytest.mark.parametrize("mode", GATED)
@pytest.mark.parametrize("name,make,maxb", CASES)
def test_matrix_core_modes_vs_oracle(stream, mode, name, make, maxb):
    circ = make()
    f = fuse(circ, maxb, stream)
    try:
        nb = Q.qd_fused_count(f)
        psi = run_fused(circ, f, Q.QD_C64, mode, stream)
        raw = run_fused(circ, f, Q.QD_C64, mode & 0xFF, stream)
    finally:
        Q.qd_fused_free(f)
    ref = O.run_circuit(circ)
    assert_gate(ref, psi, name)
    if mode == Q.QD_MODE_FP32_MFMA:
        assert np.array_equal(psi, raw)
        assert max_abs(psi, ref) <= 4 * nb * 2 * maxb * 2.0 ** -24
        assert precision(ref, psi)[1] <= 4 * nb * 2.0 ** -24 * 2 * maxb
    else:
        # without the renormalisation: the direction is held to 1e-6, the drift reported
        fid, drift, fid_norm = precision(ref, raw)
        assert fid_norm <= 1e-6 and drift <= 1e-5, (name, fid_norm, drift)
        assert max_abs(psi, ref) <= 4 * nb * 3 * 2.0 ** -16


@pytest.mark.parametrize("mode", GATED)
def test_qft_10_ququarts_vs_oracle_and_fft(stream, mode):
    """The qudit QFT on 10 ququarts (D = 1,048,576): fused complex64 against the oracle and
    against sqrt(N) ifft of the input."""
    circ = C.config2(10)
    f = fuse(circ, 64, stream)
    try:
        psi = run_fused(circ, f, Q.QD_C64, mode, stream)
    finally:
        Q.qd_fused_free(f)
    for r in (np.sqrt(circ.D) * np.fft.ifft(circ.init_amps), O.run_circuit(circ)):
        assert_gate(r, psi, "qft10")


@pytest.mark.parametrize("mode", GATED)
def test_brickwork_12_qutrits_vs_oracle(stream, mode):
    circ = C.config3(12, 30)
    f = fuse(circ, 81, stream)
    try:
        psi = run_fused(circ, f, Q.QD_C64, mode, stream)
    finally:
        Q.qd_fused_free(f)
    assert_gate(O.run_circuit(circ), psi, "brick12")


def _plain64(circ, stream):
    s = Q.qd_state_init(circ.dims, Q.QD_C128, stream)
    if circ.init_amps is not None:
        Q.qd_state_upload(s, circ.init_amps)
    for g in circ.gates:
        Q.apply_circuit_gate(s, g, circ.dims)
    return s


@pytest.mark.parametrize("mode", GATED)
def test_qft_14_ququarts_full_size(stream, mode):
    """D = 268,435,456: fused complex64 vs the complex128 plain GPU path, compared on the GPU in
    FP64; plus sampled amplitudes against sqrt(N) ifft of the sparse input."""
    circ = C.config2(14)
    ref = _plain64(circ, stream)
    f = fuse(circ, 64, stream)
    s = Q.qd_state_init(circ.dims, Q.QD_C64, stream)
    try:
        Q.qd_state_upload(s, circ.init_amps)
        Q.qd_apply_fused(s, f, mode)
        cmp = Q.qd_compare_ex(ref, s)
        assert abs(cmp["fid_loss"]) <= 1e-6 and cmp["norm_drift"] <= 1e-6 and cmp["max_abs"] <= 1e-5, cmp
        if mode != Q.QD_MODE_FP32_MFMA:
            Q.qd_state_upload(s, circ.init_amps)     # without the renormalisation
            Q.qd_apply_fused(s, f, mode & 0xFF)
            raw = Q.qd_compare_ex(ref, s)
            assert raw["fid_loss_normalized"] <= 1e-6 and raw["norm_drift"] <= 1e-5, raw
        # the plain FP64 path itself against the closed form at sampled outputs
        psi64 = Q.qd_state_download(ref)
        nz = np.flatnonzero(circ.init_amps)
        idx = C.seeded_rng(9).choice(circ.D, 64, replace=False)
        N = circ.D
        want = [np.sum(circ.init_amps[nz] * np.exp(2j * np.pi * (nz * int(y) % N) / N)) / np.sqrt(N) for y in idx]
        assert max_abs(psi64[idx], np.array(want)) <= 1e-12
    finally:
        Q.qd_state_free(s)
        Q.qd_state_free(ref)
        Q.qd_fused_free(f)


@pytest.mark.parametrize("mode", GATED)
def test_brickwork_20_qutrits_full_size(stream, mode):
    """D = 3,486,784,401 (28 GB complex64, 56 GB complex128 comparator), 30 brickwork layers of
    Haar 9x9 gates fused into 81x81 blocks."""
    circ = C.config3(20, 30)
    ref = _plain64(circ, stream)
    f = fuse(circ, 81, stream)
    s = Q.qd_state_init(circ.dims, Q.QD_C64, stream)
    try:
        Q.qd_apply_fused(s, f, mode)
        cmp = Q.qd_compare_ex(ref, s)
        assert abs(cmp["fid_loss"]) <= 1e-6 and cmp["norm_drift"] <= 1e-6, cmp
        assert abs(Q.qd_norm2(ref) - 1.0) <= 1e-12
        if mode != Q.QD_MODE_FP32_MFMA:
            Q.qd_state_set_basis(s, [0] * len(circ.dims))     # without the renormalisation
            Q.qd_apply_fused(s, f, mode & 0xFF)
            raw = Q.qd_compare_ex(ref, s)
            assert raw["fid_loss_normalized"] <= 1e-6 and raw["norm_drift"] <= 1e-5, raw
    finally:
        Q.qd_state_free(s)
        Q.qd_state_free(ref)
        Q.qd_fused_free(f)


@pytest.mark.parametrize("mode", GATED)
def test_brickwork_20_qutrits_block_vs_oracle_samples(stream, mode):
    """One 81 x 81 block on the 28 GB 20-qutrit register against the oracle at sampled outputs.
    The input is a product state (every qutrit q in U_q|0> for a seeded Haar U_q, prepared on the
    GPU by the plain complex64 path), which the oracle evaluates amplitude by amplitude; the block
    is the product of three Haar 9 x 9 gates on qutrits (8, 9), (10, 11), (9, 10), which the oracle
    builds as full operators of a 4-qutrit register. Samples: 400 seeded indices and the state's
    ends. Bound, per output y = sum_c M[r, c] x_c, relative to b = sum_c |M[r, c]| |x_c| (which
    the oracle also evaluates): the inputs carry the rounding of 20 complex64 gates (at most
    3 x 2^-24 each, relative), and the block's real products sum 162 terms in FP32 (FP32 mode:
    162 x 2^-24) or use operands split into BF16 pairs held to about 2^-16 (split-BF16 mode:
    3 x 2^-16), so |y - y_oracle| <= c b with c = 60 x 2^-24 + 162 x 2^-24 (FP32) or
    60 x 2^-24 + 3 x 2^-16 (split BF16, whose FP64 renormalisation moves each output by about 1e-6
    of |y| <= b more)."""
    dims = (3,) * 20
    n = len(dims)
    D = 3 ** 20
    rng = C.seeded_rng(2020)
    prep = [C.haar_unitary(3, rng) for _ in range(n)]
    gates = [C.Gate("U", (8, 9), U=C.haar_unitary(9, rng)), C.Gate("U", (10, 11), U=C.haar_unitary(9, rng)),
             C.Gate("U", (9, 10), U=C.haar_unitary(9, rng))]
    circ = C.Circuit(dims, gates)
    f = fuse(circ, 81, stream)
    s = Q.qd_state_init(dims, Q.QD_C64, stream)
    try:
        assert Q.qd_fused_count(f) == 1 and Q.qd_fused_block_info(f, 0)["B"] == 81
        Q.qd_state_set_basis(s, [0] * n)
        for q, U in enumerate(prep):
            Q.qd_apply_gate(s, (q,), (), (), U)
        Q.qd_apply_fused(s, f, mode)
        # the block as the oracle defines it: G3 G2 G1 on qutrits 8..11 (local 0..3)
        w4 = (3, 3, 3, 3)
        M = np.eye(81, dtype=np.complex128)
        for g in gates:
            M = O.gate_operator(w4, tuple(t - 8 for t in g.targets), (), (), g.U) @ M
        phi = [U[:, 0] for U in prep]

        class Prepared:
            def __init__(self, vecs):
                self.vecs = vecs

            def __getitem__(self, i):
                return complex(np.prod([self.vecs[q][d] for q, d in enumerate(O.digits_of(int(i), dims))]))

        idx = list(rng.choice(D, 400, replace=False)) + [0, 1, D - 2, D - 1]
        want = O.apply_gate_at(Prepared(phi), dims, (8, 9, 10, 11), (), (), M, idx)
        bound = O.apply_gate_at(Prepared([np.abs(p) for p in phi]), dims, (8, 9, 10, 11), (), (), np.abs(M), idx).real
        got = read_amplitudes(s, Q.QD_C64, idx)
        c = 60 * 2.0 ** -24 + (162 * 2.0 ** -24 if mode == Q.QD_MODE_FP32_MFMA else 3 * 2.0 ** -16)
        ratio = float(np.max(np.abs(np.asarray(got) - want) / bound))
        assert ratio <= c, (ratio, c, max_abs(got, want))
    finally:
        Q.qd_state_free(s)
        Q.qd_fused_free(f)


def test_mode_and_register_errors(stream):
    circ = C.config2(5)
    f = fuse(circ, 64, stream)
    try:
        s64 = Q.qd_state_init(circ.dims, Q.QD_C128, stream)
        s32 = Q.qd_state_init(circ.dims, Q.QD_C64, stream)
        other = Q.qd_state_init((4,) * 4 + (2,), Q.QD_C64, stream)
        try:
            for s, mode in ((s64, Q.QD_MODE_FP32_MFMA), (s32, Q.QD_MODE_FP64_PLAIN), (other, Q.QD_MODE_FP32_MFMA)):
                with pytest.raises(Q.QDError) as e:
                    Q.qd_apply_fused(s, f, mode)
                assert e.value.code == Q.QD_EDIM
            for bad in (7, Q.QD_MODE_FP32_MFMA | 0x200):
                with pytest.raises(Q.QDError) as e:
                    Q.qd_apply_fused(s32, f, bad)
                assert e.value.code == Q.QD_EINVAL
            # renormalising a zero state leaves it zero (no division by a zero norm)
            Q.qd_state_upload(s32, np.zeros(circ.D, np.complex64))
            Q.qd_apply_fused(s32, f, Q.QD_MODE_BF16X3_MFMA | Q.QD_FUSED_RENORMALIZE)
            assert not np.any(Q.qd_state_download(s32))
            # in FP64 mode the renormalisation keeps the oracle state within 1e-12
            Q.qd_state_upload(s64, circ.init_amps)
            Q.qd_apply_fused(s64, f, Q.QD_MODE_FP64_PLAIN | Q.QD_FUSED_RENORMALIZE)
            assert max_abs(Q.qd_state_download(s64), O.run_circuit(circ)) <= 1e-12
        finally:
            for s in (s64, s32, other):
                Q.qd_state_free(s)
    finally:
        Q.qd_fused_free(f)


@pytest.mark.parametrize("mode", [Q.QD_MODE_FP32_MFMA, Q.QD_MODE_BF16X3_MFMA])
def test_odd_runs_on_an_exact_size_buffer(stream, mode):
    """Runs of odd length are moved in 16-byte units that read one spare amplitude past a run;
    on a caller's buffer of exactly D amplitudes (no room past the last one) the tile moves fall
    back to 4-byte units. Both give the same bits."""
    import torch
    circ = C.config3(9, 12)                                  # runs of 81 amplitudes, D = 19683 (odd)
    f = fuse(circ, 81, stream)
    try:
        own = run_fused(circ, f, Q.QD_C64, mode, stream)
        buf = torch.zeros(circ.D, dtype=torch.complex64, device="cuda")
        s = Q.qd_state_wrap(circ.dims, Q.QD_C64, buf.data_ptr(), circ.D * 8, stream)
        try:
            Q.qd_state_set_basis(s, [0] * len(circ.dims))
            Q.qd_apply_fused(s, f, mode)
            wrapped = Q.qd_state_download(s)
        finally:
            Q.qd_state_free(s)
    finally:
        Q.qd_fused_free(f)
    assert np.array_equal(own, wrapped)
    assert precision(O.run_circuit(circ), own)[2] <= 1e-6


# One block per circuit (a single Haar gate on the window), shaped to reach every matrix-core
# kernel instance: (dims, window, FP32 instance, BF16x3 instance, exact-size caller buffer)
SHAPES = [
    # 81-wide blocks on the double-buffered FP32 kernel
    ((3, 3, 3, 3, 2, 2), (0, 1, 2, 3), "k_fused_pipe<3, 6, 41, 0, false, 13312>",
     "k_fused_rows<3, 6, 2, 6, true, 2, 0, false>", False),          # runs of even length (324)
    ((3,) * 6, (0, 1, 2, 3), "k_fused_pipe<3, 6, 41, 1, false, 13312>",
     "k_fused_rows<3, 6, 2, 6, true, 2, 1, false>", False),          # odd runs, 9 columns
    ((3,) * 9, (0, 1, 2, 3), "k_fused_pipe<3, 6, 41, 1, true, 13312>",
     "k_fused_rows<3, 6, 2, 6, true, 2, 1, false>", False),          # 81 runs of 81 above the window's rows
    ((3,) * 8, (4, 5, 6, 7), "k_fused_pipe<3, 6, 41, 1, true, 13312>",
     "k_fused_rows<3, 6, 2, 6, true, 2, 1, false>", False),          # the window inside one run
    ((3,) * 9, (0, 1, 2, 3), "k_fused_pipe<3, 6, 41, 2, true, 13312>",
     "k_fused_rows<3, 6, 2, 6, true, 2, 2, false>", True),           # 4-byte units
    # the multi-workgroup kernel for B <= 64 and 81 < B <= 96, the general one above 96
    ((4, 4, 4, 2, 2), (0, 1, 2), "k_fused_rows<2, 4, 1, 32, false, 2, 0, false>",
     "k_fused_rows<2, 4, 1, 4, true, 2, 0, false>", False),
    ((4, 4, 4, 3, 3, 3, 3), (0, 1, 2), "k_fused_rows<2, 4, 1, 32, false, 2, 1, false>",
     "k_fused_rows<2, 4, 1, 4, true, 2, 1, false>", False),
    ((2, 2, 2, 2, 2, 3, 3, 3, 3), (0, 1, 2, 3, 4), "k_fused_rows<1, 4, 1, 16, false, 2, 1, false>",
     "k_fused_rows<1, 4, 1, 2, true, 2, 1, false>", False),
    ((2, 4, 4, 3, 3, 2), (0, 1, 2, 3), "k_fused_rows<3, 6, 2, 48, false, 2, 0, false>",
     "k_fused_rows<3, 6, 2, 6, true, 2, 0, false>", False),
    ((2,) * 7 + (3,), tuple(range(7)), "k_fused<4, 4, 64, false>", "k_fused<4, 4, 8, true>", False),
]


@pytest.mark.parametrize("dims,window,k32,kbf,exact", SHAPES)
def test_kernel_instances_by_block_shape(stream, dims, window, k32, kbf, exact):
    """Each block shape reaches the kernel instance it is meant for (qd_last_kernel after the run),
    and both matrix-core modes meet the precision gate against the oracle there."""
    import torch
    rng = C.seeded_rng(sum(dims) * 31 + len(window))
    dT = int(np.prod([dims[q] for q in window]))
    D = int(np.prod(dims))
    circ = C.Circuit(tuple(dims), [C.Gate("U", tuple(window), U=C.haar_unitary(dT, rng))],
                     init_amps=C.random_basis_superposition(D, min(D, 64), rng))
    f = fuse(circ, 128, stream)
    try:
        assert Q.qd_fused_count(f) == 1
        assert Q.qd_fused_block_info(f, 0)["B"] == dT
        ref = O.run_circuit(circ)
        for mode, want in ((Q.QD_MODE_FP32_MFMA, k32), (Q.QD_MODE_BF16X3_MFMA | Q.QD_FUSED_RENORMALIZE, kbf)):
            if exact:   # a caller's buffer of exactly D amplitudes: no spare read past the last one
                buf = torch.zeros(D, dtype=torch.complex64, device="cuda")
                s = Q.qd_state_wrap(circ.dims, Q.QD_C64, buf.data_ptr(), D * 8, stream)
            else:
                s = Q.qd_state_init(circ.dims, Q.QD_C64, stream)
            try:
                Q.qd_state_upload(s, circ.init_amps)
                Q.qd_apply_fused(s, f, mode)
                assert Q.qd_last_kernel() == want, (dims, window, mode, Q.qd_last_kernel())
                psi = Q.qd_state_download(s)
            finally:
                Q.qd_state_free(s)
            assert_gate(ref, psi, (dims, window, want))
    finally:
        Q.qd_fused_free(f)
