"""GPU parity of the batched path: many circuits over uneven mixed-radix registers, one
persistent launch per gate layer, optionally recorded into a hipGraph and replayed.

complex128 batches match the oracle within 1e-12; complex64 batches within the per-gate FP32
bound (4 G d 2^-24, see test_gpu_plain) and fidelity loss <= 1e-6 per circuit.
"""
import numpy as np
import pytest

import circuits as C
import oracle as O
import paper_2211_07918_amd as Q
from gpu_util import fidelity_loss, max_abs, run_gpu, torch_stream

pytestmark = pytest.mark.gpu
U24 = 2.0 ** -24


@pytest.fixture(scope="module")
def stream():
    return torch_stream()


def small_batch(nc=48, ngates=30, seed=77, hi=2e4):
    rng = C.seeded_rng(seed)
    out = []
    for i in range(nc):
        dims = C._batch_dims(rng, 1e2, hi)
        gates = [C.random_gate(dims, rng, kinds=("X", "Z", "F", "CX", "H1"), cval_top=bool(i % 2))
                 for _ in range(ngates)]
        out.append(C.Circuit(dims, gates))
    # a few hand-made registers: single qudit, controls on the stride-1 qudit, radix 8
    out.append(C.Circuit((3,), [C.Gate("F", (0,)), C.Gate("X", (0,), a=2)] + [C.Gate("Z", (0,))] * (ngates - 2)))
    out.append(C.Circuit((2, 8, 3), [C.Gate("U", (1,), (2,), (1,), U=C.haar_unitary(8, rng))] * ngates))
    return out


def layers_of(circs):
    L = max(len(c.gates) for c in circs)
    for l in range(L):
        yield Q.GateArray([c.gates[l] if l < len(c.gates) else None for c in circs], lambda i: circs[i].dims)


def split(arena, b, circs):
    return [arena[Q.qd_batch_offset(b, i):Q.qd_batch_offset(b, i) + c.D] for i, c in enumerate(circs)]


@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
def test_small_batch_vs_oracle(stream, prec):
    circs = small_batch()
    b = Q.qd_batch_create([c.dims for c in circs], prec, stream)
    try:
        for ga in layers_of(circs):
            Q.qd_batch_apply_layer(b, ga)
        arena = Q.qd_batch_download(b, np.complex128 if prec == Q.QD_C128 else np.complex64)
        for c, psi in zip(circs, split(arena, b, circs)):
            ref = O.run_circuit(c)
            if prec == Q.QD_C128:
                assert max_abs(psi, ref) <= 1e-12
            else:
                assert max_abs(psi, ref) <= 4 * len(c.gates) * 8 * U24
                assert fidelity_loss(ref, psi) <= 1e-6
    finally:
        Q.qd_batch_free(b)


@pytest.mark.parametrize("block,spt,grid", [(64, 1, 8), (128, 2, 64), (256, 4, 1), (256, 8, 64), (192, 8, 16)])
def test_batch_tile_shapes(stream, block, spt, grid):
    """Every tile shape and both grid modes (persistent workgroups walking the tile list, or one
    workgroup per tile) give the oracle's states."""
    circs = small_batch(24, 12, seed=78)
    Q.qd_tune_set(Q.QD_TUNE_BATCH_BLOCK, block)
    Q.qd_tune_set(Q.QD_TUNE_BATCH_SPT, spt)
    Q.qd_tune_set(Q.QD_TUNE_BATCH_GRID, grid)
    b = Q.qd_batch_create([c.dims for c in circs], Q.QD_C128, stream)
    try:
        for ga in layers_of(circs):
            Q.qd_batch_apply_layer(b, ga)
        arena = Q.qd_batch_download(b, np.complex128)
    finally:
        Q.qd_batch_free(b)
        Q.qd_tune_set(Q.QD_TUNE_BATCH_BLOCK, 0)
        Q.qd_tune_set(Q.QD_TUNE_BATCH_SPT, 0)
        Q.qd_tune_set(Q.QD_TUNE_BATCH_GRID, 0)
    offs = np.cumsum([0] + [c.D for c in circs])
    for i, c in enumerate(circs):
        assert max_abs(arena[offs[i]:offs[i + 1]], O.run_circuit(c)) <= 1e-12


def test_graph_replays_match_eager(stream):
    circs = small_batch(32, 20, seed=79)
    dims = [c.dims for c in circs]
    eager = Q.qd_batch_create(dims, Q.QD_C64, stream)
    rec = Q.qd_batch_create(dims, Q.QD_C64, stream)
    try:
        gas = list(layers_of(circs))
        for ga in gas:
            Q.qd_batch_apply_layer(eager, ga)
        want = Q.qd_batch_download(eager)
        Q.qd_batch_capture(rec, True)
        for ga in gas:
            Q.qd_batch_apply_layer(rec, ga)
        Q.qd_batch_capture(rec, False)
        # recording ran nothing
        assert np.count_nonzero(Q.qd_batch_download(rec)) == len(circs)
        for rep in range(3):
            Q.qd_batch_reset(rec)
            Q.qd_batch_replay(rec)
            got = Q.qd_batch_download(rec)        # synchronises between replays
            assert np.array_equal(got, want), rep
            # eager work on the same stream between replays
            Q.qd_batch_reset(eager)
            for ga in gas[:3]:
                Q.qd_batch_apply_layer(eager, ga)
        # a second replay without reset continues from the previous state: two passes of the circuits
        Q.qd_batch_reset(rec)
        Q.qd_batch_replay(rec)
        Q.qd_batch_replay(rec)
        twice = Q.qd_batch_download(rec)
        offs = np.cumsum([0] + [c.D for c in circs])
        for i, c in enumerate(circs):
            ref = O.run_circuit(C.Circuit(c.dims, c.gates + c.gates))
            assert fidelity_loss(ref, twice[offs[i]:offs[i + 1]]) <= 1e-6
    finally:
        Q.qd_batch_free(eager)
        Q.qd_batch_free(rec)


def test_batch_errors_leave_arena(stream):
    circs = small_batch(4, 3, seed=80)
    b = Q.qd_batch_create([c.dims for c in circs], Q.QD_C64, stream)
    try:
        before = Q.qd_batch_download(b)
        rng = C.seeded_rng(3)
        bad_sets = []
        two_t = list(circs[0].gates[:1]) + [None] * 3
        d0 = circs[0].dims
        two_t[0] = C.Gate("U", (0, 1), U=C.haar_unitary(d0[0] * d0[1], rng))
        bad_sets.append(two_t)
        two_c = [None] * 4
        two_c[1] = C.Gate("X", (0,), (1, 2), (0, 0), a=1)
        bad_sets.append(two_c)
        nonunit = [None] * 4
        nonunit[2] = C.Gate("U", (0,), U=np.ones((circs[2].dims[0],) * 2))
        bad_sets.append(nonunit)
        for gs in bad_sets:
            with pytest.raises(Q.QDError) as e:
                Q.qd_batch_apply_layer(b, Q.GateArray(gs, lambda i: circs[i].dims))
            assert e.value.code in (Q.QD_EINVAL, Q.QD_ENOTUNITARY)
        assert np.array_equal(Q.qd_batch_download(b), before)
        with pytest.raises(Q.QDError):
            Q.qd_batch_replay(b)
    finally:
        Q.qd_batch_free(b)


def test_full_4096_circuits(stream):
    """4096 circuits, D log-uniform in [1e3, 1e6], 100 layers, complex64, recorded as a graph:
    every register keeps its norm, a seeded sample matches the oracle, and a sample matches the
    one-by-one plain path exactly in structure (bitwise-equal fraction reported)."""
    circs = C.config4()
    dims = [c.dims for c in circs]
    b = Q.qd_batch_create(dims, Q.QD_C64, stream)
    try:
        Q.qd_batch_capture(b, True)
        for ga in layers_of(circs):
            Q.qd_batch_apply_layer(b, ga)
        Q.qd_batch_capture(b, False)
        Q.qd_batch_replay(b)
        arena = Q.qd_batch_download(b)
    finally:
        Q.qd_batch_free(b)
    offs = np.cumsum([0] + [c.D for c in circs])
    p = (arena.real.astype(np.float64) ** 2 + arena.imag.astype(np.float64) ** 2)
    norms = np.add.reduceat(p, offs[:-1])
    assert np.max(np.abs(norms - 1.0)) <= 4 * 100 * 4 * U24
    rng = C.seeded_rng(81)
    sample = sorted(set(rng.choice(len(circs), 12, replace=False).tolist()) | {int(np.argmin(offs[1:] - offs[:-1]))})
    for i in sample:
        psi = arena[offs[i]:offs[i + 1]]
        c = circs[i]
        if c.D <= 300_000:
            assert fidelity_loss(O.run_circuit(c), psi) <= 1e-6, i
        plain = run_gpu(c, Q.QD_C64, stream)
        assert max_abs(plain, psi) <= 4 * 100 * 4 * U24, i


def all_layers(circs):
    """Every layer as one layer-major GateArray (empty slots past a circuit's end)."""
    L = max(len(c.gates) for c in circs)
    nc = len(circs)
    flat = [circs[i].gates[l] if l < len(circs[i].gates) else None for l in range(L) for i in range(nc)]
    return Q.GateArray(flat, lambda j: circs[j % nc].dims), L


@pytest.mark.parametrize("width", [1, 2, 3, 4, 8])
@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
def test_fused_layers_vs_oracle(stream, width, prec):
    """Gates composed per circuit into blocks of up to `width` give the oracle's states; the batch
    holds circuits whose gates compose and circuits that keep one gate per block (a radix-8
    controlled Haar gate, qutrit controlled shifts), and circuits of different lengths."""
    circs = small_batch(40, 23, seed=81)
    for i in (3, 10, 17):                       # shorter circuits: empty slots in the last layers
        circs[i] = C.Circuit(circs[i].dims, circs[i].gates[:5 + i])
    ga, L = all_layers(circs)
    b = Q.qd_batch_create([c.dims for c in circs], prec, stream)
    try:
        Q.qd_batch_apply_layers(b, ga, L, width)
        states = split(Q.qd_batch_download(b, np.complex128 if prec == Q.QD_C128 else np.complex64), b, circs)
    finally:
        Q.qd_batch_free(b)
    for c, psi in zip(circs, states):
        ref = O.run_circuit(c)
        if prec == Q.QD_C128:
            assert max_abs(psi, ref) <= 1e-12
        else:
            assert max_abs(psi, ref) <= 4 * len(c.gates) * 32 * U24
            assert fidelity_loss(ref, psi) <= 1e-6


def test_fused_layers_in_a_graph(stream):
    circs = small_batch(24, 16, seed=82)
    dims = [c.dims for c in circs]
    ga, L = all_layers(circs)
    eager = Q.qd_batch_create(dims, Q.QD_C64, stream)
    rec = Q.qd_batch_create(dims, Q.QD_C64, stream)
    try:
        Q.qd_batch_apply_layers(eager, ga, L, 2)
        want = Q.qd_batch_download(eager)
        Q.qd_batch_capture(rec, True)
        Q.qd_batch_apply_layers(rec, ga, L, 2)
        Q.qd_batch_capture(rec, False)
        for rep in range(3):
            Q.qd_batch_reset(rec)
            Q.qd_batch_replay(rec)
            assert np.array_equal(Q.qd_batch_download(rec), want), rep
            Q.qd_batch_reset(eager)
            Q.qd_batch_apply_layers(eager, ga, 2, 1)
    finally:
        Q.qd_batch_free(eager)
        Q.qd_batch_free(rec)


def test_fusion_autotune_keeps_the_arena_and_graph(stream):
    """The tuner restores the arena and leaves a graph the caller recorded replayable."""
    circs = small_batch(16, 8, seed=83)
    ga, L = all_layers(circs)
    b = Q.qd_batch_create([c.dims for c in circs], Q.QD_C64, stream)
    try:
        Q.qd_batch_capture(b, True)
        Q.qd_batch_apply_layers(b, ga, 3, 1)
        Q.qd_batch_capture(b, False)
        Q.qd_batch_replay(b)
        before = Q.qd_batch_download(b)
        Q.qd_batch_autotune_layers(b, ga, L)
        assert Q.qd_tune_get(Q.QD_TUNE_BATCH_FUSE) in (1, 2, 3, 4, 6, 8)
        assert Q.qd_tune_get(Q.QD_TUNE_BATCH_SPT_MID) in (0, 1, 2, 4, 8)
        assert Q.qd_tune_get(Q.QD_TUNE_BATCH_SPT_WIDE) in (0, 1, 2, 4, 8)
        assert np.array_equal(Q.qd_batch_download(b), before)
        Q.qd_batch_reset(b)
        Q.qd_batch_replay(b)
        assert np.array_equal(Q.qd_batch_download(b), before)
        with pytest.raises(Q.QDError):
            Q.qd_batch_apply_layers(b, ga, L, 9)
        with pytest.raises(Q.QDError):
            Q.qd_tune_set(Q.QD_TUNE_BATCH_FUSE, 9)
    finally:
        Q.qd_batch_free(b)
        for prm in (Q.QD_TUNE_BATCH_FUSE, Q.QD_TUNE_BATCH_SPT_MID, Q.QD_TUNE_BATCH_SPT_WIDE):
            Q.qd_tune_set(prm, 0)


@pytest.mark.parametrize("mid,wide", [(1, 1), (8, 4), (0, 8)])
def test_slice_class_shapes_keep_results(stream, mid, wide):
    """Every slices-per-thread setting of the wide slice classes gives the oracle's states."""
    circs = small_batch(24, 17, seed=85)
    ga, L = all_layers(circs)
    b = Q.qd_batch_create([c.dims for c in circs], Q.QD_C128, stream)
    try:
        Q.qd_tune_set(Q.QD_TUNE_BATCH_SPT_MID, mid)
        Q.qd_tune_set(Q.QD_TUNE_BATCH_SPT_WIDE, wide)
        Q.qd_batch_apply_layers(b, ga, L, 8)
        states = split(Q.qd_batch_download(b, np.complex128), b, circs)
    finally:
        Q.qd_batch_free(b)
        Q.qd_tune_set(Q.QD_TUNE_BATCH_SPT_MID, 0)
        Q.qd_tune_set(Q.QD_TUNE_BATCH_SPT_WIDE, 0)
    for c, psi in zip(circs, states):
        assert max_abs(psi, O.run_circuit(c)) <= 1e-12


def test_full_4096_circuits_at_the_tuned_width(stream):
    """The 4096-circuit, 100-layer complex64 batch at the fusion width the tuner picks, recorded as
    a graph (as the benchmark times it): every register keeps its norm; a seeded sample matches
    the oracle and the one-by-one plain path within the FP32 bound of 100 passes over slices of
    up to 32 amplitudes."""
    circs = C.config4()
    ga, L = all_layers(circs)
    b = Q.qd_batch_create([c.dims for c in circs], Q.QD_C64, stream)
    try:
        Q.qd_batch_autotune_layers(b, ga, L)
        print("tuned fusion width", Q.qd_tune_get(Q.QD_TUNE_BATCH_FUSE), flush=True)
        Q.qd_batch_capture(b, True)
        Q.qd_batch_apply_layers(b, ga, L, 0)
        Q.qd_batch_capture(b, False)
        Q.qd_batch_replay(b)
        arena = Q.qd_batch_download(b)
    finally:
        Q.qd_batch_free(b)
        for prm in (Q.QD_TUNE_BATCH_FUSE, Q.QD_TUNE_BATCH_SPT_MID, Q.QD_TUNE_BATCH_SPT_WIDE):
            Q.qd_tune_set(prm, 0)
    offs = np.cumsum([0] + [c.D for c in circs])
    p = (arena.real.astype(np.float64) ** 2 + arena.imag.astype(np.float64) ** 2)
    norms = np.add.reduceat(p, offs[:-1])
    assert np.max(np.abs(norms - 1.0)) <= 4 * 100 * 32 * U24
    rng = C.seeded_rng(84)
    sample = sorted(set(rng.choice(len(circs), 12, replace=False).tolist()) | {int(np.argmin(offs[1:] - offs[:-1]))})
    for i in sample:
        psi = arena[offs[i]:offs[i + 1]]
        c = circs[i]
        if c.D <= 300_000:
            assert fidelity_loss(O.run_circuit(c), psi) <= 1e-6, i
        plain = run_gpu(c, Q.QD_C64, stream)
        assert max_abs(plain, psi) <= 4 * 100 * 32 * U24, i


def test_empty_layers_are_no_ops(stream):
    """No layers, and layers whose every slot is empty, leave the arena as it is at any width."""
    circs = small_batch(8, 6, seed=86)
    ga, L = all_layers(circs)
    nc = len(circs)
    b = Q.qd_batch_create([c.dims for c in circs], Q.QD_C128, stream)
    try:
        Q.qd_batch_apply_layers(b, ga, 3, 1)
        before = Q.qd_batch_download(b, np.complex128)
        Q.qd_batch_apply_layers(b, ga, 0, 4)
        empty = Q.GateArray([None] * (2 * nc), lambda j: circs[j % nc].dims)
        for w in (1, 2, 8):
            Q.qd_batch_apply_layers(b, empty, 2, w)
        assert np.array_equal(Q.qd_batch_download(b, np.complex128), before)
        # an empty layer between real ones changes nothing either
        mixed = Q.GateArray([circs[i].gates[0] for i in range(nc)] + [None] * nc + [circs[i].gates[1] for i in range(nc)],
                            lambda j: circs[j % nc].dims)
        Q.qd_batch_reset(b)
        Q.qd_batch_apply_layers(b, mixed, 3, 8)
        got = split(Q.qd_batch_download(b, np.complex128), b, circs)
    finally:
        Q.qd_batch_free(b)
    for c, psi in zip(circs, got):
        assert max_abs(psi, O.run_circuit(C.Circuit(c.dims, c.gates[:2]))) <= 1e-12
