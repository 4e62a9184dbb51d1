"""GPU checks of the autotuners: tuned tile shapes keep results exact, tables round-trip through
their JSON files, and the cost-model fusion width builds a correct fused circuit."""
import numpy as np
import pytest

import circuits as C
import oracle as O
import paper_2211_07918_amd as Q
from gpu_util import fidelity_loss, max_abs, run_gpu, torch_stream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stream():
    return torch_stream()


@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
def test_autotune_keeps_results(stream, prec, tmp_path):
    c = C.config1_shrink(150)
    scratch = Q.qd_state_init(c.dims, prec, stream)
    path = str(tmp_path / "tune.json")
    try:
        Q.qd_autotune(scratch, path)
    finally:
        Q.qd_state_free(scratch)
    try:
        psi = run_gpu(c, prec, stream)
        ref = O.run_circuit(c)
        if prec == Q.QD_C128:
            assert max_abs(psi, ref) <= 1e-12
        else:
            assert fidelity_loss(ref, psi) <= 1e-6
        text = open(path).read()
        assert '"bucket": 0' in text and '"batch_block"' in text
        Q.qd_tune_load(path)
        psi2 = run_gpu(c, prec, stream)
        assert np.array_equal(psi, psi2)
    finally:
        Q.qd_tune_set(Q.QD_TUNE_RUN_MIN, 0)   # back to the defaults


def test_batch_autotune_restores_arena(stream):
    rng = C.seeded_rng(90)
    circs = []
    for _ in range(40):
        dims = C._batch_dims(rng, 1e2, 3e4)
        circs.append(C.Circuit(dims, [C.random_gate(dims, rng) for _ in range(6)]))
    b = Q.qd_batch_create([c.dims for c in circs], Q.QD_C128, stream)
    try:
        gas = [Q.GateArray([c.gates[l] for c in circs], lambda i: circs[i].dims) for l in range(6)]
        Q.qd_batch_apply_layer(b, gas[0])
        before = Q.qd_batch_download(b, np.complex128)
        Q.qd_batch_autotune(b, gas[1])
        assert np.array_equal(Q.qd_batch_download(b, np.complex128), before)
        for ga in gas[1:]:
            Q.qd_batch_apply_layer(b, ga)
        arena = Q.qd_batch_download(b, np.complex128)
    finally:
        Q.qd_batch_free(b)
        Q.qd_tune_set(Q.QD_TUNE_BATCH_BLOCK, 0)
    offs = np.cumsum([0] + [c.D for c in circs])
    for i, c in enumerate(circs):
        assert max_abs(arena[offs[i]:offs[i + 1]], O.run_circuit(c)) <= 1e-12


@pytest.mark.parametrize("make", [lambda: C.config2(6), lambda: C.config3(7, 8), lambda: C.config1_shrink(60)])
def test_auto_fusion_width(stream, make):
    circ = make()
    ga = Q.GateArray(circ.gates, lambda i: circ.dims)
    f = Q.qd_fuse(circ.dims, ga, 0, stream)
    try:
        Bs = [Q.qd_fused_block_info(f, b)["B"] for b in range(Q.qd_fused_count(f))]
        assert max(Bs) <= 128
        s = Q.qd_state_init(circ.dims, Q.QD_C128, stream)
        try:
            if circ.init_amps is not None:
                Q.qd_state_upload(s, circ.init_amps)
            Q.qd_apply_fused(s, f, Q.QD_MODE_FP64_PLAIN)
            assert max_abs(Q.qd_state_download(s), O.run_circuit(circ)) <= 1e-12
        finally:
            Q.qd_state_free(s)
    finally:
        Q.qd_fused_free(f)
