"""qd_norm2_noalloc (partials in a static device array, result written to caller device memory)
against qd_norm2 through the C ABI: bitwise equal, on consecutive calls whose second input is
smaller than the first, in both precisions."""
import numpy as np
import pytest

import paper_2211_07918_amd as Q
from gpu_util import torch_stream

pytestmark = pytest.mark.gpu


def _state(dims, prec, stream, seed):
    rng = np.random.default_rng(seed)
    D = int(np.prod(dims))
    amps = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    amps /= np.linalg.norm(amps)
    s = Q.qd_state_init(dims, prec, stream)
    Q.qd_state_upload(s, amps)
    return s


@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
def test_noalloc_norm_matches_qd_norm2(prec):
    import torch
    stream = torch_stream()
    # a register whose reduction uses every one of the 2048 partials, then one of 24 amplitudes
    # (a single partial), then the large one again: nothing of an earlier call may leak
    cases = [((2,) * 10 + (3,) * 8, 11), ((3, 2, 4), 12), ((2,) * 10 + (3,) * 8, 13), ((5, 7), 14)]
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    for i, (dims, seed) in enumerate(cases):
        s = _state(dims, prec, stream, seed)
        try:
            Q.qd_norm2_noalloc(s, out.data_ptr() + 8 * i)
            torch.cuda.synchronize()
            got = float(out[i].item())
            want = Q.qd_norm2(s)
        finally:
            Q.qd_state_free(s)
        print(f"noalloc norm2 prec={prec} dims={dims}: {got!r} vs {want!r}", flush=True)
        assert got == want, (dims, got, want)
        assert abs(got - 1.0) < (1e-12 if prec == Q.QD_C128 else 1e-5)


def test_noalloc_norm_rejects_null_output():
    stream = torch_stream()
    s = Q.qd_state_init((2, 3), Q.QD_C128, stream)
    try:
        with pytest.raises(Q.QDError) as e:
            Q.qd_norm2_noalloc(s, 0)
        assert e.value.code == Q.QD_EINVAL
    finally:
        Q.qd_state_free(s)
