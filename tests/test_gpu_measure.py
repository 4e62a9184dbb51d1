"""GPU parity of the readout after the gates (qd_sample, qd_support, qd_marginals) against the
measurement oracle (oracle/measure.py), on the very amplitudes the GPU holds (downloaded).

Shots and support lists are integer work: bit-exact. Marginals are FP64 sums in another order:
1e-13 relative. Registers span several 64-amplitude chunks, several 128-chunk blocks and ragged
tails; the full-size case is the hybrid 20-qudit register after its 500 seeded gates."""
import numpy as np
import pytest

import circuits as C
import oracle as O
from oracle import measure as M
import paper_2211_07918_amd as Q
from gpu_util import torch_stream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stream():
    return torch_stream()


def rand_words(n, seed):
    return np.random.default_rng(seed).integers(0, 2 ** 64, n, dtype=np.uint64, endpoint=False)


def random_state(dims, seed, zero_frac=0.0):
    rng = np.random.default_rng(seed)
    D = int(np.prod(dims))
    psi = rng.normal(size=D) + 1j * rng.normal(size=D)
    if zero_frac:
        psi[rng.random(D) < zero_frac] = 0.0
    return psi / np.linalg.norm(psi)


def upload(dims, psi, prec, stream):
    s = Q.qd_state_init(dims, prec, stream)
    Q.qd_state_upload(s, psi)
    held = Q.qd_state_download(s)
    return s, held


def check_all(s, held, dims, shots=20000, seed=0, eps_list=(0.0,)):
    r = rand_words(shots, seed)
    r[:4] = [0, 1, 2 ** 63, 2 ** 64 - 1]
    got = Q.qd_sample(s, r)
    want = M.sample(held, r)
    assert np.array_equal(got, want)
    for eps in eps_list:
        idx, amps, probs, count = Q.qd_support(s, eps)
        w_idx = M.support(held, eps)
        assert count == w_idx.size
        assert np.array_equal(idx, w_idx)
        assert np.array_equal(amps, held[w_idx])
        assert np.array_equal(probs, M.exact_probabilities(held)[w_idx])
    got_m = Q.qd_marginals(s)
    for a, b in zip(got_m, M.marginals(held, dims)):
        assert np.allclose(a, b, rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
def test_worked_example(stream, prec):
    dims = (2, 3, 3)
    s = Q.qd_state_init(dims, prec, stream)
    try:
        for g in [C.Gate("F", (0,)), C.Gate("X", (1,), (0,), (1,), a=2)]:
            Q.apply_circuit_gate(s, g, dims)
        held = Q.qd_state_download(s)
        idx, amps, probs, count = Q.qd_support(s)
        assert idx.tolist() == [0, 15] and count == 2
        if prec == Q.QD_C128:
            assert [repr(float(a.real)) for a in amps] == ["0.7071067811865475"] * 2
        out = Q.kets(s, method="amplitude")
        assert [list(d.keys())[0] for d in out] == ["|000>", "|120>"]
        pk = Q.kets(s)
        assert [list(d.values())[0] for d in pk] == M.exact_probabilities(held)[[0, 15]].tolist()
        r = np.array([0, 2 ** 62, 2 ** 63 - 1, 2 ** 63, 2 ** 64 - 1], dtype=np.uint64)
        assert Q.qd_sample(s, r).tolist() == M.sample(held, r).tolist() == [0, 0, 0, 15, 15]
        check_all(s, held, dims, shots=500)
    finally:
        Q.qd_state_free(s)


@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
@pytest.mark.parametrize("dims", [(2, 3, 5, 7, 11, 13), (3,) * 9, (4, 2, 3, 4, 2, 3, 4), (7, 5), (2,)])
def test_random_states(stream, dims, prec):
    s, held = upload(dims, random_state(dims, 10 + len(dims)), prec, stream)
    try:
        check_all(s, held, dims, seed=len(dims), eps_list=(0.0, 1.0 / np.prod(dims)))
    finally:
        Q.qd_state_free(s)


@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
def test_many_blocks_and_segments(stream, prec):
    # 1728 blocks of 128 chunks: two per segment of the top-level scan; marginals over two levels
    dims = (2,) * 17 + (3, 3, 3) + (2, 2)
    psi = random_state(dims, 77, zero_frac=0.3)
    s, held = upload(dims, psi, prec, stream)
    try:
        check_all(s, held, dims, shots=30000, seed=5, eps_list=(0.0, 3e-8))
    finally:
        Q.qd_state_free(s)


@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
def test_sparse_and_extreme_states(stream, prec):
    dims = (2, 3) * 7 + (5,)
    D = int(np.prod(dims))
    rng = np.random.default_rng(3)
    # a few non-zero entries: in the first chunk, in a middle block, in the last (ragged) chunk
    psi = np.zeros(D, dtype=np.complex128)
    nz = [0, 5, 64 * 128 * 3 + 17, D // 2, D - 1]
    psi[nz] = rng.normal(size=len(nz)) + 1j * rng.normal(size=len(nz))
    psi /= np.linalg.norm(psi)
    s, held = upload(dims, psi, prec, stream)
    try:
        check_all(s, held, dims, shots=5000, seed=9)
        assert set(Q.qd_sample(s, rand_words(5000, 1)).tolist()) <= set(nz)
        # a basis state at the last index
        Q.qd_state_set_basis(s, [d - 1 for d in dims])
        held = Q.qd_state_download(s)
        assert np.all(Q.qd_sample(s, rand_words(1000, 2)) == D - 1)
        check_all(s, held, dims, shots=100, seed=4)
    finally:
        Q.qd_state_free(s)


def test_errors_and_determinism(stream):
    dims = (3, 4, 5)
    psi = random_state(dims, 4)
    s, held = upload(dims, 1.5 * psi, Q.QD_C128, stream)      # squared norm 2.25: still weighted
    try:
        r = rand_words(2000, 3)
        assert np.array_equal(Q.qd_sample(s, r), M.sample(held, r))
        Q.qd_state_upload(s, 2.1 * psi)                         # squared norm 4.41: rejected
        with pytest.raises(Q.QDError) as e:
            Q.qd_sample(s, r)
        assert e.value.code == Q.QD_EINVAL
        Q.qd_state_upload(s, 0 * psi)
        with pytest.raises(Q.QDError):
            Q.qd_sample(s, r)
        assert Q.qd_support(s)[3] == 0
        Q.qd_state_upload(s, psi)
        a = Q.qd_marginals(s)
        b = Q.qd_marginals(s)
        assert all(np.array_equal(x, y) for x, y in zip(a, b))
        assert Q.qd_sample(s, np.zeros(0, dtype=np.uint64)).size == 0
        with pytest.raises(Q.QDError):
            Q.qd_support(s, -1.0)
    finally:
        Q.qd_state_free(s)


def test_device_pointers(stream):
    import torch
    dims = (3, 3, 2, 5, 4)
    s, held = upload(dims, random_state(dims, 8), Q.QD_C64, stream)
    try:
        r = rand_words(4096, 6)
        rt = torch.from_numpy(r.view(np.int64)).to("cuda")
        out = torch.empty(4096, dtype=torch.int64, device="cuda")
        Q.qd_sample_device(s, rt.data_ptr(), 4096, out.data_ptr())
        assert np.array_equal(out.cpu().numpy(), M.sample(held, r))
    finally:
        Q.qd_state_free(s)


def test_hybrid_20_qudits_full_size(stream):
    """The benchmark's register (D = 107,495,424) after its 500 gates in complex128: 100,000 shots,
    the support count at 1e-12 and the marginals, against the oracle on the downloaded state."""
    circ = C.config1()
    s = Q.qd_state_init(circ.dims, Q.QD_C128, stream)
    try:
        for g in circ.gates:
            Q.apply_circuit_gate(s, g, circ.dims)
        held = Q.qd_state_download(s)
        r = rand_words(100_000, 11)
        assert np.array_equal(Q.qd_sample(s, r), M.sample(held, r))
        _, _, _, count = Q.qd_support(s, 1e-12, max_out=0)
        assert count == M.support(held, 1e-12).size
        for a, b in zip(Q.qd_marginals(s), M.marginals(held, circ.dims)):
            assert np.allclose(a, b, rtol=1e-12, atol=1e-300)
    finally:
        Q.qd_state_free(s)
