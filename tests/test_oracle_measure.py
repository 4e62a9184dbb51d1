"""Pins of the measurement oracle (oracle/measure.py) against what the paper and the mathematics fix:
the worked example of Sec. 3.9, the Born rule of Sec. 2.1.1 (statistically), closed forms for
basis, uniform and GHZ states, brute-force digit enumeration for marginals, and the boundary
behaviour of the inverse cumulative distribution."""
import json
import os

import numpy as np
import pytest

import circuits as C
import oracle as O
from oracle import measure as M

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")


def worked_example():
    g = json.load(open(GOLDEN))
    dims = tuple(g["dims"])
    circ = C.Circuit(dims, [C.Gate("F", (0,)), C.Gate("X", (1,), (0,), (1,), a=2)])
    return g, dims, O.run_circuit(circ)


def test_worked_example_support_kets_and_amplitudes():
    g, dims, psi = worked_example()
    idx = M.support(psi)
    kets = [M.ket_string(int(i), dims) for i in idx]
    assert kets == ["|" + k + ">" for k in g["expected_amplitudes"]]
    for i, k in zip(idx, g["expected_amplitudes"]):
        assert repr(float(psi[i].real)) == g["expected_amplitudes"][k]
        assert psi[i].imag == 0.0


def test_worked_example_marginals_and_shots():
    _, dims, psi = worked_example()
    m = M.marginals(psi, dims)
    p = 0.7071067811865475 ** 2
    assert np.allclose(m[0], [p, p], rtol=0, atol=1e-16)
    assert np.allclose(m[1], [p, 0.0, p], rtol=0, atol=1e-16)
    assert np.allclose(m[2], [2 * p, 0.0, 0.0], rtol=0, atol=1e-16)
    # two equal weights: the lower half of the random words draws |000>, the upper half |120>
    r = np.array([0, 2 ** 62, 2 ** 63 - 1, 2 ** 63, 3 * 2 ** 62, 2 ** 64 - 1], dtype=np.uint64)
    assert M.sample(psi, r).tolist() == [0, 0, 0, 15, 15, 15]


def test_boundary_falls_to_the_next_state_with_weight():
    # p = (1/4, 0, 1/4, 1/2) exactly: weights 2^60, 0, 2^60, 2^61 (total 2^62); r = 2^62 puts t on
    # the first boundary, which belongs to the next state with weight
    psi = np.array([0.5, 0.0, 0.5, 0.5 + 0.5j], dtype=np.complex128)
    assert M.sample_weights(psi).tolist() == [2 ** 60, 0, 2 ** 60, 2 ** 61]
    r = np.array([0, 2 ** 62 - 1, 2 ** 62, 2 ** 63 - 1, 2 ** 63, 2 ** 64 - 1], dtype=np.uint64)
    assert M.sample(psi, r).tolist() == [0, 0, 2, 2, 3, 3]


@pytest.mark.parametrize("dims,values", [((3, 2, 4), (2, 1, 3)), ((5,), (4,)), ((2, 2, 2, 2), (0, 1, 1, 0))])
def test_basis_state(dims, values):
    psi = O.basis_state(dims, values)
    x = O.index_of(values, dims)
    r = np.random.default_rng(1).integers(0, 2 ** 64, 100, dtype=np.uint64, endpoint=False)
    r[:2] = [0, 2 ** 64 - 1]
    assert np.all(M.sample(psi, r) == x)
    assert M.support(psi).tolist() == [x]
    m = M.marginals(psi, dims)
    for q, v in enumerate(values):
        assert m[q].tolist() == [1.0 if j == v else 0.0 for j in range(dims[q])]


@pytest.mark.parametrize("k", [1, 3, 6])
def test_uniform_superposition_closed_form(k):
    # F_2 on every qubit: all 2^k probabilities are the same FP64 number, so the weights are equal
    dims = (2,) * k
    circ = C.Circuit(dims, [C.Gate("F", (q,)) for q in range(k)])
    psi = O.run_circuit(circ)
    w = M.sample_weights(psi)
    assert len(set(w.tolist())) == 1
    # equal weights w, total 2^k w: t = floor(r 2^k w / 2^64), so the shot is the top k bits of r
    r = np.concatenate([np.arange(2 ** k, dtype=np.uint64) << np.uint64(64 - k),
                        np.random.default_rng(2).integers(0, 2 ** 64, 200, dtype=np.uint64, endpoint=False)])
    assert np.array_equal(M.sample(psi, r), (r >> np.uint64(64 - k)).astype(np.int64))
    for m in M.marginals(psi, dims):
        assert np.allclose(m, 0.5, atol=1e-15)


@pytest.mark.parametrize("d,n", [(3, 3), (4, 2), (2, 5)])
def test_ghz_marginals_and_support(d, n):
    dims = (d,) * n
    gates = [C.Gate("F", (0,))]
    for k in range(1, n):
        for v in range(1, d):
            gates.append(C.Gate("X", (k,), (0,), (v,), a=v))
    psi = O.run_circuit(C.Circuit(dims, gates))
    sup = M.support(psi, 1e-12)
    assert sup.tolist() == [O.index_of([j] * n, dims) for j in range(d)]
    for m in M.marginals(psi, dims):
        assert np.allclose(m, 1.0 / d, atol=1e-15)


def test_marginals_brute_force_enumeration():
    rng = np.random.default_rng(5)
    dims = (3, 2, 4, 3)
    D = int(np.prod(dims))
    psi = rng.normal(size=D) + 1j * rng.normal(size=D)
    psi /= np.linalg.norm(psi)
    p = np.abs(psi) ** 2
    want = [np.zeros(d) for d in dims]
    for x in range(D):
        for q, v in enumerate(O.digits_of(x, dims)):
            want[q][v] += p[x]
    got = M.marginals(psi, dims)
    for a, b in zip(got, want):
        assert np.allclose(a, b, rtol=0, atol=1e-15)
        assert abs(a.sum() - 1.0) < 1e-14


def test_shot_frequencies_follow_the_born_rule():
    rng = np.random.default_rng(6)
    D = 12
    psi = rng.normal(size=D) + 1j * rng.normal(size=D)
    psi[[3, 7]] = 0.0
    psi /= np.linalg.norm(psi)
    p = np.abs(psi) ** 2
    shots = 200_000
    r = rng.integers(0, 2 ** 64, shots, dtype=np.uint64, endpoint=False)
    counts = np.bincount(M.sample(psi, r), minlength=D)
    assert counts[3] == 0 and counts[7] == 0
    nz = p > 0
    chi2 = float(np.sum((counts[nz] - shots * p[nz]) ** 2 / (shots * p[nz])))
    # 9 degrees of freedom: P(chi2 > 30) ~ 4e-4
    assert chi2 < 30.0, chi2


def test_support_threshold_and_ket_format():
    psi = np.array([1e-9, 0.0, 0.6, 0.8j, 0.0, 0.0], dtype=np.complex128)
    assert M.support(psi).tolist() == [0, 2, 3]
    assert M.support(psi, 1e-12).tolist() == [2, 3]
    assert M.ket_string(5, (2, 3)) == "|12>"
    assert M.ket_string(13 * 3 + 2, (2, 16, 3)) == "|0,13,2>"
    with pytest.raises(ValueError):
        M.ket_string(6, (2, 3))


def test_sampling_rejects_bad_inputs():
    psi = np.array([1.0, 1.0, 1.0, 1.0], dtype=np.complex128)    # squared norm 4
    with pytest.raises(ValueError):
        M.sample(psi, np.array([5], dtype=np.uint64))
    with pytest.raises(ValueError):
        M.sample(np.zeros(3, dtype=np.complex128), np.array([5], dtype=np.uint64))
