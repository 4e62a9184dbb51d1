"""Pins of the front-end oracle (oracle/frontend.py): a QASM program whose final state is derived
by hand from the gate definitions of Sec. 2.1, the Moment rule of Sec. 3.5 simulated literally
(slide a pushed Moment back while its qudits hold identities), and the Toffoli decomposition of
Sec. 3.4, checked against the printed sequence and, by brute force, against the multi-controlled
X operator on the subspace where the intermediate levels are free."""
import itertools

import numpy as np
import pytest

import circuits as C
import oracle as O
from oracle import frontend as F

# Own test program (all constructs of the Sec. 4 QASM on a qutrit-qubit-ququart register).
# Hand derivation from |000>: H q -> (|0> + |1>)/sqrt2 on q; CX q p 2 (q fires on 1) -> p = 2 on
# the q = 1 branch; X r 3 -> r = 3; CX p r (p fires on 2) -> r = 3 + 1 = 0 (mod 4) on that branch;
# Z q -> phase omega_2 = -1 on q = 1. Final: (|0,0,3> - |2,1,0>)/sqrt2, flat indices 3 and 20.
PROGRAM = """
# hand-made program
.qudit 3
qudit P (3)
qudit q(2)
qudit r (4)
.begin
H q
CX q P 2
X r 3
cx p R      # names are case-insensitive
Z q
.end
"""


def to_circuit(dims, gates):
    out = []
    for kind, t, a, ctl, cv in gates:
        out.append(C.Gate(kind, (t,), tuple(ctl), tuple(cv), a=a if kind == "X" else 1))
    return C.Circuit(tuple(dims), out)


def test_program_parses_and_gives_the_hand_derived_state():
    names, dims, gates = F.parse_qasm(PROGRAM)
    assert names == ["p", "q", "r"] and dims == [3, 2, 4]
    assert gates == [("F", 1, 0, (), ()), ("X", 0, 2, (1,), (1,)), ("X", 2, 3, (), ()), ("X", 2, 1, (0,), (2,)),
                     ("Z", 1, 0, (), ())]
    psi = O.run_circuit(to_circuit(dims, gates))
    want = np.zeros(24, dtype=np.complex128)
    want[3] = 0.7071067811865475
    want[20] = -0.7071067811865475
    assert np.array_equal(psi, want)


MALFORMED = [
    ".qudit 2\nqudit a (2)\n.begin\n.end",                  # count mismatch
    "qudit a (2)\nqudit a (3)\n.begin\n.end",                # duplicate name
    "qudit a (1)\n.begin\n.end",                            # dimension
    "qudit a (2)\n.begin\nX a 2\n.end",                     # shift outside 1..d-1
    "qudit a (2)\nqudit b (2)\n.begin\nCX a a\n.end",       # control = target
    "qudit a (2)\n.begin\nY a\n.end",                       # unknown gate
    "qudit a (2)\n.begin\nX b\n.end",                       # unknown qudit
    "qudit a (2)\n.begin\nX a\n",                           # no .end
    "qudit a (2)\n.begin\nH a 1\n.end",                     # H takes no shift
    "qudit a (2)\n.begin\n.end\nX a",                       # after .end
]


@pytest.mark.parametrize("bad", MALFORMED)
def test_malformed_programs_are_rejected(bad):
    with pytest.raises(F.QasmError):
        F.parse_qasm(bad)


def slide_moments(n, gates):
    """The Sec. 3.5 process, literally: each gate is pushed as a new Moment (its qudits busy, the
    others identity) and swapped back while the previous Moment holds identities on all of its
    qudits."""
    stack = []          # list of Moments; a Moment is a list of gate indices per qudit (None = I)
    where = {}
    for gi, (kind, t, a, ctl, cv) in enumerate(gates):
        qs = (t,) + tuple(ctl)
        m = [None] * n
        for q in qs:
            m[q] = gi
        stack.append(m)
        pos = len(stack) - 1
        while pos > 0 and all(stack[pos - 1][q] is None for q in qs):
            for q in qs:
                stack[pos - 1][q], stack[pos][q] = gi, None
            pos -= 1
        where[gi] = pos
        if all(x is None for x in stack[-1]):
            stack.pop()
    return [where[i] for i in range(len(gates))]


def random_gates(rng, dims, count, max_ctl=3):
    n = len(dims)
    out = []
    for _ in range(count):
        t = int(rng.integers(n))
        others = [q for q in range(n) if q != t]
        m = int(rng.integers(0, min(max_ctl, len(others)) + 1))
        ctl = tuple(int(x) for x in rng.choice(others, m, replace=False)) if m else ()
        kind = ["X", "Z", "F"][int(rng.integers(3))] if not ctl else "X"
        a = int(rng.integers(1, dims[t])) if kind == "X" else 0
        out.append((kind, t, a, ctl, tuple(dims[c] - 1 for c in ctl)))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_moments_match_the_sliding_rule_and_keep_the_state(seed):
    rng = np.random.default_rng(seed)
    dims = [int(x) for x in rng.integers(2, 5, size=5)]
    gates = random_gates(rng, dims, 40)
    lay = F.moments(gates)
    assert lay == slide_moments(len(dims), gates)
    # a Moment never holds two gates on one qudit
    for m in set(lay):
        used = [q for g, l in zip(gates, lay) if l == m for q in (g[1],) + tuple(g[3])]
        assert len(used) == len(set(used))
    # running Moment by Moment (stable within a Moment) gives the same state
    order = sorted(range(len(gates)), key=lambda i: lay[i])
    a = O.run_circuit(to_circuit(dims, gates))
    b = O.run_circuit(to_circuit(dims, [gates[i] for i in order]))
    assert np.allclose(a, b, atol=1e-13, rtol=0)


def test_moment_depths_of_known_circuits():
    n = 6
    chain = [("X", q + 1, 1, (q,), (1,)) for q in range(n - 1)]      # CX ladder: depth n - 1
    assert F.moments(chain) == list(range(n - 1))
    brick = []
    for layer in range(4):
        for q in range(layer % 2, n - 1, 2):
            brick.append(("X", q + 1, 1, (q,), (1,)))
    assert max(F.moments(brick)) + 1 == 4
    assert F.moments([("F", q, 0, (), ()) for q in range(n)]) == [0] * n


def test_toffoli_decomposition_is_the_printed_sequence():
    # Toffoli((0, 1, 2), plus=1) on a qubit, an intermediate qutrit and a qubit (Sec. 3.4); each
    # generalized CNOT fires when its control holds d_c - 1
    got = F.decompose_mct([2, 3, 2], 2, 1, (0, 1), (1, 1))
    assert got == [("X", 1, 1, (0,), (1,)), ("X", 2, 1, (1,), (2,)), ("X", 1, 2, (0,), (1,))]


@pytest.mark.parametrize("dims,ctl,vals,t,a", [
    ([2, 3, 2], (0, 1), (1, 1), 2, 1),
    ([2, 3, 3, 2], (0, 1, 2), (1, 1, 1), 3, 1),
    ([3, 4, 4, 3], (0, 1, 2), (2, 0, 2), 3, 2),
    ([2, 3, 3, 3, 2], (0, 3, 1, 2), (1, 1, 0, 1), 4, 1),
    ([4, 3, 5], (2, 0), (3, 1), 1, 2),
])
def test_chain_equals_the_multi_controlled_gate(dims, ctl, vals, t, a):
    """Brute force over every basis state whose intermediate qudits are off their markers."""
    chain = F.decompose_mct(dims, t, a, ctl, vals)
    U = O.x_gate(dims[t], a)
    full = O.gate_operator(dims, (t,), ctl, vals, U)
    prod = np.eye(full.shape[0], dtype=np.complex128)
    for kind, tt, aa, cc, vv in chain:
        prod = O.gate_operator(dims, (tt,), cc, vv, O.x_gate(dims[tt], aa)) @ prod
    markers = {c: v + 1 for c, v in zip(ctl[1:], vals[1:])}
    for x in range(full.shape[0]):
        digs = O.digits_of(x, dims)
        if any(digs[c] == m for c, m in markers.items()):
            continue
        assert np.array_equal(prod[:, x], full[:, x]), (x, digs)
    assert len(chain) == 2 * len(ctl) - 1


def test_chain_needs_a_free_level():
    with pytest.raises(ValueError):
        F.decompose_mct([2, 2, 2], 2, 1, (0, 1), (1, 1))   # qudit 1 has no level above 1
    assert F.decompose_mct([2, 2], 1, 1, (0,), (1,)) == [("X", 1, 1, (0,), (1,))]


def test_decompose_circuit_keeps_other_gates():
    dims = [2, 3, 2]
    gates = [("F", 0, 0, (), ()), ("X", 2, 1, (0, 1), (1, 1)), ("Z", 1, 0, (), ())]
    out = F.decompose_circuit(dims, gates)
    assert out[0] == gates[0] and out[-1] == gates[-1] and len(out) == 5
