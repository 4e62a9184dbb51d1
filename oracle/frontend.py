"""Oracle for the circuit front-end: the QuDiet QASM reader, Moment packing and the decomposition of
a multi-controlled Toffoli into generalized CNOTs through an intermediate level. TEST
INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU-baseline leg).

A gate here is a tuple (kind, target, a, controls, control_values): kind "X" (shift by a), "Z" or
"F" (the generalized Hadamard, QASM "H"), on one target qudit, with zero or more controls.

What the paper fixes:
  * QuDiet QASM (Sec. 4): ".qudit n", one "qudit NAME (d)" line per qudit, then the gates between
    ".begin" and ".end"; "X q" / "X q a" (shift a, default 1), "H q", "Z q", "CX c t" /
    "CX c t a". A generalized CNOT fires when its control holds d_c - 1 (Sec. 2.1).
  * Moments (Sec. 3.5): a pushed gate moves back through the preceding Moments while every qudit
    it acts on (targets and controls) holds an identity there, and stops at the initial state or
    at the first Moment where one of its qudits is busy. So a gate's Moment is one past the
    latest Moment of any earlier gate that shares a qudit with it (0-based: the first is 0).
  * Toffoli (Sec. 3.4): Toffoli((0, 1, 2), plus=1) becomes cx((0,1), +1), cx((1,2), +1),
    cx((0,1), +2) on wires whose middle one has an extra level.

Readings:
  * names are case-insensitive and '#' starts a comment: the paper's sample program writes one
    qudit's name with a capital letter, and one of its generalized CNOTs names the same qudit as
    control and target where the text describes the second qutrit acting on the third (such a line
    is rejected here). An "MCT c1 .. ck t [a]" line (extension) is a multi-controlled X whose
    controls fire on d_c - 1;
  * a multi-controlled X with controls c_1..c_k (values v_1..v_k) is decomposed as a chain:
    control c_{i-1} raises c_i by 1 (i = 2..k), so c_i reaches v_i + 1 exactly when c_1..c_i all
    hold their values; the last marker shifts the target; the chain is undone in reverse order
    with shifts d_{c_i} - 1 (i.e. -1). Marker of c_1 is v_1, of c_i (i >= 2) v_i + 1, which must be
    a level of that qudit (v_i + 2 <= d_{c_i}). For k = 2 on dims (2, 3, 2) this is the sequence
    printed in Sec. 3.4.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

__all__ = ["parse_qasm", "moments", "decompose_mct", "decompose_circuit", "QasmError"]

Gate = Tuple[str, int, int, Tuple[int, ...], Tuple[int, ...]]


class QasmError(ValueError):
    pass


def parse_qasm(text: str):
    """(names, dims, gates) of a QuDiet QASM program (Sec. 4)."""
    names: List[str] = []
    dims: List[int] = []
    gates: List[Gate] = []
    declared = None
    state = "head"   # head -> body -> done
    for lineno, raw in enumerate(text.splitlines(), 1):
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        tok = line.replace("(", " ( ").replace(")", " ) ").split()
        key = tok[0].lower()
        if state == "head":
            if key == ".qudit":
                if len(tok) != 2 or not tok[1].isdigit() or declared is not None:
                    raise QasmError(f"line {lineno}: bad .qudit")
                declared = int(tok[1])
            elif key == "qudit":
                if len(tok) != 5 or tok[2] != "(" or tok[4] != ")" or not tok[3].isdigit():
                    raise QasmError(f"line {lineno}: bad qudit declaration")
                name, d = tok[1].lower(), int(tok[3])
                if name in names or not 2 <= d <= 256:
                    raise QasmError(f"line {lineno}: duplicate qudit or dimension outside 2..256")
                names.append(name)
                dims.append(d)
            elif key == ".begin":
                if not names or (declared is not None and declared != len(names)):
                    raise QasmError(f"line {lineno}: qudit count does not match .qudit")
                state = "body"
            else:
                raise QasmError(f"line {lineno}: unexpected line before .begin")
            continue
        if state == "done":
            raise QasmError(f"line {lineno}: text after .end")
        if key == ".end":
            state = "done"
            continue
        args = tok[1:]
        shift = None
        if args:
            last = args[-1]
            body = last[1:] if last.startswith("-") else last
            if body.isascii() and body.isdigit() and len(body) <= 6:
                shift = int(last)
                args = args[:-1]
        try:
            wires = [names.index(a.lower()) for a in args]
        except ValueError:
            raise QasmError(f"line {lineno}: unknown qudit") from None
        if key in ("x", "h", "z"):
            if len(wires) != 1 or (key != "x" and shift is not None):
                raise QasmError(f"line {lineno}: bad {key.upper()} gate")
            t = wires[0]
            a = 1 if shift is None else shift
            if key == "x" and not 1 <= a <= dims[t] - 1:
                raise QasmError(f"line {lineno}: shift outside 1..d-1")
            gates.append(({"x": "X", "h": "F", "z": "Z"}[key], t, a if key == "x" else 0, (), ()))
        elif key in ("cx", "mct"):
            if len(wires) < 2 or (key == "cx" and len(wires) != 2) or len(set(wires)) != len(wires):
                raise QasmError(f"line {lineno}: bad {key.upper()} gate")
            ctl, t = tuple(wires[:-1]), wires[-1]
            a = 1 if shift is None else shift
            if not 1 <= a <= dims[t] - 1:
                raise QasmError(f"line {lineno}: shift outside 1..d-1")
            gates.append(("X", t, a, ctl, tuple(dims[c] - 1 for c in ctl)))
        else:
            raise QasmError(f"line {lineno}: unknown gate {tok[0]}")
    if state != "done":
        raise QasmError("missing .begin or .end")
    return names, dims, gates


def moments(gates: Sequence[Gate]) -> List[int]:
    """Moment of every gate (Sec. 3.5), 0-based."""
    last = {}
    out = []
    for kind, t, a, ctl, cv in gates:
        qs = (t,) + tuple(ctl)
        m = 1 + max((last[q] for q in qs if q in last), default=-1)
        out.append(m)
        for q in qs:
            last[q] = m
    return out


def decompose_mct(dims: Sequence[int], target: int, a: int, controls: Sequence[int],
                  values: Sequence[int]) -> List[Gate]:
    """Generalized CNOT chain for a multi-controlled X (Sec. 3.4 and the chain reading above)."""
    k = len(controls)
    if k <= 1:
        return [("X", target, a, tuple(controls), tuple(values))]
    for i in range(1, k):
        if values[i] + 2 > dims[controls[i]]:
            raise ValueError("control qudit has no level above its value for the intermediate marker")
    marker = [values[0]] + [v + 1 for v in values[1:]]
    out: List[Gate] = []
    for i in range(1, k):
        out.append(("X", controls[i], 1, (controls[i - 1],), (marker[i - 1],)))
    out.append(("X", target, a, (controls[-1],), (marker[-1],)))
    for i in range(k - 1, 0, -1):
        out.append(("X", controls[i], dims[controls[i]] - 1, (controls[i - 1],), (marker[i - 1],)))
    return out


def decompose_circuit(dims: Sequence[int], gates: Sequence[Gate]) -> List[Gate]:
    """Every X with two or more controls replaced by its chain; other gates unchanged."""
    out: List[Gate] = []
    for g in gates:
        kind, t, a, ctl, cv = g
        if kind == "X" and len(ctl) >= 2:
            out.extend(decompose_mct(dims, t, a, ctl, cv))
        else:
            out.append(g)
    return out
