"""Host-side checks of libqd (CPU only: no call here touches a GPU).

* the library loads and exports every function include/qd.h declares;
* register strides, named gate matrices and gate classes agree with the oracle / definitions;
* every validation error code of qd_apply_gate is produced by qd_validate_gate;
* the fusion planner returns valid in-order partitions within the block bound;
* the magic-number division used by the kernels is exact (compiled with g++ on the host).
"""
import os
import re
import subprocess

import numpy as np
import pytest

import circuits as C
import oracle as O
import paper_2211_07918_amd as Q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qd.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(qd_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = Q.load()
    names = _declared_functions()
    assert len(names) >= 40
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wraps each of them under the same name
    assert not [n for n in names if not hasattr(Q, n)]


def test_nm_shows_c_linkage():
    out = subprocess.run(["nm", "-D", "--defined-only", Q.lib_path()], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (qd_[a-z0-9_]+)$", out, flags=re.M))
    assert set(_declared_functions()) <= exported


@pytest.mark.parametrize("dims", [(2,), (3, 2, 4), (2, 3, 3), (4,) * 14, (3,) * 20, (256, 2, 255)])
def test_register_strides(dims):
    D, st = Q.qd_register_strides(dims)
    assert D == O.register_size(dims)
    assert st == O.strides(dims)


def test_register_errors():
    with pytest.raises(Q.QDError) as e:
        Q.qd_register_strides([2, 1])
    assert e.value.code == Q.QD_EDIM
    with pytest.raises(Q.QDError) as e:
        Q.qd_register_strides([257])
    assert e.value.code == Q.QD_EDIM
    with pytest.raises(Q.QDError) as e:
        Q.qd_register_strides([2] * 65)
    assert e.value.code == Q.QD_EINVAL
    with pytest.raises(Q.QDError) as e:
        Q.qd_register_strides([256] * 8)          # 2^64 overflows int64
    assert e.value.code == Q.QD_EOVERFLOW


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6, 7, 8, 9, 16, 255, 256])
def test_named_gates_match_oracle(d):
    assert np.array_equal(Q.qd_gate_matrix(Q.QD_GATE_Z, d), O.z_gate(d))
    assert np.array_equal(Q.qd_gate_matrix(Q.QD_GATE_F, d), O.f_gate(d))
    assert np.array_equal(Q.qd_gate_matrix(Q.QD_GATE_I, d), np.eye(d))
    for a in sorted({1, d // 2, d - 1}):
        assert np.array_equal(Q.qd_gate_matrix(Q.QD_GATE_X, d, a), O.x_gate(d, a))


def test_named_gate_errors():
    for a in (0, 3, -1):
        with pytest.raises(Q.QDError) as e:
            Q.qd_gate_matrix(Q.QD_GATE_X, 3, a)
        assert e.value.code == Q.QD_EINVAL
    with pytest.raises(Q.QDError) as e:
        Q.qd_gate_matrix(7, 3)
    assert e.value.code == Q.QD_EINVAL
    with pytest.raises(Q.QDError) as e:
        Q.qd_gate_matrix(Q.QD_GATE_F, 1)
    assert e.value.code == Q.QD_EDIM


def test_validation_codes():
    dims = [2, 3, 4]
    X3 = O.x_gate(3, 1)
    ok = Q.qd_validate_gate
    assert ok(dims, [1], [0], [1], X3) == Q.QD_OK
    assert ok(dims, [1], [1], [0], X3) == Q.QD_EINVAL            # control == target
    assert ok(dims, [1, 1], [], [], np.eye(9)) == Q.QD_EINVAL    # duplicate target
    assert ok(dims, [3], [], [], X3) == Q.QD_EINVAL              # target out of range
    assert ok(dims, [1], [0], [2], X3) == Q.QD_EINVAL            # control value >= d_c
    assert ok(dims, [1], [0], [-1], X3) == Q.QD_EINVAL
    assert ok(dims, [1], [5], [0], X3) == Q.QD_EINVAL            # control out of range
    assert ok(dims, [1], [0, 0], [0, 1], X3) == Q.QD_EINVAL      # duplicate control
    assert ok(dims, [], [], [], X3) == Q.QD_EINVAL               # no target
    assert ok([2, 2, 2], [0, 1, 2], [0], [0], np.eye(8)) == Q.QD_EINVAL  # k + m > n
    bad = np.ones((3, 3)) / 3.0
    assert ok(dims, [1], [], [], bad) == Q.QD_ENOTUNITARY
    assert ok(dims, [1], [], [], bad, Q.QD_FLAG_SKIP_UNITARY_CHECK) == Q.QD_OK
    nan = X3.copy()
    nan[0, 0] = np.nan
    assert ok(dims, [1], [], [], nan, Q.QD_FLAG_SKIP_UNITARY_CHECK) == Q.QD_ENOTUNITARY
    assert ok([4] * 6, [0, 1, 2, 3, 4, 5], [], [], np.eye(4096)) == Q.QD_EDIM  # d_T > 1024
    assert ok(dims, [2], [], [], X3) == Q.QD_EDIM                # U size != d_T (binding check)
    assert ok(dims, [1], [], [], X3 * (1 + 1e-9)) == Q.QD_ENOTUNITARY
    assert ok(dims, [1], [], [], X3 * (1 + 1e-12)) == Q.QD_OK


def test_gate_classes():
    assert Q.qd_gate_class(O.z_gate(5)) == Q.QD_CLASS_DIAGONAL
    assert Q.qd_gate_class(O.x_gate(5, 2)) == Q.QD_CLASS_MONOMIAL
    assert Q.qd_gate_class(O.f_gate(3)) == Q.QD_CLASS_DENSE
    sw = C.qudit_qft_gates(4, 2)[-1].U
    assert Q.qd_gate_class(sw) == Q.QD_CLASS_MONOMIAL
    assert Q.qd_gate_class(np.diag(np.exp(1j * np.arange(16)))) == Q.QD_CLASS_DIAGONAL
    assert Q.qd_gate_class(np.eye(1)) == Q.QD_CLASS_DIAGONAL


def test_routes():
    dims = [2, 3, 4, 3, 2, 2, 3, 2, 2, 2]   # strides of the last qudits are 1, 2, 4, 8, ...
    r = lambda t, U, c=(), v=(), prec=Q.QD_C128: Q.qd_gate_route(dims, prec, t, c, v, U)
    assert r([0], O.f_gate(2)) == Q.QD_ROUTE_DIRECT
    assert r([9], O.f_gate(2)) == Q.QD_ROUTE_TILED
    assert r([6], O.f_gate(3)) == Q.QD_ROUTE_TILED
    assert r([9], O.z_gate(2)) == Q.QD_ROUTE_DIAG
    assert r([1], O.x_gate(3, 1), [0], [1]) == Q.QD_ROUTE_DIRECT
    assert r([1, 2], np.eye(12)[::-1]) == Q.QD_ROUTE_DIRECT        # monomial d_T = 12
    assert r([1, 2], C.haar_unitary(12, C.seeded_rng(1))) == Q.QD_ROUTE_DIRECT      # dense 12, large strides
    assert r([2, 6], C.haar_unitary(12, C.seeded_rng(1))) == Q.QD_ROUTE_GEMM        # dense 12, a small stride
    assert r([1, 2, 3], C.haar_unitary(36, C.seeded_rng(1))) == Q.QD_ROUTE_GEMM
    assert r([1, 2, 3, 0], C.haar_unitary(72, C.seeded_rng(1))) == Q.QD_ROUTE_GENERIC  # above 64
    assert r([1, 2, 3], np.eye(36)[::-1]) == Q.QD_ROUTE_GEMM                       # monomial, no fast case
    Q.qd_tune_set(Q.QD_TUNE_RUN_MIN, 1)
    try:
        assert r([9], O.f_gate(2)) == Q.QD_ROUTE_DIRECT
    finally:
        Q.qd_tune_set(Q.QD_TUNE_RUN_MIN, 0)
    assert Q.qd_tune_get(Q.QD_TUNE_RUN_MIN) == 16


def _skips_lines(dims, controls, values, line):
    """Whether some 128-byte line (`line` amplitudes) holds no amplitude where every control of
    stride below a line has its value, judged over one period of those controls' digit pattern
    (at most 64 lines, as the library looks; a longer period counts as no skip)."""
    st = O.strides(dims)
    low = [(st[c], dims[c], v) for c, v in zip(controls, values) if st[c] < line]
    P = 1
    for s, d, _ in low:
        P = np.lcm(P, s * d)
    per = int(np.lcm(P, line) // line)
    if per < 2 or per > 64:
        return False
    i = np.arange(per * line)
    match = np.ones(i.size, bool)
    for s, d, v in low:
        match &= (i // s) % d == v
    return not match.reshape(per, line).any(axis=1).all()


@pytest.mark.parametrize("prec", [Q.QD_C128, Q.QD_C64])
def test_inline_control_route_rule(prec):
    """Controls inside a line (stride below one 128-byte line) leave the tile geometry as it is
    without them, so such a gate takes the route of its uncontrolled form, except that it moves to
    the direct kernel (which skips lines) when its controls leave some line without a matching
    amplitude and every target stride is at least one line. Run threshold raised to 1024 so that
    the tile route is the rule; seeded registers of qubits to ququints, one or two targets."""
    line = 8 if prec == Q.QD_C128 else 16
    rng = np.random.default_rng(2211)
    Q.qd_tune_set(Q.QD_TUNE_RUN_MIN, 1024)
    try:
        seen = {}
        for _ in range(600):
            n = int(rng.integers(6, 10))
            dims = [int(x) for x in rng.integers(2, 6, size=n)]
            st = O.strides(dims)
            inl = [q for q in range(n) if st[q] < line]
            m = int(rng.integers(1, 3))
            if len(inl) < m:
                continue
            c = [int(x) for x in rng.permutation(inl)[:m]]
            rest = [q for q in range(n) if q not in c and st[q] < 1024]
            k = int(rng.integers(1, 3))
            if len(rest) < k:
                continue
            t = [int(x) for x in rng.permutation(rest)[:k]]
            v = [int(rng.integers(0, dims[q])) for q in c]
            dT = int(np.prod([dims[q] for q in t]))
            U = C.haar_unitary(dT, rng)
            plain = Q.qd_gate_route(dims, prec, t, [], [], U)
            got = Q.qd_gate_route(dims, prec, t, c, v, U)
            if plain not in (Q.QD_ROUTE_DIRECT, Q.QD_ROUTE_TILED):
                continue   # d_T beyond the slice kernels: GEMM or generic
            skip = min(st[q] for q in t) >= line and _skips_lines(dims, c, v, line)
            want = Q.QD_ROUTE_DIRECT if (plain == Q.QD_ROUTE_TILED and skip) else plain
            assert got == want, (dims, t, c, v, prec)
            key = "moved" if plain != want else ("tiled" if want == Q.QD_ROUTE_TILED else "direct")
            seen[key] = seen.get(key, 0) + 1
        assert seen.get("tiled", 0) >= 50 and seen.get("moved", 0) >= 50, seen
    finally:
        Q.qd_tune_set(Q.QD_TUNE_RUN_MIN, 0)


def test_tune_parameters():
    for p, v in ((Q.QD_TUNE_DIRECT_BLOCK, 128), (Q.QD_TUNE_DIRECT_SPT, 1), (Q.QD_TUNE_TILE_ELEMS, 1024),
                 (Q.QD_TUNE_BATCH_GRID, 16)):
        old = Q.qd_tune_get(p)
        Q.qd_tune_set(p, v)
        assert Q.qd_tune_get(p) == v
        Q.qd_tune_set(p, 0)
        assert Q.qd_tune_get(p) == old
    for p, v in ((Q.QD_TUNE_DIRECT_BLOCK, 100), (Q.QD_TUNE_DIRECT_SPT, 3), (Q.QD_TUNE_TILE_ELEMS, 1000),
                 (Q.QD_TUNE_BATCH_GRID, 65), (Q.QD_TUNE_BATCH_FUSE, 9), (Q.QD_TUNE_BATCH_SPT_MID, 3),
                 (Q.QD_TUNE_BATCH_SPT_WIDE, 16), (42, 1)):
        with pytest.raises(Q.QDError):
            Q.qd_tune_set(p, v)


def test_batch_slice_class_parameters():
    """Slices per thread of the wide batched slice classes: 0 is the default rule, else 1, 2, 4, 8."""
    for p in (Q.QD_TUNE_BATCH_SPT_MID, Q.QD_TUNE_BATCH_SPT_WIDE):
        assert Q.qd_tune_get(p) == 0
        for v in (1, 2, 4, 8, 0):
            Q.qd_tune_set(p, v)
            assert Q.qd_tune_get(p) == v


# ------------------------------------------------------------------------------ fusion planner
def _is_diag(g, dims):
    U = O.gate_unitary(g, dims)
    return not np.any(U - np.diag(np.diag(U)))


def _check_plan(dims, gates, blocks, nb, maxb):
    assert len(blocks) == len(gates) and sorted(set(blocks)) == list(range(nb))
    for b in range(nb):
        win = set(q for g, bb in zip(gates, blocks) if bb == b for q in g.qudits())
        assert int(np.prod([dims[q] for q in win])) <= maxb
    # gates that do not commute keep their order
    diag = [_is_diag(g, dims) for g in gates]
    for i in range(len(gates)):
        for j in range(i + 1, len(gates)):
            if set(gates[i].qudits()) & set(gates[j].qudits()) and not (diag[i] and diag[j]):
                assert blocks[i] <= blocks[j], (i, j)
    # block b starts with the earliest gate not placed in an earlier block
    for b in range(nb):
        first = min(i for i, bb in enumerate(blocks) if bb == b)
        assert all(blocks[i] < b for i in range(first))


@pytest.mark.parametrize("maxb", [16, 64, 81, 128])
def test_fuse_plan_valid(maxb):
    for circ in (C.config2(6), C.config3(8, 6), C.config1_shrink(60), C.config0()):
        gates = [g for g in circ.gates if np.prod([circ.dims[q] for q in g.qudits()]) <= maxb]
        blocks, nb = Q.qd_fuse_plan(circ.dims, gates, maxb)
        _check_plan(circ.dims, gates, blocks, nb, maxb)


@pytest.mark.parametrize("make,maxb", [(lambda: C.config2(5), 64), (lambda: C.config3(6, 8), 81),
                                       (lambda: C.config1_shrink(120), 27), (lambda: C.config0(), 27)])
def test_fuse_plan_order_is_exact(make, maxb):
    """Applying the gates block by block (members in circuit order) gives the circuit's state."""
    circ = make()
    if circ.init_amps is None:
        circ.init_amps = C.random_basis_superposition(circ.D, 20, C.seeded_rng(8))
    blocks, nb = Q.qd_fuse_plan(circ.dims, circ.gates, maxb)
    order = [i for b in range(nb) for i, bb in enumerate(blocks) if bb == b]
    assert sorted(order) == list(range(len(circ.gates)))
    reordered = C.Circuit(circ.dims, [circ.gates[i] for i in order], init_amps=circ.init_amps)
    assert np.max(np.abs(O.run_circuit(reordered) - O.run_circuit(circ))) <= 1e-13


def test_fuse_plan_counts():
    c2 = C.config2(14)
    _, nb = Q.qd_fuse_plan(c2.dims, c2.gates, 64)
    assert nb <= 50
    c3 = C.config3(20, 30)
    _, nb = Q.qd_fuse_plan(c3.dims, c3.gates, 81)
    assert nb <= 110


def test_fuse_plan_errors():
    c = C.config3(4, 2)
    with pytest.raises(Q.QDError) as e:
        Q.qd_fuse_plan(c.dims, c.gates, 8)       # a 9x9 gate does not fit
    assert e.value.code == Q.QD_EDIM
    with pytest.raises(Q.QDError) as e:
        Q.qd_fuse_plan(c.dims, c.gates, 129)
    assert e.value.code == Q.QD_EINVAL


# ------------------------------------------------------------------------------ magic division
def test_magic_division_exact(tmp_path):
    src = tmp_path / "magic_check.cpp"
    src.write_text(r'''
#include <cstdio>
#include <cstdint>
#include <random>
#include "qd_magic.h"
int main() {
  std::mt19937_64 rng(7);
  const uint32_t edge[] = {0u, 1u, 2u, 3u, 255u, 256u, 65535u, 65536u, 2147483647u, 2147483648u,
                           4294967294u, 4294967295u, 3486784400u, 107495423u};
  uint64_t bad = 0, n_checks = 0;
  auto check = [&](uint32_t d, uint32_t n) {
    const qd::Magic32 m = qd::make_magic32(d);
    ++n_checks;
    if (qd::magic_div(n, m) != n / d) ++bad;
  };
  for (uint32_t d = 1; d <= 4096; ++d) {
    for (uint32_t n : edge) check(d, n);
    for (int i = 0; i < 2000; ++i) check(d, uint32_t(rng()));
    for (uint32_t q = 1; q < 64; ++q) {           // around multiples of d
      const uint64_t base = uint64_t(q) * d * 977u;
      if (base + 1 < 4294967296ull && base >= 1) { check(d, uint32_t(base)); check(d, uint32_t(base - 1)); check(d, uint32_t(base + 1)); }
    }
  }
  const uint32_t bigd[] = {6561u, 59049u, 531441u, 1u << 20, 3486784401u, 4294967295u, 107495424u};
  for (uint32_t d : bigd) { for (uint32_t n : edge) check(d, n); for (int i = 0; i < 100000; ++i) check(d, uint32_t(rng())); }
  std::printf("%llu %llu\n", (unsigned long long)bad, (unsigned long long)n_checks);
  return bad != 0;
}
''')
    exe = tmp_path / "magic_check"
    inc = os.path.join(ROOT, "paper_2211_07918_amd", "csrc")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", inc, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    bad, total = map(int, r.stdout.split())
    assert r.returncode == 0 and bad == 0 and total > 8_000_000


# ------------------------------------------------------------------------------ tuning table files
def test_tune_load_and_save(tmp_path):
    dims = [2, 3, 4, 3, 2, 2, 3, 2, 2, 2]
    F4 = O.f_gate(4)
    assert Q.qd_gate_route(dims, Q.QD_C128, [2], [], [], F4) == Q.QD_ROUTE_DIRECT
    p = tmp_path / "tune.json"
    # stride class 4 (256-4095) tiled: qudit 2 (stride 288) is staged in LDS
    p.write_text('[\n{"prec": 0, "bucket": 4, "tiled": 1, "block": 256, "spt": 1, "tile_elems": 2048},\n'
                 '{"batch_block": 128, "batch_spt": 4, "batch_grid": 32, "batch_fuse": 6, "batch_spt_mid": 2, '
                 '"batch_spt_wide": 1}\n]\n')
    Q.qd_tune_load(str(p))
    try:
        assert Q.qd_gate_route(dims, Q.QD_C128, [2], [], [], F4) == Q.QD_ROUTE_TILED
        assert Q.qd_tune_get(Q.QD_TUNE_BATCH_BLOCK) == 128 and Q.qd_tune_get(Q.QD_TUNE_BATCH_SPT) == 4
        assert Q.qd_tune_get(Q.QD_TUNE_BATCH_GRID) == 32 and Q.qd_tune_get(Q.QD_TUNE_BATCH_FUSE) == 6
        assert Q.qd_tune_get(Q.QD_TUNE_BATCH_SPT_MID) == 2 and Q.qd_tune_get(Q.QD_TUNE_BATCH_SPT_WIDE) == 1
        out = tmp_path / "saved.json"
        Q.qd_tune_save(str(out))
        text = out.read_text()
        assert '"bucket": 4, "tiled": 1' in text
        assert '"batch_fuse": 6, "batch_spt_mid": 2, "batch_spt_wide": 1' in text
    finally:
        # an explicit setting discards the tuned table and restores the defaults
        for prm in (Q.QD_TUNE_BATCH_BLOCK, Q.QD_TUNE_BATCH_SPT, Q.QD_TUNE_BATCH_GRID, Q.QD_TUNE_BATCH_FUSE,
                    Q.QD_TUNE_BATCH_SPT_MID, Q.QD_TUNE_BATCH_SPT_WIDE):
            Q.qd_tune_set(prm, 0)
    assert Q.qd_gate_route(dims, Q.QD_C128, [2], [], [], F4) == Q.QD_ROUTE_DIRECT
    bad = tmp_path / "bad.json"
    bad.write_text('[{"prec": 0, "bucket": 9, "tiled": 1, "block": 256, "spt": 1, "tile_elems": 2048}]\n')
    with pytest.raises(Q.QDError):
        Q.qd_tune_load(str(bad))
    with pytest.raises(Q.QDError):
        Q.qd_tune_load(str(tmp_path / "missing.json"))


def test_tune_stride_classes_split_at_4096(tmp_path):
    """Target strides of 256-4095 amplitudes (class 4) and of 4096 or more (class 5) take separate
    tuned entries: a tiled entry for class 4 routes a complex64 qubit gate of stride 2048 to the LDS
    tile kernel and leaves the qubit of stride 4096 on the direct kernel; class 5 entries load and
    save; class 6 does not exist."""
    dims = [2] * 14                       # qudit 1: stride 4096, qudit 2: stride 2048
    X2 = O.x_gate(2, 1)
    entry = '{"prec": 1, "bucket": %d, "tiled": %d, "block": 256, "spt": 1, "tile_elems": 4096}'
    p = tmp_path / "tune.json"
    try:
        for b, tiled in ((4, 1), (5, 0)):
            p.write_text("[\n" + entry % (b, tiled) + "\n]\n")
            Q.qd_tune_load(str(p))
            assert Q.qd_gate_route(dims, Q.QD_C64, [2], [], [], X2) == (Q.QD_ROUTE_TILED if b == 4 else Q.QD_ROUTE_DIRECT)
            assert Q.qd_gate_route(dims, Q.QD_C64, [1], [], [], X2) == Q.QD_ROUTE_DIRECT
            out = tmp_path / "saved.json"
            Q.qd_tune_save(str(out))
            assert ('"bucket": %d, "tiled": %d, "block": 256' % (b, tiled)) in out.read_text()
        p.write_text("[\n" + entry % (6, 0) + "\n]\n")
        with pytest.raises(Q.QDError):
            Q.qd_tune_load(str(p))
    finally:
        Q.qd_tune_set(Q.QD_TUNE_RUN_MIN, 0)   # discards the loaded table


def test_batch_create_rejects_before_device_work():
    """Batch creation validates every register before it allocates: bad precision, a bad radix and a
    register of D >= 2^32 fail with no device call (this runs without a GPU)."""
    cases = (([[2, 3]], 7, Q.QD_EINVAL), ([[2, 257]], Q.QD_C64, Q.QD_EDIM),
             ([[2, 3], [2] * 32], Q.QD_C64, Q.QD_EOVERFLOW))
    for dims_list, prec, code in cases:
        with pytest.raises(Q.QDError) as e:
            Q.qd_batch_create(dims_list, prec, 0)
        assert e.value.code == code, (dims_list, prec)


def test_readout_rejects_null_arguments():
    """The readout calls check their pointers before any device work (this runs without a GPU)."""
    import ctypes
    lib = Q.load()
    v = ctypes.c_double()
    buf = (ctypes.c_double * 4)()
    assert lib.qd_probabilities_norm2(None, buf, 0, ctypes.byref(v)) == Q.QD_EINVAL
    assert lib.qd_norm2(None, ctypes.byref(v)) == Q.QD_EINVAL
    assert lib.qd_probabilities(None, buf, 0) == Q.QD_EINVAL


def test_batch_tuning_keys(tmp_path):
    """Per-key slices per thread of the batched kernel: range checks, and a save / load round trip
    that keeps every key."""
    keep = [Q.qd_batch_tune_key_get(k) for k in range(Q.QD_BATCH_KEYS)]
    try:
        for bad_key, v in ((-1, 2), (Q.QD_BATCH_KEYS, 2)):
            with pytest.raises(Q.QDError):
                Q.qd_batch_tune_key_set(bad_key, v)
        with pytest.raises(Q.QDError):
            Q.qd_batch_tune_key_set(0, 3)
        want = [(0, 1, 2, 4, 8)[k % 5] for k in range(Q.QD_BATCH_KEYS)]
        for k, v in enumerate(want):
            Q.qd_batch_tune_key_set(k, v)
        path = str(tmp_path / "t.json")
        Q.qd_tune_save(path)
        text = open(path).read()
        assert '"batch_key": 11, "gate": "composed", "d_T": "12-32", "min_stride": ">= 16"' in text
        for k in range(Q.QD_BATCH_KEYS):
            Q.qd_batch_tune_key_set(k, 0)
        Q.qd_tune_load(path)
        assert [Q.qd_batch_tune_key_get(k) for k in range(Q.QD_BATCH_KEYS)] == want
    finally:
        for k, v in enumerate(keep):
            Q.qd_batch_tune_key_set(k, v)
