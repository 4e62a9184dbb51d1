#!/usr/bin/env python3
"""Throughput of the qudit gate-application path on one MI355X.

Workload (one step): the hybrid register of 10 qubits + 8 qutrits + 2 ququarts
(D = 2^10 3^8 4^2 = 107,495,424 amplitudes, complex128) is set to |0...0>, the 500 seeded gates
(Haar d x d unitaries on single qudits and controlled shifts on qudit pairs) are applied one by
one through the C ABI, and the FP64 probabilities and the squared norm are read out.

value = amplitude-updates/s over the timed steps (an uncontrolled gate updates D amplitudes, a
controlled one D / prod d_c). Every gate launch is bracketed by HIP events on the stream the
library launches on; the dominant kernel's average duration gives the roofline figure.

Extras in the same JSON line (outside the timed steps): the streaming-copy HBM ceiling, the
fused complex64 paths (FP32 / split-BF16 matrix cores) against the complex128 plain path on
the qudit QFT, the batched path, and the oracle timed on the host cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-extras]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "amplitude-updates/s + HBM GB/s; fused FP32 vs plain FP64 at ≤1e-6 fidelity loss"
HBM_PEAK_GBPS = 8000.0
# MI355X 32-bit integer vector issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one wave64
# VALU instruction per SIMD every 4 cycles; the 157.3 TFLOP/s FP32 figure counts an FMA as two
# flops and dual-issued packed FP32, neither of which integer digit work uses)
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip copy ceiling, fused and batched extras")
    ap.add_argument("--extras-only", action="store_true",
                    help="run only the --extras legs and print {\"extras\": ...} (for profiling one leg alone); "
                         "not the benchmark line")
    ap.add_argument("--no-big", action="store_true", help="skip the 20-qutrit (28 + 56 GB) precision run")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile shapes")
    ap.add_argument("--extras", default="copy,tiny,qft,brick,batch,measure,frontend,sparse,density",
                    help="comma list of extras: copy, tiny, qft, brick, batch, measure, frontend, sparse, density")
    ap.add_argument("--batch-no-serial", action="store_true",
                    help="batched leg: skip the one-by-one comparison (409,600 separate launches), e.g. "
                         "under a counter profiler")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


class TimingEvent:
    """A HIP timing event created with hipEventDisableSystemFence on the HIP runtime torch loaded:
    recording it skips the system-scope cache writeback and invalidation that a default event
    performs (the event only times work; nothing waits on it). Same interface as the part of
    torch.cuda.Event used here."""
    _hip = None
    FLAG = 0x20000000   # hipEventDisableSystemFence

    def __init__(self, torch, stream):
        import ctypes
        if TimingEvent._hip is None:
            TimingEvent._hip = ctypes.CDLL(os.path.join(torch.__path__[0], "lib", "libamdhip64.so"))
        self._c = ctypes
        self.stream = stream
        self.e = ctypes.c_void_p()
        rc = TimingEvent._hip.hipEventCreateWithFlags(ctypes.byref(self.e), ctypes.c_uint(self.FLAG))
        if rc != 0:
            raise RuntimeError(f"hipEventCreateWithFlags failed ({rc})")

    def record(self):
        rc = TimingEvent._hip.hipEventRecord(self.e, self._c.c_void_p(self.stream))
        if rc != 0:
            raise RuntimeError(f"hipEventRecord failed ({rc})")

    def elapsed_time(self, end) -> float:
        ms = self._c.c_float()
        rc = TimingEvent._hip.hipEventElapsedTime(self._c.byref(ms), self.e, end.e)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return ms.value

    def __del__(self):
        if TimingEvent._hip is not None and self.e:
            TimingEvent._hip.hipEventDestroy(self.e)


def gate_plan(circ, Q):
    import numpy as np
    D = circ.D
    out = []
    for g in circ.gates:
        U = Q.gate_unitary(g, circ.dims)
        dc = int(np.prod([circ.dims[c] for c in g.controls])) if g.controls else 1
        out.append({"t": list(g.targets), "c": list(g.controls), "v": list(g.cvals), "U": U,
                    "active": D // dc, "key": None})
    return out


def bench_plain(args, Q, torch, circ):
    import numpy as np
    stream = torch.cuda.current_stream().cuda_stream
    plan = gate_plan(circ, Q)
    D = circ.D
    s = Q.qd_state_init(circ.dims, Q.QD_C128, stream)
    probs = torch.empty(D, dtype=torch.float64, device="cuda")
    zeros = [0] * len(circ.dims)

    def step(ev=None, label=False):
        """One step; ev maps a gate's position to the (start, end) events recorded around it."""
        Q.qd_state_set_basis(s, zeros)
        for i, g in enumerate(plan):
            pair = ev.get(i) if ev is not None else None
            if pair is not None:
                pair[0].record()
            Q.qd_apply_gate(s, g["t"], g["c"], g["v"], g["U"])
            if pair is not None:
                pair[1].record()
            if label:
                g["key"] = Q.qd_last_kernel()   # the kernel instance the library launched
        return Q.qd_probabilities_norm2(s, probs.data_ptr())[1]   # both readouts, one pass; synchronises

    def new_events(positions):
        return {i: (TimingEvent(torch, stream), TimingEvent(torch, stream)) for i in positions}

    step(label=True)          # untimed: the first warm-up step also records each gate's kernel
    for _ in range(args.warmup - 1):
        step()
    # Untimed: one step with events around every gate, for the per-kernel breakdown and to find the
    # dominant kernel. Even without its system-scope fence an event record costs GPU time between
    # two kernels (around all 500 gates about 2.4 ms a step, 3.8 ms with the fence), so the timed
    # steps carry events only around the launches of the dominant kernel (about 0.4 ms a step),
    # whose average duration they measure, and only every other timed step does (the first, third,
    # ...), which halves that cost while still sampling hundreds of launches across the timed region.
    full = new_events(range(len(plan)))
    step(full)
    torch.cuda.synchronize()
    per_key = {}
    for i, g in enumerate(plan):
        d = per_key.setdefault(g["key"], {"ms": 0.0, "n": 0, "bytes": 0.0})
        d["ms"] += full[i][0].elapsed_time(full[i][1])
        d["n"] += 1
        d["bytes"] += 2.0 * 16.0 * g["active"]
    dom_key = max(per_key, key=lambda k: per_key[k]["ms"])
    sample = [i for i, g in enumerate(plan) if g["key"] == dom_key]
    timed = list(range(0, args.steps, 2))
    events = [new_events(sample) if k % 2 == 0 else {} for k in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    norms, marks = [], [t0]
    for k in range(args.steps):
        norms.append(step(events[k]))          # the readout synchronises: each step ends on the host clock
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Q.qd_state_free(s)
    step_ms = sorted(1e3 * (b - a) for a, b in zip(marks, marks[1:]))

    dom_ms = [events[k][i][0].elapsed_time(events[k][i][1]) for k in timed for i in sample]
    avg_ms = sum(dom_ms) / len(dom_ms)
    bytes_per_launch = sum(2.0 * 16.0 * plan[i]["active"] for i in sample) / len(sample)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    upd = sum(g["active"] for g in plan)
    total_bytes = sum(2.0 * 16.0 * g["active"] for g in plan)
    gate_ms = sum(v["ms"] for v in per_key.values())
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    kernels = {k: {"launches_per_step": v["n"], "avg_us": 1e3 * v["ms"] / v["n"],
                   "GBps": v["bytes"] / (v["ms"] * 1e-3) / 1e9}
               for k, v in sorted(per_key.items(), key=lambda kv: -kv[1]["ms"])}
    return {
        "ms_per_step": ms_per_step,
        "step_ms": {"median": step_ms[len(step_ms) // 2], "min": step_ms[0], "max": step_ms[-1],
                    "runs": len(step_ms)},
        "value": upd * args.steps / (t1 - t0),
        "gates_per_s": len(plan) * args.steps / (t1 - t0),
        "hbm_GBps_gates": total_bytes / (gate_ms * 1e-3) / 1e9,
        "norm_drift": max(abs(n - 1.0) for n in norms),
        "roofline": {"bound": "hbm", "kernel": dom_key, "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS, "traffic": None,
                     "avg_launch_us": avg_ms * 1e3, "algorithmic_bytes_per_launch": bytes_per_launch,
                     "timed_launches": len(dom_ms),
                     "timing": "HIP events (no system-scope fence) around each launch of the kernel in every other timed step (the first, third, ...); no other gate carries events there"},
        "kernels": kernels,
    }


def code_digest(text: str) -> str:
    """sha256 of C++/HIP source with its comments and whitespace removed: a counter summary stays
    valid across edits that only touch comments or layout."""
    import hashlib
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return hashlib.sha256(re.sub(r"\s+", "", text).encode()).hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` (its qd_last_kernel label) from the committed
    hardware-counter summary, if that summary was taken on the current source of the gate kernels
    (else None), with a note of where the figure comes from."""
    import glob
    src = os.path.join(ROOT, "paper_2211_07918_amd", "csrc", "qd_gates.hip")
    digest = code_digest(open(src).read())
    for path in glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md")):
        fields = {}
        for line in open(path):
            if ": " in line and not line.startswith(("#", "`", "|")):
                k, v = line.split(": ", 1)
                fields[k.strip()] = v.strip()
        if fields.get("source_code_sha256") == digest and fields.get("label", "").replace(" ", "") == kernel.replace(" ", ""):
            return (float(fields["traffic_bytes_per_launch"]),
                    f"rocprofv3 FETCH_SIZE + WRITE_SIZE counters from the committed summary "
                    f"{os.path.relpath(path, ROOT)} (taken on the current gate-kernel source), not measured in this run")
    return None, "no counter summary for the current gate-kernel source"


def bench_copy(Q, torch):
    stream = torch.cuda.current_stream().cuda_stream
    nbytes = 4 << 30
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(2):
        Q.qd_stream_copy(b.data_ptr(), a.data_ptr(), nbytes, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 10
    for _ in range(reps):
        Q.qd_stream_copy(b.data_ptr(), a.data_ptr(), nbytes, stream)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 2 * nbytes, "avg_us": ms * 1e3, "GBps": 2 * nbytes / (ms * 1e-3) / 1e9}


def _ev(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _plain_state(Q, circ, prec, stream):
    s = Q.qd_state_init(circ.dims, prec, stream)
    if circ.init_amps is not None:
        Q.qd_state_upload(s, circ.init_amps)
    return s


def bench_fused(Q, torch, circ, maxb, name, warm=True):
    """Fused complex64 (FP32 and split-BF16 matrix cores) against the complex128 plain path on the
    same circuit: time, throughput, matrix-core utilisation and the precision report."""
    import numpy as np
    stream = torch.cuda.current_stream().cuda_stream
    plans = [(g.targets, g.controls, g.cvals, Q.gate_unitary(g, circ.dims)) for g in circ.gates]
    ref = _plain_state(Q, circ, Q.QD_C128, stream)
    e0, e1 = _ev(torch)
    torch.cuda.synchronize()
    e0.record()
    for t, c, v, U in plans:
        Q.qd_apply_gate(ref, t, c, v, U)
    e1.record()
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1)
    t0 = time.perf_counter()
    f = Q.qd_fuse(circ.dims, Q.GateArray(circ.gates, lambda i: circ.dims), maxb, stream)
    fuse_s = time.perf_counter() - t0
    nb = Q.qd_fused_count(f)
    Bs = [Q.qd_fused_block_info(f, b)["B"] for b in range(nb)]
    useful = float(sum(8.0 * B * circ.D for B in Bs))
    out = {"D": circ.D, "gates": len(circ.gates), "blocks": nb, "max_block_dim": maxb, "fuse_s": fuse_s,
           "plain_c128_ms": plain_ms, "plain_c128_amp_upd_per_s": len(circ.gates) * circ.D / (plain_ms * 1e-3)}
    # FP32 as the path leaves the state; BF16x3 with the path's FP64 renormalisation on the GPU as
    # its last step (inside the timed region), and without it (reported, not gated)
    legs = ((Q.QD_MODE_FP32_MFMA, "fp32_mfma", 157.3),
            (Q.QD_MODE_BF16X3_MFMA | Q.QD_FUSED_RENORMALIZE, "bf16x3_mfma", 2500.0 / 3),
            (Q.QD_MODE_BF16X3_MFMA, "bf16x3_mfma_no_renormalisation", 2500.0 / 3))
    for mode, mname, peak in legs:
        if warm:
            s = _plain_state(Q, circ, Q.QD_C64, stream)
            Q.qd_apply_fused(s, f, mode)        # warm-up pass (states are not reused below)
            Q.qd_state_free(s)
        s = _plain_state(Q, circ, Q.QD_C64, stream)
        torch.cuda.synchronize()
        e0.record()
        Q.qd_apply_fused(s, f, mode)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        cmp = Q.qd_compare_ex(ref, s)
        Q.qd_state_free(s)
        tf = useful / (ms * 1e-3) / 1e12
        gate = abs(cmp["fid_loss"]) <= 1e-6 and cmp["norm_drift"] <= 1e-6
        out[mname] = {"ms": ms, "ms_per_block": ms / nb, "amp_upd_per_s": len(circ.gates) * circ.D / (ms * 1e-3),
                      "useful_TFLOPs": tf, "peak_TFLOPs": peak, "mfma_frac": tf / peak,
                      "hbm_GBps": nb * 16.0 * circ.D / (ms * 1e-3) / 1e9,
                      "speedup_vs_plain_c128": plain_ms / ms, "max_abs": cmp["max_abs"], "fid_loss": cmp["fid_loss"],
                      "abs_fid_loss": abs(cmp["fid_loss"]), "norm_drift": cmp["norm_drift"],
                      "fid_loss_normalized": cmp["fid_loss_normalized"],
                      "renormalised_on_gpu": bool(mode & Q.QD_FUSED_RENORMALIZE),
                      "meets_1e-6_fidelity_and_drift": gate}
        log(f"{name} {mname}: {ms:.1f} ms ({nb} blocks), {tf:.1f} TFLOP/s, x{plain_ms / ms:.2f} vs plain c128, "
            f"|fid_loss| {abs(cmp['fid_loss']):.2e}, norm drift {cmp['norm_drift']:.2e} "
            f"({'meets' if gate else 'misses'} the 1e-6 bound; normalised fid_loss {cmp['fid_loss_normalized']:.2e})")
    Q.qd_state_free(ref)
    Q.qd_fused_free(f)
    return out


def bench_measure(Q, torch, circ, shots=1_000_000, reps=3):
    """Readout of the benchmark register after its 500 gates (complex128): shots of a measurement
    of every qudit with the random words already in device memory, per-qudit marginals, and the
    number of states above 1e-12. Each call synchronises; the best of `reps` wall times counts."""
    import numpy as np
    stream = torch.cuda.current_stream().cuda_stream
    s = Q.qd_state_init(circ.dims, Q.QD_C128, stream)
    for g in circ.gates:
        Q.apply_circuit_gate(s, g, circ.dims)
    r = np.random.default_rng(2024).integers(0, 2 ** 64, shots, dtype=np.uint64, endpoint=False)
    rt = torch.from_numpy(r.view(np.int64)).to("cuda")
    out = torch.empty(shots, dtype=torch.int64, device="cuda")

    def best(fn):
        fn()
        t = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            t.append(time.perf_counter() - t0)
        return min(t)

    t_sample = best(lambda: Q.qd_sample_device(s, rt.data_ptr(), shots, out.data_ptr()))
    t_marg = best(lambda: Q.qd_marginals(s))
    count = Q.qd_support(s, 1e-12, max_out=0)[3]
    t_supp = best(lambda: Q.qd_support(s, 1e-12, max_out=0))
    Q.qd_state_free(s)
    state_bytes = 16.0 * circ.D
    res = {"D": circ.D, "shots": shots,
           "sample_ms": t_sample * 1e3, "shots_per_s": shots / t_sample,
           "sample_state_GBps": state_bytes / t_sample / 1e9,
           "marginals_ms": t_marg * 1e3, "marginals_state_GBps": state_bytes / t_marg / 1e9,
           "support_count_ms": t_supp * 1e3, "support_count_state_GBps": state_bytes / t_supp / 1e9,
           "states_above_1e-12": int(count)}
    return res


def bench_frontend(Q, n_q=20, n_g=200_000, seed=7):
    """Host-side front-end on a seeded program of n_g gates (H, X with shifts, Z, CX) over a
    20-qudit hybrid register: QASM parse and Moment packing, best of three."""
    import numpy as np
    rng = np.random.default_rng(seed)
    dims = [int(x) for x in rng.choice([2, 3, 4], size=n_q)]
    lines = [f".qudit {n_q}"] + [f"qudit w{i} ({d})" for i, d in enumerate(dims)] + [".begin"]
    for _ in range(n_g):
        t = int(rng.integers(n_q))
        r = rng.random()
        if r < 0.4:
            lines.append(f"H w{t}")
        elif r < 0.6:
            lines.append(f"X w{t} {int(rng.integers(1, dims[t]))}")
        elif r < 0.7:
            lines.append(f"Z w{t}")
        else:
            c = int(rng.choice([q for q in range(n_q) if q != t]))
            lines.append(f"CX w{c} w{t}")
    lines.append(".end")
    text = "\n".join(lines)

    def best(fn):
        t = []
        for _ in range(3):
            t0 = time.perf_counter()
            fn()
            t.append(time.perf_counter() - t0)
        return min(t)

    t_parse = best(lambda: Q.qd_circuit_free(Q.qd_qasm_parse(text)))
    c = Q.qd_qasm_parse(text)
    t_mom = best(lambda: Q.qd_circuit_moments(c))
    depth = Q.qd_circuit_moments(c)[1]
    Q.qd_circuit_free(c)
    return {"gates": n_g, "bytes": len(text), "parse_ms": t_parse * 1e3, "parse_gates_per_s": n_g / t_parse,
            "moments_ms_incl_binding": t_mom * 1e3, "depth": depth}


def _lib_network(Q, net, dims):
    """A Toffoli network as a library circuit, decomposed by the library's front-end (Sec. 3.4)."""
    c = Q.qd_circuit_create(dims)
    for g in net:
        Q.qd_circuit_add(c, Q.QD_GATE_X, g.targets[0], g.a, g.controls, g.cvals)
    dc = Q.qd_circuit_decompose(c)
    Q.qd_circuit_free(c)
    return dc


def bench_sparse(Q, torch, reps=3, cpu_seconds=10.0, cpu=True):
    """Sparse state on a permutation-heavy workload: a 600-gate Toffoli network, decomposed through
    intermediate qutrits, over the 2^24 superposed inputs of a 32-qubit + 8-qutrit register
    (D = 2^32 3^8, beyond any dense state). A second network on a register that fits the dense
    complex128 path is timed both ways. Algorithmic bytes of a monomial launch: every index read
    (8 B) and every moved index written (8 B); the moved count is the library's update counter."""
    import numpy as np
    import circuits as C
    st = torch.cuda.current_stream().cuda_stream
    tn = C.toffoli_network(32, 8, 16, 600, C.seeded_rng(1005))
    sp = Q.qd_sparse_init(tn.dims, 1 << 24, st)
    e0, e1 = _ev(torch)
    torch.cuda.synchronize()
    e0.record()
    for g in tn.inputs:
        Q.apply_circuit_gate_sparse(sp, g, tn.dims)
    e1.record()
    torch.cuda.synchronize()
    t_inputs = e0.elapsed_time(e1)
    n = Q.qd_sparse_count(sp)
    dc = _lib_network(Q, tn.network, tn.dims)
    ng = Q.qd_circuit_size(dc)[1]
    gates = Q.qd_circuit_gates(dc)
    Q.qd_circuit_apply_sparse(sp, dc)                  # warm-up (the network is a permutation)
    u0 = Q.qd_sparse_updates(sp)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        Q.qd_circuit_apply_sparse(sp, dc)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    upd = (Q.qd_sparse_updates(sp) - u0) / reps
    assert Q.qd_sparse_count(sp) == n and abs(Q.qd_sparse_norm2(sp) - 1.0) < 1e-12
    Q.qd_sparse_free(sp)
    Q.qd_circuit_free(dc)
    # the network runs as fused launches (digits of each entry held on chip, the list read and
    # written once per launch): integer work, not HBM traffic, bounds it. Algorithmic operations:
    # 2 per control checked (read the digit, compare) for every entry and gate, 5 per shift applied
    # (read, add, compare, select, write) for every matching entry.
    ctl = sum(len(g[3]) for g in gates)
    alg_ops = 2.0 * n * ctl + 5.0 * upd
    ops_peak = VALU_LANE_OPS
    big = {"workload": "Toffoli network, 600 gates (decomposed: %d) on 32 qubits + 8 qutrits, 2^24 entries" % ng,
           "D": 2 ** 32 * 3 ** 8, "entries": n, "gates": ng, "inputs_ms": t_inputs, "network_ms": ms,
           "gates_per_s": ng / (ms * 1e-3), "gate_entry_steps_per_s": n * ng / (ms * 1e-3),
           "amp_upd_per_s": upd / (ms * 1e-3), "updates_per_network": upd,
           "list_bytes_per_network": 16.0 * n,
           "roofline": {"bound": "alu", "kernel": "k_mono_run<true, 2>", "achieved": alg_ops / (ms * 1e-3) / 1e12,
                        "peak": ops_peak / 1e12, "unit": "Tops/s (32-bit integer lane operations)",
                        "frac": alg_ops / (ms * 1e-3) / ops_peak, "ops_per_network": alg_ops}}
    # a register the dense path holds: 20 qubits + 4 qutrits (D = 2^20 3^4), 2^16 entries
    tn2 = C.toffoli_network(20, 4, 12, 300, C.seeded_rng(1006))
    dc2 = _lib_network(Q, tn2.network, tn2.dims)
    ng2 = Q.qd_circuit_size(dc2)[1]
    sp = Q.qd_sparse_init(tn2.dims, 1 << 16, st)
    s = Q.qd_state_init(tn2.dims, Q.QD_C128, st)
    for g in tn2.inputs:
        Q.apply_circuit_gate_sparse(sp, g, tn2.dims)
        Q.apply_circuit_gate(s, g, tn2.dims)
    Q.qd_circuit_apply_sparse(sp, dc2)
    Q.qd_circuit_apply(s, dc2)
    torch.cuda.synchronize()
    e0.record()
    Q.qd_circuit_apply_sparse(sp, dc2)
    e1.record()
    torch.cuda.synchronize()
    ms_sp = e0.elapsed_time(e1)
    e0.record()
    Q.qd_circuit_apply(s, dc2)
    e1.record()
    torch.cuda.synchronize()
    ms_dense = e0.elapsed_time(e1)
    chk = Q.qd_state_init(tn2.dims, Q.QD_C128, st)
    Q.qd_sparse_to_dense(sp, chk)
    diff = float(np.max(np.abs(Q.qd_state_download(chk) - Q.qd_state_download(s))))
    n2 = Q.qd_sparse_count(sp)
    for h in (chk, s):
        Q.qd_state_free(h)
    Q.qd_sparse_free(sp)
    Q.qd_circuit_free(dc2)
    small = {"workload": "Toffoli network, 300 gates (decomposed: %d) on 20 qubits + 4 qutrits, 2^16 entries" % ng2,
             "D": 2 ** 20 * 3 ** 4, "entries": n2, "sparse_ms": ms_sp, "dense_c128_ms": ms_dense,
             "speedup_vs_dense": ms_dense / ms_sp, "max_abs_vs_dense": diff}
    out = {"big": big, "vs_dense": small}
    if cpu:
        out["cpu_oracle"] = bench_sparse_cpu(tn, cpu_seconds)
    return out


def bench_sparse_cpu(tn, seconds):
    """The sparse oracle (never tuned) on a bounded sample of the big network's workload: 2^16 of
    its input basis states walked through the decomposed network until `seconds` are spent."""
    import numpy as np
    import oracle as O
    from oracle import frontend as F
    from oracle import sparse as S
    dims = tn.dims
    gates = F.decompose_circuit(dims, [("X", g.targets[0], g.a, tuple(g.controls), tuple(g.cvals)) for g in tn.network])
    st = O.strides(dims)
    rng = np.random.default_rng(3)
    bits = rng.integers(0, 2, size=(1 << 16, 24))
    wires = list(range(16)) + list(range(32, 40))
    idx = np.unique((bits * np.array([st[q] for q in wires], dtype=np.int64)).sum(axis=1))
    amp = np.full(idx.size, 2.0 ** -12 + 0j)
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _, t, a, ctl, cv in gates:
            idx, amp = S.apply_gate(dims, idx, amp, (t,), ctl, cv, O.x_gate(dims[t], a))
            done += 1
            if time.perf_counter() - t0 >= seconds:
                break
    dt = time.perf_counter() - t0
    return {"value": done * idx.size / dt, "unit": "entries/s (entries processed per gate)", "cores": 1,
            "kind": "oracle", "sample": f"{idx.size} entries of the same register through {done} decomposed gates, "
                                        f"NumPy, 1 thread, {dt:.1f} s"}


def _noisy_ops(C, dims, ngates, seed, p=1e-3):
    """A noisy circuit as data: each gate of the random-circuit sampler (one target, at most one
    control) followed by a depolarizing channel of strength p on its target."""
    circ = C.random_circuit(dims, ngates, C.seeded_rng(seed), max_targets=1, max_controls=1)
    ops = []
    for g in circ.gates:
        ops.append(("gate", g))
        ops.append(("chan", g.targets[0], p))
    return circ, ops


def bench_density(Q, torch, reps=3, cpu_seconds=10.0, cpu=True):
    """Density matrix of 7 qubits + 4 qutrits (D = 10,368, so D^2 = 1.07e8 elements, 1.72 GB in
    complex128): 60 gates, each followed by a depolarizing channel on its target. A pass reads and
    writes its active elements (algorithmic bytes 2 x 16 per element)."""
    import numpy as np
    import circuits as C
    st = torch.cuda.current_stream().cuda_stream
    dims = (2,) * 7 + (3,) * 4
    D = int(np.prod(dims))
    circ, ops = _noisy_ops(C, dims, 60, 1008)
    kraus = {d: Q.qd_channel_kraus(Q.QD_CHANNEL_DEPOLARIZING, d, 1e-3) for d in set(dims)}
    lib_ops = [o if o[0] == "gate" else ("chan", (o[1],), kraus[dims[o[1]]]) for o in ops]
    # passes, as qd_density_apply_ops forms them: a run of consecutive operations whose targets and
    # controls together span qudits of dimension <= 4 is one composed pass over all D^2 elements;
    # any other channel is one pass; any other gate is one pass when its embedding on targets and
    # controls has d_G <= 4 (d_G <= 3 for a controlled U that is not diagonal), else two, each
    # touching the D^2 / d_c elements whose control digits match
    def support(o):
        if o[0] == "gate":
            return set(o[1].targets) | set(o[1].controls)
        return {o[1]}

    def span(qs):
        return int(np.prod([dims[q] for q in qs]))

    passes, active, i = 0, 0, 0
    while i < len(ops):
        S = support(ops[i])
        j = i + 1
        if span(S) <= 4:
            while j < len(ops) and span(S | support(ops[j])) <= 4:
                S |= support(ops[j])
                j += 1
        if j - i > 1 or ops[i][0] == "chan":
            passes += 1
            active += D * D
        else:
            g = ops[i][1]
            dc = int(np.prod([dims[c] for c in g.controls])) if g.controls else 1
            dG = int(np.prod([dims[q] for q in g.targets])) * dc
            diag = Q.qd_gate_class(Q.gate_unitary(g, dims)) == Q.QD_CLASS_DIAGONAL
            fused = dG <= (3 if g.controls and not diag else 4)
            passes += 1 if fused else 2
            active += D * D if fused else 2 * (D * D // dc)
        i = j
    rho = Q.qd_density_init(dims, Q.QD_C128, st)

    def run():
        Q.qd_density_apply_ops(rho, lib_ops)

    run()                                              # warm-up
    e0, e1 = _ev(torch)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    tr = Q.qd_density_trace(rho)
    pur = Q.qd_density_purity(rho)
    Q.qd_state_free(rho)
    alg = 2.0 * 16.0 * active
    out = {"workload": "density matrix, 7 qubits + 4 qutrits (D = 10,368), 60 gates + 60 depolarizing channels",
           "elements": D * D, "operations": len(ops), "passes": passes, "circuit_ms": ms, "ms_per_pass": ms / passes,
           "element_updates_per_s": len(ops) * D * D / (ms * 1e-3),
           "element_updates_unit": "one operation over all D^2 elements",
           "trace_re": tr.real, "purity": pur,
           "roofline": {"bound": "hbm", "achieved": alg / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                        "frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS}}
    if cpu:
        out["cpu_oracle"] = bench_density_cpu(C, cpu_seconds)
    return out


def bench_density_cpu(C, seconds):
    """The density oracle (never tuned; full operators and matrix products) on a bounded sample of the
    same workload: the same noisy-circuit recipe on 3 qubits + 2 qutrits (D = 72)."""
    import numpy as np
    import oracle as O
    from oracle import density as Dm
    from threadpoolctl import threadpool_limits
    dims = (2,) * 3 + (3,) * 2
    D = int(np.prod(dims))
    circ, ops = _noisy_ops(C, dims, 60, 1008)
    rho = Dm.from_state(O.basis_state(dims))
    done = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            for o in ops:
                if o[0] == "gate":
                    g = o[1]
                    rho = Dm.apply_unitary(rho, dims, g.targets, g.controls, g.cvals, O.gate_unitary(g, dims))
                else:
                    rho = Dm.apply_channel(rho, dims, (o[1],), Dm.depolarizing(dims[o[1]], 1e-3))
                done += 1
                if time.perf_counter() - t0 >= seconds:
                    break
        dt = time.perf_counter() - t0
    return {"value": done * D * D / dt, "unit": "element updates/s (one operation over all D^2 elements)",
            "cores": 1, "kind": "oracle",
            "sample": f"{done} operations of the same recipe on 3 qubits + 2 qutrits (D = {D}), NumPy, 1 thread, {dt:.1f} s"}


_BATCH_SLICES = set(range(2, 10)) | {12, 16, 18, 24, 27, 32}


def batch_schedule(circs, W):
    """Launches and algorithmic bytes (complex64, read + write of every amplitude a pass touches) of
    qd_batch_apply_layers at fusion width W, by the library's block rule: a circuit's next gates
    join a block while it has at most W of them and their qudits number at most 4 with a slice
    size in {2..9, 12, 16, 18, 24, 27, 32}; a one-gate block touches D / d_c amplitudes, a composed
    one all D."""
    import numpy as np
    launches, nbytes = 0, 0
    for c in circs:
        blocks, cur, q = 0, [], set()
        for g in c.gates:
            u = q | set(g.targets) | set(g.controls)
            if cur and len(cur) < W and len(u) <= 4 and int(np.prod([c.dims[x] for x in u])) in _BATCH_SLICES:
                cur.append(g)
                q = u
                continue
            if cur:
                blocks += 1
                nbytes += _block_bytes(c, cur)
            cur, q = [g], set(g.targets) | set(g.controls)
        if cur:
            blocks += 1
            nbytes += _block_bytes(c, cur)
        launches = max(launches, blocks)
    return launches, nbytes


def _block_bytes(c, gates):
    import numpy as np
    if len(gates) > 1 or not gates[0].controls:
        return 16 * c.D
    return 16 * c.D // int(np.prod([c.dims[x] for x in gates[0].controls]))


def bench_batch(Q, torch, ncirc=4096, serial=True, cpu_seconds=10.0):
    """4096 seeded circuits over uneven registers, 100 layers, complex64, recorded into a hipGraph:
    one persistent launch per layer (fusion width 1) and each circuit's gates composed into
    blocks of up to the autotuned fusion width, against the same gates applied one by one
    (plain path)."""
    import numpy as np
    import circuits as C
    stream = torch.cuda.current_stream().cuda_stream
    circs = C.config4(ncirc)
    L = len(circs[0].gates)
    gas = [Q.GateArray([c.gates[l] for c in circs], lambda i: circs[i].dims) for l in range(L)]
    flat = Q.GateArray([c.gates[l] for l in range(L) for c in circs], lambda j: circs[j % ncirc].dims)
    upd = 0
    for c in circs:
        for g in c.gates:
            upd += c.D // (int(np.prod([c.dims[x] for x in g.controls])) if g.controls else 1)
    b = Q.qd_batch_create([c.dims for c in circs], Q.QD_C64, stream)
    Q.qd_batch_autotune(b, gas[0])
    block, spt = Q.qd_tune_get(Q.QD_TUNE_BATCH_BLOCK), Q.qd_tune_get(Q.QD_TUNE_BATCH_SPT)
    grid = Q.qd_tune_get(Q.QD_TUNE_BATCH_GRID)
    Q.qd_batch_autotune_layers(b, flat, L)
    width = Q.qd_tune_get(Q.QD_TUNE_BATCH_FUSE)
    spt_cls = (Q.qd_tune_get(Q.QD_TUNE_BATCH_SPT_MID), Q.qd_tune_get(Q.QD_TUNE_BATCH_SPT_WIDE))
    e0, e1 = _ev(torch)
    reps = 3

    def graph_ms(w):
        Q.qd_batch_compose_ms(b)               # drop the timings of earlier recordings
        Q.qd_batch_capture(b, True)
        Q.qd_batch_apply_layers(b, flat, L, w)  # the compositions run here, once, in FP64 on the GPU
        Q.qd_batch_capture(b, False)
        comp = Q.qd_batch_compose_ms(b)
        Q.qd_batch_replay(b)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            Q.qd_batch_replay(b)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, comp

    ms1, _ = graph_ms(1)
    ms, compose_ms = graph_ms(width) if width != 1 else (ms1, 0.0)
    Q.qd_batch_free(b)
    import tempfile
    tpath = os.path.join(tempfile.gettempdir(), "qd_tune_batch.json")
    Q.qd_tune_save(tpath)
    keys = [json.loads(line.rstrip(",\n")) for line in open(tpath) if '"batch_key"' in line]
    one_s = None
    if serial:
        # one by one: every gate of every circuit through qd_apply_gate on its own state
        states = [Q.qd_state_init(c.dims, Q.QD_C64, stream) for c in circs]
        mats = [[(g.targets, g.controls, g.cvals, Q.gate_unitary(g, c.dims)) for g in c.gates] for c in circs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s, m in zip(states, mats):
            for t, cc, v, U in m:
                Q.qd_apply_gate(s, t, cc, v, U)
        torch.cuda.synchronize()
        one_s = time.perf_counter() - t0
        for s in states:
            Q.qd_state_free(s)
    launches, nbytes = batch_schedule(circs, width)
    cpu = oracle_rate(circs[:64], cpu_seconds, "a seeded 64-circuit subset of the same 4096") if cpu_seconds else None
    return {"cpu_oracle": cpu, "circuits": ncirc, "layers": L, "sum_D": int(sum(c.D for c in circs)), "graph_ms": ms,
            "compose_ms_gpu_fp64": compose_ms, "tuned_keys": [k for k in keys if k["spt"]],
            "fusion_width": width, "graph_ms_width1": ms1, "launches": launches,
            "algorithmic_bytes": nbytes, "hbm_GBps": nbytes / (ms * 1e-3) / 1e9,
            "amp_upd_per_s": upd / (ms * 1e-3), "gates_per_s": ncirc * L / (ms * 1e-3),
            "hbm_GBps_width1": 16.0 * upd / (ms1 * 1e-3) / 1e9, "one_by_one_s": one_s,
            "speedup_vs_one_by_one": one_s / (ms * 1e-3) if one_s else None, "tuned_block": block, "tuned_spt": spt,
            "tuned_grid": "one workgroup per tile" if grid >= 64 else f"{grid} workgroups per CU",
            "tuned_spt_d5_9": spt_cls[0] or "rule", "tuned_spt_d12_32": spt_cls[1] or "rule"}


def bench_cfg0(Q, torch, reps=50):
    """6 qutrits (D = 729), 40 gates: launch-bound, so the figure is the latency per gate. Each
    repetition sets |0..0> and applies the 40 gates through qd_apply_gate, bracketed by HIP events;
    the median over the repetitions is reported, with the host-side wall time per call."""
    import numpy as np
    import circuits as C
    stream = torch.cuda.current_stream().cuda_stream
    c = C.config0()
    mats = [(g.targets, g.controls, g.cvals, Q.gate_unitary(g, c.dims)) for g in c.gates]
    s = Q.qd_state_init(c.dims, Q.QD_C128, stream)
    zeros = [0] * len(c.dims)

    def run():
        Q.qd_state_set_basis(s, zeros)
        for t, cc, v, U in mats:
            Q.qd_apply_gate(s, t, cc, v, U)

    for _ in range(5):
        run()
    e = [_ev(torch) for _ in range(reps)]
    walls = []
    for a, b in e:
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        a.record()
        run()
        b.record()
        walls.append(time.perf_counter() - w0)
    torch.cuda.synchronize()
    Q.qd_state_free(s)
    gpu = sorted(a.elapsed_time(b) for a, b in e)
    walls.sort()
    n = len(mats)
    return {"workload": "6 qutrits (D = 729), 40 gates, complex128", "gates": n,
            "us_per_gate_median": 1e3 * gpu[len(gpu) // 2] / n, "us_per_gate_min": 1e3 * gpu[0] / n,
            "host_us_per_call_median": 1e6 * walls[len(walls) // 2] / n, "repetitions": reps,
            "cpu_oracle": bench_cfg0_cpu(c)}


def bench_cfg0_cpu(c, reps=20):
    """Both oracle forms on the same 40 gates, one BLAS thread: the per-gate contraction (O1) and
    the paper's own execution, full D x D operators multiplied and applied (O2)."""
    import numpy as np
    import oracle as O
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for _ in range(reps):
            O.run_circuit(c)
        t1 = time.perf_counter()
        O.run_circuit_operator(c)
        t2 = time.perf_counter()
    o1 = (t1 - t0) / reps
    return {"value": len(c.gates) * c.D / o1, "unit": "amplitude-updates/s", "cores": 1, "kind": "oracle",
            "us_per_gate_contraction": 1e6 * o1 / len(c.gates),
            "ms_per_circuit_operator_products": 1e3 * (t2 - t1),
            "sample": f"the whole workload: {reps} runs of the 40 gates by per-gate contraction, one run through "
                      f"full 729 x 729 operators, NumPy, 1 thread"}


def oracle_rate(circs, seconds, what):
    """The oracle's per-gate contraction (never tuned) over the gates of `circs` in order, one BLAS
    thread, until `seconds` of work are done: amplitude-updates/s (a controlled gate updates
    D / prod d_c amplitudes)."""
    import numpy as np
    import oracle as O
    from threadpoolctl import threadpool_limits
    upd, ngates, ncirc = 0, 0, 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for c in circs:
            psi = O.initial_state(c)
            for g in c.gates:
                psi = O.apply_gate(psi, c.dims, g.targets, g.controls, g.cvals, O.gate_unitary(g, c.dims))
                dc = int(np.prod([c.dims[x] for x in g.controls])) if g.controls else 1
                upd += c.D // dc
                ngates += 1
                if time.perf_counter() - t0 >= seconds:
                    break
            ncirc += 1
            if time.perf_counter() - t0 >= seconds:
                break
        dt = time.perf_counter() - t0
    return {"value": upd / dt, "unit": "amplitude-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{what}: {ngates} gates over {ncirc} circuit(s), NumPy complex128 contraction, 1 thread, "
                      f"{dt:.1f} s"}


# The paper's own simulation times (context, not a target): end-to-end runs of whole circuits
# (operator construction, then execution), on the hardware and backends it names. The qudit
# dimensions of its benchmark circuits are not given, so none converts to amplitude-updates/s.
PAPER_CONTEXT = {
    "hardware": "Intel Core i5-6300U at 2.40 GHz with 8 GB RAM (stated for the Table 3 runs); the GPU of its "
                "cuda / sparse-cuda backends is not named; precision not stated (printed amplitudes are float64)",
    "times_ms_loading_then_execution": {
        "Sec. 3.9 worked example, dims (2,3,3), 2 gates, sparse backend": [0.192, 1.085],
        "Table 1 toffoli_2_tof (3 qudits, 3 gates), numpy backend": [0.289, 1.219],
        "Table 1 alu-bdd_288_tof (7 qudits, 18 gates), numpy backend": [0.755, 93.461],
        "Table 2 dc1_220_tof (11 qudits, 435 gates), sparse-cuda backend": [13.96, 2329661.45],
        "Table 2 0410184_169_tof (14 qudits, 60 gates), sparse-cuda backend": [6.58, 337.46],
        "Table 3 BV_n14 (14 qudits, 16 gates), cuda backend": [2.25, 75112.75],
        "Table 3 SAT_n11 (11 qudits, 139 gates), sparse-cuda backend": [8.62, 12229.81],
    },
    "largest run without a time": "20 qutrits, depth 80 (Sec. 4, on the i5-6300U)",
}


def host_info():
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover - Linux has it
        affinity = os.cpu_count()
    return {"cpu_model": model, "cpu_count": os.cpu_count(), "affinity_cpus": affinity}


def bench_cpu(circ, seconds, threads=1):
    """The oracle (never tuned) on the full register, gate by gate from |0...0>, with `threads`
    BLAS threads, until `seconds` of work are done."""
    import numpy as np
    import oracle as O
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=threads):
        dims = circ.dims
        psi = O.basis_state(dims)
        upd = 0
        n = 0
        t0 = time.perf_counter()
        for g in circ.gates:
            psi = O.apply_gate(psi, dims, g.targets, g.controls, g.cvals, O.gate_unitary(g, dims))
            dc = int(np.prod([dims[c] for c in g.controls])) if g.controls else 1
            upd += circ.D // dc
            n += 1
            if time.perf_counter() - t0 >= seconds:
                break
        dt = time.perf_counter() - t0
    return {"value": upd / dt, "unit": "amplitude-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} of {len(circ.gates)} gates of the same workload at full size "
                      f"(D={circ.D}), NumPy complex128 contraction, {threads} BLAS thread(s), {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(a multi-GPU run would shard the register, which this library does not do)", file=sys.stderr)
        sys.exit(2)
    import torch

    import circuits as C
    import paper_2211_07918_amd as Q

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    Q.load()
    circ = C.config1()
    tuning = None
    if not args.no_tune:
        import tempfile
        scratch = Q.qd_state_init(circ.dims, Q.QD_C128, torch.cuda.current_stream().cuda_stream)
        path = os.path.join(tempfile.gettempdir(), "qd_tune_bench.json")
        Q.qd_autotune(scratch, path)
        Q.qd_state_free(scratch)
        tuning = open(path).read().replace("\n", "")
        log(f"autotuned: {tuning}")
    if not args.extras_only:
        log(f"plain complex128: D={circ.D} gates={len(circ.gates)} steps={args.steps} warmup={args.warmup}")
        plain = bench_plain(args, Q, torch, circ)
        traffic, source = measured_traffic(plain["roofline"]["kernel"])
        plain["roofline"]["traffic"] = traffic
        plain["roofline"]["traffic_source"] = source
        log(f"plain: {plain['ms_per_step']:.2f} ms/step, {plain['value']:.3e} amp-upd/s, "
            f"dominant {plain['roofline']['kernel']} {plain['roofline']['achieved']:.0f} GB/s")
    extras = {}
    which = set() if args.no_extras else set(args.extras.split(","))
    if "copy" in which:
        extras["copy_ceiling"] = bench_copy(Q, torch)
        log(f"copy ceiling: {extras['copy_ceiling']['GBps']:.0f} GB/s")
    cpu_s = 0.0 if args.no_cpu else min(args.cpu_seconds, 10.0)
    if "tiny" in which:
        t0 = bench_cfg0(Q, torch)
        extras["tiny_6_qutrits"] = t0
        log(f"tiny: {t0['us_per_gate_median']:.2f} us per gate (median of {t0['repetitions']}), "
            f"oracle {t0['cpu_oracle']['us_per_gate_contraction']:.0f} us per gate")
    if "qft" in which:
        q = bench_fused(Q, torch, C.config2(14), 64, "qft14")
        if cpu_s:
            q["cpu_oracle"] = oracle_rate([C.config2(10)], cpu_s, "the same QFT on 10 ququarts (D = 1,048,576)")
        extras["fused_qft_14_ququarts"] = q
    if "brick" in which and not args.no_big:
        b = bench_fused(Q, torch, C.config3(20, 30), 81, "brick20", warm=False)
        if cpu_s:
            b["cpu_oracle"] = oracle_rate([C.config3(12, 30)], cpu_s,
                                          "the same 30-layer brickwork on 12 qutrits (D = 531,441)")
        extras["fused_brickwork_20_qutrits"] = b
    if "batch" in which:
        extras["batched_4096_circuits"] = bench_batch(Q, torch, serial=not args.batch_no_serial, cpu_seconds=cpu_s)
        bb = extras["batched_4096_circuits"]
        log(f"batched: {bb['graph_ms']:.1f} ms per 100 layers at fusion width {bb['fusion_width']} "
            f"(compositions {bb['compose_ms_gpu_fp64']:.2f} ms on the GPU in FP64, at recording) "
            f"({bb['graph_ms_width1']:.1f} ms at width 1), {bb['amp_upd_per_s']:.3e} amp-upd/s, "
            f"{bb['hbm_GBps']:.0f} GB/s over {bb['launches']} launches"
            + (f", x{bb['speedup_vs_one_by_one']:.1f} vs one by one" if bb['speedup_vs_one_by_one'] else ""))
    if "frontend" in which:
        fe = bench_frontend(Q)
        extras["frontend_qasm"] = fe
        log(f"front-end: {fe['gates']} QASM gates parsed in {fe['parse_ms']:.1f} ms, depth {fe['depth']}")
    if "measure" in which:
        mm = bench_measure(Q, torch, circ)
        extras["measurement_hybrid20q"] = mm
        log(f"measurement: {mm['shots']} shots in {mm['sample_ms']:.2f} ms ({mm['shots_per_s']:.3e} shots/s), "
            f"marginals {mm['marginals_ms']:.2f} ms, support count {mm['support_count_ms']:.2f} ms")
    if "sparse" in which:
        sp = bench_sparse(Q, torch, cpu=not args.no_cpu, cpu_seconds=min(args.cpu_seconds, 10.0))
        extras["sparse_toffoli_network"] = sp
        b = sp["big"]
        log(f"sparse: {b['entries']} entries x {b['gates']} gates in {b['network_ms']:.2f} ms "
            f"({b['gate_entry_steps_per_s']:.3e} gate-entry steps/s, {b['roofline']['achieved']:.2f} Tops/s alg. = "
            f"{100 * b['roofline']['frac']:.0f}% of the integer issue rate), "
            f"x{sp['vs_dense']['speedup_vs_dense']:.0f} vs dense c128 on the 2^16-entry network")
    if "density" in which:
        dn = bench_density(Q, torch, cpu=not args.no_cpu, cpu_seconds=min(args.cpu_seconds, 10.0))
        extras["density_noisy_circuit"] = dn
        log(f"density: {dn['operations']} operations as {dn['passes']} passes over {dn['elements']} elements in "
            f"{dn['circuit_ms']:.1f} ms ({dn['ms_per_pass']:.3f} ms/pass, {dn['roofline']['achieved']:.0f} GB/s = "
            f"{100 * dn['roofline']['frac']:.0f}% of HBM peak, {dn['element_updates_per_s']:.3e} element updates/s), "
            f"trace {dn['trace_re']:.12f}")
    if tuning:
        extras["tuning"] = tuning
    if args.extras_only:
        print(json.dumps({"extras": extras}), flush=True)
        return
    out = {
        "metric": METRIC,
        "value": plain["value"],
        "unit": "amplitude-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": plain["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded circuits; no dataset)",
        "config": {"workload": "hybrid register 10 qubits + 8 qutrits + 2 ququarts, 500 seeded gates "
                               "(Haar d x d / controlled shifts), complex128 plain path + FP64 readout",
                   "D": circ.D, "gates": len(circ.gates), "precision": "complex128"},
        "gates_per_s": plain["gates_per_s"],
        "hbm_GBps": plain["hbm_GBps_gates"],
        "norm_drift": plain["norm_drift"],
        "roofline": plain["roofline"],
        "step_ms": plain["step_ms"],
        "kernels": plain["kernels"],
        "paper_context": PAPER_CONTEXT,
    }
    if not args.no_cpu:
        host = host_info()
        out["cpu_baseline"] = bench_cpu(circ, args.cpu_seconds, 1)
        out["cpu_baseline"]["host"] = host
        log(f"cpu oracle: {out['cpu_baseline']['value']:.3e} amp-upd/s on 1 thread ({host['cpu_model']})")
        # the same oracle with a BLAS thread per CPU this process may use (context, not the baseline)
        ncpu = max(1, min(host["affinity_cpus"] or 1, 64))
        if ncpu > 1:
            allc = bench_cpu(circ, args.cpu_seconds, ncpu)
            extras["cpu_oracle_all_cores"] = allc
            log(f"cpu oracle: {allc['value']:.3e} amp-upd/s on {ncpu} threads")
    if extras:
        out["extras"] = extras
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
