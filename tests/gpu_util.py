"""Helpers shared by the GPU tests: run a circuit through libqd's C ABI and compare with the oracle."""
import numpy as np

import paper_2211_07918_amd as Q


def torch_stream():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch.cuda.current_stream().cuda_stream


def run_gpu(circuit, prec=Q.QD_C128, stream=0, gates=None, download=True):
    """Apply the circuit's gates one by one with qd_apply_gate on a fresh library-owned state."""
    s = Q.qd_state_init(circuit.dims, prec, stream)
    try:
        if circuit.init_amps is not None:
            Q.qd_state_upload(s, circuit.init_amps)
        elif circuit.init_basis is not None:
            Q.qd_state_set_basis(s, circuit.init_basis)
        for g in (circuit.gates if gates is None else gates):
            Q.apply_circuit_gate(s, g, circuit.dims)
        return Q.qd_state_download(s) if download else None
    finally:
        Q.qd_state_free(s)


def max_abs(a, b):
    return float(np.max(np.abs(np.asarray(a, np.complex128) - np.asarray(b, np.complex128)))) if np.size(a) else 0.0


def fidelity_loss(ref, psi):
    inner = np.vdot(np.asarray(ref, np.complex128), np.asarray(psi, np.complex128))
    return float(1.0 - abs(inner) ** 2)


def read_amplitudes(s, prec, idx):
    """Amplitudes of a device state at flat indices, copied one by one (for states too large to
    download whole)."""
    import ctypes
    import os
    import torch
    hip = ctypes.CDLL(os.path.join(torch.__path__[0], "lib", "libamdhip64.so"))
    base = Q.qd_state_device_ptr(s)
    esz, dt = (16, np.complex128) if prec == Q.QD_C128 else (8, np.complex64)
    buf = (ctypes.c_char * esz)()
    torch.cuda.synchronize()
    out = np.empty(len(idx), np.complex128)
    for k, i in enumerate(idx):
        rc = hip.hipMemcpy(buf, ctypes.c_void_p(base + esz * int(i)), ctypes.c_size_t(esz), ctypes.c_int(2))
        assert rc == 0, rc
        out[k] = np.frombuffer(bytes(buf), dtype=dt)[0]
    return out
