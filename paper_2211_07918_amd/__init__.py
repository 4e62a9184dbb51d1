"""Python binding of libqd (include/qd.h): argument marshalling only.

Every function here has the name of the C entry point it calls and does no arithmetic of its own:
it converts NumPy arrays / Python sequences to C arrays, calls libqd, and raises QDError when the
status is not QD_OK. Device memory and streams come from the caller (for instance PyTorch:
``torch.cuda.current_stream().cuda_stream`` and ``tensor.data_ptr()``) as plain integers.

The shared library is built in-tree by ``python -m paper_2211_07918_amd.build``; importing this
package never builds it, and every call fails loudly if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "QDError", "lib_path", "load",
    "QD_OK", "QD_EINVAL", "QD_EDIM", "QD_ENOTUNITARY", "QD_ENOMEM", "QD_EOVERFLOW", "QD_EDEVICE",
    "QD_C128", "QD_C64", "QD_MODE_FP64_PLAIN", "QD_MODE_FP32_MFMA", "QD_MODE_BF16X3_MFMA", "QD_FUSED_RENORMALIZE",
    "QD_FLAG_SKIP_UNITARY_CHECK", "QD_GATE_X", "QD_GATE_Z", "QD_GATE_F", "QD_GATE_I",
    "QD_CLASS_DENSE", "QD_CLASS_MONOMIAL", "QD_CLASS_DIAGONAL",
    "QD_CHANNEL_DEPOLARIZING", "QD_CHANNEL_DEPHASING", "QD_CHANNEL_AMPLITUDE_DAMPING",
    "qd_density_init", "qd_density_from_state", "qd_density_apply_gate", "qd_density_apply_channel",
    "qd_channel_kraus", "qd_density_trace", "qd_density_probabilities", "qd_density_purity",
    "qd_density_fidelity", "qd_density_size", "qd_density_dims", "apply_circuit_gate_density",
    "qd_density_apply_ops", "QD_OP_GATE", "QD_OP_CHANNEL",
    "QD_TUNE_DIRECT_BLOCK", "QD_TUNE_DIRECT_SPT", "QD_TUNE_TILE_BLOCK", "QD_TUNE_TILE_ELEMS",
    "QD_TUNE_DIAG_BLOCK", "QD_TUNE_BATCH_BLOCK", "QD_TUNE_BATCH_SPT", "QD_TUNE_FUSED_COLS", "QD_TUNE_RUN_MIN",
    "QD_TUNE_BATCH_GRID", "QD_TUNE_BATCH_FUSE", "QD_TUNE_BATCH_SPT_MID", "QD_TUNE_BATCH_SPT_WIDE",
    "qd_batch_apply_layers", "qd_batch_autotune_layers", "qd_batch_compose_ms", "QD_BATCH_KEYS",
    "qd_batch_tune_key_set", "qd_batch_tune_key_get",
    "QD_ROUTE_DIRECT", "QD_ROUTE_TILED", "QD_ROUTE_DIAG", "QD_ROUTE_GENERIC", "QD_ROUTE_GEMM", "qd_gate_route",
    "qd_version", "qd_last_error", "qd_last_kernel", "qd_state_gate_launches", "qd_register_strides", "qd_gate_matrix", "qd_validate_gate",
    "qd_gate_class", "qd_state_init", "qd_state_wrap", "qd_state_set_basis", "qd_state_upload",
    "qd_state_download", "qd_state_size", "qd_state_dims", "qd_state_precision", "qd_state_device_ptr",
    "qd_state_sync", "qd_state_free", "qd_apply_gate", "qd_apply_gate_ex", "qd_fuse_plan",
    "qd_fuse", "qd_fused_count", "qd_fused_block_info", "qd_fused_block_gates", "qd_fused_download_block",
    "qd_apply_fused", "qd_fused_free", "qd_probabilities", "qd_norm2", "qd_probabilities_norm2", "qd_norm2_noalloc", "qd_compare", "qd_compare_ex",
    "qd_normalize", "qd_sample", "qd_sample_device", "qd_marginals", "qd_support", "qd_ket_string", "kets",
    "qd_circuit_create", "qd_circuit_add", "qd_qasm_parse", "qd_circuit_size", "qd_circuit_dims", "qd_circuit_name",
    "qd_circuit_gate", "qd_circuit_gates", "qd_circuit_moments", "qd_circuit_decompose", "qd_circuit_apply",
    "qd_circuit_free", "qd_circuit_apply_sparse",
    "qd_sparse_init", "qd_sparse_upload", "qd_sparse_set_basis", "qd_sparse_apply_gate", "qd_sparse_apply_gates",
    "qd_sparse_count",
    "qd_sparse_download", "qd_sparse_device_lists", "qd_sparse_norm2", "qd_sparse_probabilities",
    "qd_sparse_to_dense", "qd_sparse_updates", "qd_sparse_sync", "qd_sparse_free", "apply_circuit_gate_sparse",
    "qd_batch_create", "qd_batch_size", "qd_batch_offset", "qd_batch_reset",
    "qd_batch_apply_layer", "qd_batch_capture", "qd_batch_replay", "qd_batch_download",
    "qd_batch_free", "qd_tune_set", "qd_tune_get", "qd_autotune", "qd_tune_load", "qd_tune_save", "qd_batch_autotune",
    "qd_stream_copy",
    "gate_unitary", "apply_circuit_gate", "GateArray",
]

QD_OK, QD_EINVAL, QD_EDIM, QD_ENOTUNITARY, QD_ENOMEM, QD_EOVERFLOW, QD_EDEVICE = 0, -1, -2, -3, -4, -5, -6
QD_C128, QD_C64 = 0, 1
QD_MODE_FP64_PLAIN, QD_MODE_FP32_MFMA, QD_MODE_BF16X3_MFMA = 0, 1, 2
QD_FUSED_RENORMALIZE = 0x100
QD_FLAG_SKIP_UNITARY_CHECK = 1
QD_GATE_X, QD_GATE_Z, QD_GATE_F, QD_GATE_I = 0, 1, 2, 3
QD_CLASS_DENSE, QD_CLASS_MONOMIAL, QD_CLASS_DIAGONAL = 0, 1, 2
QD_CHANNEL_DEPOLARIZING, QD_CHANNEL_DEPHASING, QD_CHANNEL_AMPLITUDE_DAMPING = 0, 1, 2
QD_OP_GATE, QD_OP_CHANNEL = 0, 1
QD_BATCH_KEYS = 12
QD_ROUTE_DIRECT, QD_ROUTE_TILED, QD_ROUTE_DIAG, QD_ROUTE_GENERIC, QD_ROUTE_GEMM = 0, 1, 2, 3, 4
(QD_TUNE_DIRECT_BLOCK, QD_TUNE_DIRECT_SPT, QD_TUNE_TILE_BLOCK, QD_TUNE_TILE_ELEMS, QD_TUNE_DIAG_BLOCK,
 QD_TUNE_BATCH_BLOCK, QD_TUNE_BATCH_SPT, QD_TUNE_FUSED_COLS, QD_TUNE_RUN_MIN, QD_TUNE_BATCH_GRID,
 QD_TUNE_BATCH_FUSE, QD_TUNE_BATCH_SPT_MID, QD_TUNE_BATCH_SPT_WIDE) = range(13)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class QDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libqd error {code}: {msg}")
        self.code = code


def lib_path() -> str:
    return os.path.join(_HERE, "libqd.so")


class _DensityOp(C.Structure):
    _fields_ = [("kind", C.c_int32), ("k", C.c_int32), ("targets", C.POINTER(C.c_int32)), ("m", C.c_int32),
                ("controls", C.POINTER(C.c_int32)), ("control_values", C.POINTER(C.c_int32)),
                ("nk", C.c_int32), ("mats", C.POINTER(C.c_double))]


class _Gate(C.Structure):
    _fields_ = [("k", C.c_int32), ("targets", C.POINTER(C.c_int32)), ("m", C.c_int32),
                ("controls", C.POINTER(C.c_int32)), ("control_values", C.POINTER(C.c_int32)),
                ("U", C.POINTER(C.c_double))]


_P = C.c_void_p
_I32P = C.POINTER(C.c_int32)
_I64P = C.POINTER(C.c_int64)
_DP = C.POINTER(C.c_double)

_SIGS = {
    "qd_version": (C.c_char_p, []),
    "qd_last_error": (C.c_char_p, []),
    "qd_last_kernel": (C.c_char_p, []),
    "qd_register_strides": (C.c_int, [_I32P, C.c_int32, _I64P, _I64P]),
    "qd_gate_matrix": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, _DP]),
    "qd_validate_gate": (C.c_int, [_I32P, C.c_int32, _I32P, C.c_int32, _I32P, _I32P, C.c_int32, _DP, C.c_uint32]),
    "qd_gate_class": (C.c_int, [_DP, C.c_int32]),
    "qd_gate_route": (C.c_int, [_I32P, C.c_int32, C.c_int32, _I32P, C.c_int32, _I32P, _I32P, C.c_int32, _DP, _I32P]),
    "qd_state_init": (C.c_int, [_I32P, C.c_int32, C.c_int32, _P, C.POINTER(_P)]),
    "qd_state_wrap": (C.c_int, [_I32P, C.c_int32, C.c_int32, _P, C.c_int64, _P, C.POINTER(_P)]),
    "qd_state_set_basis": (C.c_int, [_P, _I32P]),
    "qd_state_upload": (C.c_int, [_P, _P, C.c_int64]),
    "qd_state_download": (C.c_int, [_P, _P, C.c_int64]),
    "qd_state_size": (C.c_int, [_P, _I64P]),
    "qd_state_dims": (C.c_int, [_P, _I32P, _I32P]),
    "qd_state_precision": (C.c_int, [_P, _I32P]),
    "qd_state_device_ptr": (C.c_int, [_P, C.POINTER(_P)]),
    "qd_state_gate_launches": (C.c_int, [_P, _I64P]),
    "qd_state_sync": (C.c_int, [_P]),
    "qd_state_free": (None, [_P]),
    "qd_apply_gate": (C.c_int, [_P, _I32P, C.c_int32, _I32P, _I32P, C.c_int32, _DP]),
    "qd_apply_gate_ex": (C.c_int, [_P, _I32P, C.c_int32, _I32P, _I32P, C.c_int32, _DP, C.c_uint32]),
    "qd_fuse_plan": (C.c_int, [_I32P, C.c_int32, C.POINTER(_Gate), C.c_int32, C.c_int32, _I32P, _I32P]),
    "qd_fuse": (C.c_int, [_I32P, C.c_int32, C.POINTER(_Gate), C.c_int32, C.c_int32, _P, C.POINTER(_P)]),
    "qd_fused_count": (C.c_int, [_P, _I32P]),
    "qd_fused_block_info": (C.c_int, [_P, C.c_int32, _I32P, _I32P, _I32P, _I32P, _I32P]),
    "qd_fused_download_block": (C.c_int, [_P, C.c_int32, _DP]),
    "qd_fused_block_gates": (C.c_int, [_P, C.c_int32, _I32P]),
    "qd_apply_fused": (C.c_int, [_P, _P, C.c_int32]),
    "qd_fused_free": (None, [_P]),
    "qd_probabilities": (C.c_int, [_P, _DP, C.c_int32]),
    "qd_norm2": (C.c_int, [_P, _DP]),
    "qd_probabilities_norm2": (C.c_int, [_P, _DP, C.c_int32, _DP]),
    "qd_norm2_noalloc": (C.c_int, [_P, _P]),
    "qd_compare": (C.c_int, [_P, _P, _DP, _DP, _DP]),
    "qd_compare_ex": (C.c_int, [_P, _P, _DP]),
    "qd_normalize": (C.c_int, [_P, _DP]),
    "qd_sample": (C.c_int, [_P, _P, C.c_int64, _P, C.c_int32]),
    "qd_marginals": (C.c_int, [_P, _DP]),
    "qd_support": (C.c_int, [_P, C.c_double, C.c_int64, _P, _P, _P, _I64P]),
    "qd_ket_string": (C.c_int, [_I32P, C.c_int32, C.c_int64, C.c_char_p, C.c_int32]),
    "qd_circuit_create": (C.c_int, [_I32P, C.c_int32, C.POINTER(_P)]),
    "qd_circuit_add": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, _I32P, _I32P, C.c_int32]),
    "qd_qasm_parse": (C.c_int, [C.c_char_p, C.POINTER(_P)]),
    "qd_circuit_size": (C.c_int, [_P, _I32P, _I64P]),
    "qd_circuit_dims": (C.c_int, [_P, _I32P]),
    "qd_circuit_name": (C.c_int, [_P, C.c_int32, C.c_char_p, C.c_int32]),
    "qd_circuit_gate": (C.c_int, [_P, C.c_int64, _I32P, _I32P, _I32P, _I32P, _I32P, _I32P]),
    "qd_circuit_moments": (C.c_int, [_P, _I32P, _I32P]),
    "qd_circuit_decompose": (C.c_int, [_P, C.POINTER(_P)]),
    "qd_circuit_apply": (C.c_int, [_P, _P]),
    "qd_circuit_free": (None, [_P]),
    "qd_circuit_apply_sparse": (C.c_int, [_P, _P]),
    "qd_sparse_init": (C.c_int, [_I32P, C.c_int32, C.c_int64, _P, C.POINTER(_P)]),
    "qd_sparse_upload": (C.c_int, [_P, _P, _P, C.c_int64]),
    "qd_sparse_set_basis": (C.c_int, [_P, _I32P]),
    "qd_sparse_apply_gate": (C.c_int, [_P, _I32P, C.c_int32, _I32P, _I32P, C.c_int32, _DP, C.c_uint32]),
    "qd_sparse_count": (C.c_int, [_P, _I64P]),
    "qd_sparse_apply_gates": (C.c_int, [_P, C.POINTER(_Gate), C.c_int32, C.c_uint32]),
    "qd_sparse_download": (C.c_int, [_P, _P, _P, C.c_int64, _I64P]),
    "qd_sparse_device_lists": (C.c_int, [_P, C.POINTER(_P), C.POINTER(_P), _I64P]),
    "qd_sparse_norm2": (C.c_int, [_P, _DP]),
    "qd_sparse_probabilities": (C.c_int, [_P, _P, C.c_int32, C.c_int64]),
    "qd_sparse_to_dense": (C.c_int, [_P, _P]),
    "qd_sparse_sync": (C.c_int, [_P]),
    "qd_sparse_updates": (C.c_int, [_P, _I64P]),
    "qd_density_init": (C.c_int, [_I32P, C.c_int32, C.c_int32, _P, C.POINTER(_P)]),
    "qd_density_from_state": (C.c_int, [_P, _P]),
    "qd_density_apply_gate": (C.c_int, [_P, _I32P, C.c_int32, _I32P, _I32P, C.c_int32, _DP, C.c_uint32]),
    "qd_density_apply_channel": (C.c_int, [_P, _I32P, C.c_int32, _DP, C.c_int32, C.c_uint32]),
    "qd_channel_kraus": (C.c_int, [C.c_int32, C.c_int32, C.c_double, _DP, C.c_int32, _I32P]),
    "qd_density_trace": (C.c_int, [_P, _DP, _DP]),
    "qd_density_probabilities": (C.c_int, [_P, _DP, C.c_int32]),
    "qd_density_purity": (C.c_int, [_P, _DP]),
    "qd_density_fidelity": (C.c_int, [_P, _P, _DP]),
    "qd_density_size": (C.c_int, [_P, _I32P]),
    "qd_density_apply_ops": (C.c_int, [_P, C.POINTER(_DensityOp), C.c_int32, C.c_uint32]),
    "qd_sparse_free": (None, [_P]),
    "qd_batch_create": (C.c_int, [C.c_int32, _I32P, _I32P, C.c_int32, _P, C.POINTER(_P)]),
    "qd_batch_size": (C.c_int, [_P, _I64P]),
    "qd_batch_offset": (C.c_int, [_P, C.c_int32, _I64P]),
    "qd_batch_reset": (C.c_int, [_P]),
    "qd_batch_apply_layer": (C.c_int, [_P, C.POINTER(_Gate)]),
    "qd_batch_capture": (C.c_int, [_P, C.c_int32]),
    "qd_batch_replay": (C.c_int, [_P]),
    "qd_batch_download": (C.c_int, [_P, _P, C.c_int64]),
    "qd_batch_free": (None, [_P]),
    "qd_tune_set": (C.c_int, [C.c_int32, C.c_int32]),
    "qd_tune_get": (C.c_int, [C.c_int32, _I32P]),
    "qd_autotune": (C.c_int, [_P, C.c_char_p]),
    "qd_tune_load": (C.c_int, [C.c_char_p]),
    "qd_tune_save": (C.c_int, [C.c_char_p]),
    "qd_batch_autotune": (C.c_int, [_P, C.POINTER(_Gate)]),
    "qd_batch_apply_layers": (C.c_int, [_P, C.POINTER(_Gate), C.c_int32, C.c_int32]),
    "qd_batch_compose_ms": (C.c_int, [_P, _DP]),
    "qd_batch_tune_key_set": (C.c_int, [C.c_int32, C.c_int32]),
    "qd_batch_tune_key_get": (C.c_int, [C.c_int32, _I32P]),
    "qd_batch_autotune_layers": (C.c_int, [_P, C.POINTER(_Gate), C.c_int32]),
    "qd_stream_copy": (C.c_int, [_P, _P, C.c_int64, _P]),
}


def load():
    """Load libqd.so (built in-tree). Raises if it is missing: there is no fallback path."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise QDError(QD_EDEVICE, f"{path} is not built; run `python -m paper_2211_07918_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def _check(rc: int):
    if rc != QD_OK:
        raise QDError(rc, load().qd_last_error().decode())


def _i32(seq) -> C.Array:
    seq = [int(v) for v in seq]
    return (C.c_int32 * max(1, len(seq)))(*seq)


def _cplx(U) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(U, dtype=np.complex128))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_DP)


# ------------------------------------------------------------------------------ library, register
def qd_version() -> str:
    return load().qd_version().decode()


def qd_last_error() -> str:
    return load().qd_last_error().decode()


def qd_last_kernel() -> str:
    """Kernel instance of this thread's last gate launch (a profiling label)."""
    return load().qd_last_kernel().decode()


def qd_register_strides(dims: Sequence[int]):
    D = C.c_int64()
    st = (C.c_int64 * len(dims))()
    _check(load().qd_register_strides(_i32(dims), len(dims), C.byref(D), st))
    return int(D.value), [int(x) for x in st]


def qd_gate_matrix(kind: int, d: int, a: int = 0) -> np.ndarray:
    U = np.zeros((d, d), dtype=np.complex128)
    _check(load().qd_gate_matrix(kind, d, a, _dptr(U)))
    return U


def qd_validate_gate(dims, targets, controls, control_values, U, flags: int = 0) -> int:
    """Returns the status code (no exception): QD_OK or the error qd_apply_gate would return."""
    Uc = _cplx(U)
    try:
        _check_shape(dims, targets, Uc)
    except QDError as e:
        return e.code
    return int(load().qd_validate_gate(_i32(dims), len(dims), _i32(targets), len(targets), _i32(controls),
                                       _i32(control_values), len(controls), _dptr(Uc), flags))


def qd_gate_route(dims, prec, targets, controls, control_values, U) -> int:
    Uc = _cplx(U)
    _check_shape(dims, targets, Uc)
    r = C.c_int32()
    _check(load().qd_gate_route(_i32(dims), len(dims), prec, _i32(targets), len(targets), _i32(controls),
                                _i32(control_values), len(controls), _dptr(Uc), C.byref(r)))
    return int(r.value)


def qd_gate_class(U) -> int:
    Uc = _cplx(U)
    return int(load().qd_gate_class(_dptr(Uc), Uc.shape[0]))


# ------------------------------------------------------------------------------ states
def qd_state_init(dims: Sequence[int], prec: int = QD_C128, stream: int = 0) -> int:
    h = _P()
    _check(load().qd_state_init(_i32(dims), len(dims), prec, _P(stream or None), C.byref(h)))
    return h.value


def qd_state_wrap(dims: Sequence[int], prec: int, dev_ptr: int, nbytes: int, stream: int = 0) -> int:
    h = _P()
    _check(load().qd_state_wrap(_i32(dims), len(dims), prec, _P(dev_ptr), nbytes, _P(stream or None), C.byref(h)))
    return h.value


def qd_state_set_basis(s: int, values: Sequence[int]):
    _check(load().qd_state_set_basis(_P(s), _i32(values)))


def _state_dtype(s: int):
    p = C.c_int32()
    _check(load().qd_state_precision(_P(s), C.byref(p)))
    return np.complex128 if p.value == QD_C128 else np.complex64


def qd_state_size(s: int) -> int:
    D = C.c_int64()
    _check(load().qd_state_size(_P(s), C.byref(D)))
    return int(D.value)


def qd_state_dims(s: int):
    n = C.c_int32()
    dims = (C.c_int32 * 64)()
    _check(load().qd_state_dims(_P(s), dims, C.byref(n)))
    return [int(x) for x in dims[:n.value]]


def _check_shape(dims, targets, Uc):
    if not len(targets) or any(not 0 <= int(t) < len(dims) for t in targets):
        return  # the library reports the bad target list
    dT = int(np.prod([dims[int(t)] for t in targets]))
    if Uc.shape != (dT, dT):
        raise QDError(QD_EDIM, f"U has shape {Uc.shape}, the targets need ({dT}, {dT})")


def qd_state_precision(s: int) -> int:
    p = C.c_int32()
    _check(load().qd_state_precision(_P(s), C.byref(p)))
    return int(p.value)


def qd_state_upload(s: int, amps):
    a = np.ascontiguousarray(np.asarray(amps, dtype=_state_dtype(s)))
    _check(load().qd_state_upload(_P(s), a.ctypes.data_as(_P), a.size))


def qd_state_download(s: int) -> np.ndarray:
    out = np.empty(qd_state_size(s), dtype=_state_dtype(s))
    _check(load().qd_state_download(_P(s), out.ctypes.data_as(_P), out.size))
    return out


def qd_state_gate_launches(s: int) -> int:
    v = C.c_int64()
    _check(load().qd_state_gate_launches(_P(s), C.byref(v)))
    return int(v.value)


def qd_state_device_ptr(s: int) -> int:
    p = _P()
    _check(load().qd_state_device_ptr(_P(s), C.byref(p)))
    return p.value or 0


def qd_state_sync(s: int):
    _check(load().qd_state_sync(_P(s)))


def qd_state_free(s: int):
    if s:
        load().qd_state_free(_P(s))


# ------------------------------------------------------------------------------ gates
def qd_apply_gate(s: int, targets, controls, control_values, U):
    Uc = _cplx(U)
    _check_shape(qd_state_dims(s), targets, Uc)
    _check(load().qd_apply_gate(_P(s), _i32(targets), len(targets), _i32(controls), _i32(control_values),
                                len(controls), _dptr(Uc)))


def qd_apply_gate_ex(s: int, targets, controls, control_values, U, flags: int):
    Uc = _cplx(U)
    _check_shape(qd_state_dims(s), targets, Uc)
    _check(load().qd_apply_gate_ex(_P(s), _i32(targets), len(targets), _i32(controls), _i32(control_values),
                                   len(controls), _dptr(Uc), flags))


_KIND = {"X": QD_GATE_X, "Z": QD_GATE_Z, "F": QD_GATE_F}


def gate_unitary(gate, dims) -> np.ndarray:
    """Unitary of a gate record (attributes kind, targets, a, U): named gates are built by
    qd_gate_matrix from the acting wire's dimension, explicit ones are passed through."""
    if gate.kind == "U":
        return _cplx(gate.U)
    return qd_gate_matrix(_KIND[gate.kind], int(dims[gate.targets[0]]), int(gate.a))


def apply_circuit_gate(s: int, gate, dims, flags: int = 0):
    """qd_apply_gate_ex for one gate record."""
    qd_apply_gate_ex(s, gate.targets, gate.controls, gate.cvals, gate_unitary(gate, dims), flags)


class GateArray:
    """A C array of qd_gate built from gate records (keeps the referenced buffers alive)."""

    def __init__(self, gates, dims_of):
        """dims_of(i) gives the register dims of gate i (one register for qd_fuse, one per circuit
        for the batched layer). A gate record of None is an empty slot (k = 0)."""
        self._keep = []
        self.arr = (_Gate * max(1, len(gates)))()
        for i, g in enumerate(gates):
            if g is None:
                self.arr[i].k = 0
                continue
            U = gate_unitary(g, dims_of(i))
            t, c, v = _i32(g.targets), _i32(g.controls), _i32(g.cvals)
            self._keep += [U, t, c, v]
            self.arr[i].k = len(g.targets)
            self.arr[i].targets = C.cast(t, _I32P)
            self.arr[i].m = len(g.controls)
            self.arr[i].controls = C.cast(c, _I32P)
            self.arr[i].control_values = C.cast(v, _I32P)
            self.arr[i].U = _dptr(U)
        self.n = len(gates)


# ------------------------------------------------------------------------------ fusion
def qd_fuse_plan(dims, gates, max_block_dim: int):
    ga = gates if isinstance(gates, GateArray) else GateArray(gates, lambda i: dims)
    blk = (C.c_int32 * max(1, ga.n))()
    nb = C.c_int32()
    _check(load().qd_fuse_plan(_i32(dims), len(dims), ga.arr, ga.n, max_block_dim, blk, C.byref(nb)))
    return [int(b) for b in blk[:ga.n]], int(nb.value)


def qd_fuse(dims, gates, max_block_dim: int, stream: int = 0) -> int:
    ga = gates if isinstance(gates, GateArray) else GateArray(gates, lambda i: dims)
    h = _P()
    _check(load().qd_fuse(_i32(dims), len(dims), ga.arr, ga.n, max_block_dim, _P(stream or None), C.byref(h)))
    return h.value


def qd_fused_count(f: int) -> int:
    n = C.c_int32()
    _check(load().qd_fused_count(_P(f), C.byref(n)))
    return int(n.value)


def qd_fused_block_info(f: int, b: int):
    k, B, first, ng = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    win = (C.c_int32 * 64)()
    _check(load().qd_fused_block_info(_P(f), b, C.byref(k), win, C.byref(B), C.byref(first), C.byref(ng)))
    gs = (C.c_int32 * max(1, ng.value))()
    _check(load().qd_fused_block_gates(_P(f), b, gs))
    return {"window": [int(x) for x in win[:k.value]], "B": int(B.value), "first_gate": int(first.value),
            "ngates": int(ng.value), "gates": [int(x) for x in gs[:ng.value]]}


def qd_fused_block_gates(f: int, b: int):
    return qd_fused_block_info(f, b)["gates"]


def qd_fused_download_block(f: int, b: int) -> np.ndarray:
    B = qd_fused_block_info(f, b)["B"]
    out = np.empty((B, B), dtype=np.complex128)
    _check(load().qd_fused_download_block(_P(f), b, _dptr(out)))
    return out


def qd_apply_fused(s: int, f: int, mode: int):
    _check(load().qd_apply_fused(_P(s), _P(f), mode))


def qd_fused_free(f: int):
    if f:
        load().qd_fused_free(_P(f))


# ------------------------------------------------------------------------------ readout
def qd_probabilities(s: int, out_dev_ptr: Optional[int] = None):
    """FP64 probabilities: into device memory at out_dev_ptr (asynchronous), or returned as a
    NumPy array when out_dev_ptr is None."""
    if out_dev_ptr is not None:
        _check(load().qd_probabilities(_P(s), C.cast(_P(out_dev_ptr), _DP), 1))
        return None
    out = np.empty(qd_state_size(s), dtype=np.float64)
    _check(load().qd_probabilities(_P(s), _dptr(out), 0))
    return out


def qd_norm2(s: int) -> float:
    v = C.c_double()
    _check(load().qd_norm2(_P(s), C.byref(v)))
    return float(v.value)


def qd_probabilities_norm2(s: int, out_dev_ptr: Optional[int] = None):
    """Probabilities and ||psi||^2 from one pass: (None, norm2) with the probabilities written to
    device memory at out_dev_ptr, or (NumPy array, norm2) when out_dev_ptr is None."""
    v = C.c_double()
    if out_dev_ptr is not None:
        _check(load().qd_probabilities_norm2(_P(s), C.cast(_P(out_dev_ptr), _DP), 1, C.byref(v)))
        return None, float(v.value)
    out = np.empty(qd_state_size(s), dtype=np.float64)
    _check(load().qd_probabilities_norm2(_P(s), _dptr(out), 0, C.byref(v)))
    return out, float(v.value)


def qd_norm2_noalloc(s: int, out_dev_ptr: int):
    """qd_norm2 into one FP64 value at a device address the caller owns; asynchronous, and the
    library allocates nothing for it."""
    _check(load().qd_norm2_noalloc(_P(s), _P(out_dev_ptr)))


def qd_compare(ref64: int, s: int):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    _check(load().qd_compare(_P(ref64), _P(s), C.byref(a), C.byref(b), C.byref(c)))
    return float(a.value), float(b.value), float(c.value)


def qd_compare_ex(ref64: int, s: int) -> dict:
    out = (C.c_double * 5)()
    _check(load().qd_compare_ex(_P(ref64), _P(s), out))
    return {"max_abs": out[0], "fid_loss": out[1], "norm_drift": out[2], "norm2": out[3],
            "fid_loss_normalized": out[4]}


def qd_normalize(s: int) -> float:
    v = C.c_double()
    _check(load().qd_normalize(_P(s), C.byref(v)))
    return float(v.value)


# ------------------------------------------------------------------------------ measurement
def qd_sample(s: int, rand) -> np.ndarray:
    """Shot outcomes (basis indices, int64) for the uniform 64-bit random words `rand` (host)."""
    r = np.ascontiguousarray(np.asarray(rand, dtype=np.uint64))
    out = np.empty(r.size, dtype=np.int64)
    _check(load().qd_sample(_P(s), r.ctypes.data_as(_P), r.size, out.ctypes.data_as(_P), 0))
    return out


def qd_sample_device(s: int, rand_dev_ptr: int, shots: int, out_dev_ptr: int) -> None:
    """Shots with the random words and the outcomes in device memory."""
    _check(load().qd_sample(_P(s), _P(rand_dev_ptr), int(shots), _P(out_dev_ptr), 1))


def qd_marginals(s: int) -> list:
    """Per-qudit outcome distributions (FP64): entry q has d_q values."""
    dims = qd_state_dims(s)
    out = np.empty(int(sum(dims)), dtype=np.float64)
    _check(load().qd_marginals(_P(s), _dptr(out)))
    offs = np.cumsum([0] + dims)
    return [out[offs[q]:offs[q + 1]].copy() for q in range(len(dims))]


def qd_support(s: int, eps: float = 0.0, max_out: Optional[int] = None):
    """States with probability > eps, ascending: (indices, amplitudes, probabilities, count).
    At most max_out entries are returned (all when None); count is the full number."""
    cnt = C.c_int64()
    _check(load().qd_support(_P(s), float(eps), 0, None, None, None, C.byref(cnt)))
    n = cnt.value if max_out is None else min(cnt.value, int(max_out))
    cdt = np.complex128 if qd_state_precision(s) == QD_C128 else np.complex64
    idx = np.empty(n, dtype=np.int64)
    amps = np.empty(n, dtype=cdt)
    probs = np.empty(n, dtype=np.float64)
    if n:
        _check(load().qd_support(_P(s), float(eps), n, idx.ctypes.data_as(_P), amps.ctypes.data_as(_P),
                                 probs.ctypes.data_as(_P), C.byref(cnt)))
    return idx, amps, probs, int(cnt.value)


def qd_ket_string(dims, index: int) -> str:
    buf = C.create_string_buffer(8 * len(dims) + 8)
    _check(load().qd_ket_string(_i32(dims), len(dims), int(index), buf, len(buf)))
    return buf.value.decode()


def kets(s: int, eps: float = 0.0, method: str = "probability"):
    """run() output in the paper's print form: one {ket: value} per state with probability > eps,
    value the probability (method "probability") or the amplitude (method "amplitude")."""
    dims = qd_state_dims(s)
    idx, amps, probs, _ = qd_support(s, eps)
    vals = probs if method == "probability" else amps
    return [{qd_ket_string(dims, int(i)): (float(v) if method == "probability" else complex(v))}
            for i, v in zip(idx, vals)]


# ------------------------------------------------------------------------------ circuit front-end
def qd_circuit_create(dims) -> int:
    out = _P()
    _check(load().qd_circuit_create(_i32(dims), len(dims), C.byref(out)))
    return out.value


def qd_circuit_add(c: int, kind: int, target: int, a: int = 0, controls=(), values=()) -> None:
    _check(load().qd_circuit_add(_P(c), int(kind), int(target), int(a), _i32(controls), _i32(values), len(controls)))


def qd_qasm_parse(text: str) -> int:
    out = _P()
    _check(load().qd_qasm_parse(text.encode(), C.byref(out)))
    return out.value


def qd_circuit_size(c: int):
    n, g = C.c_int32(), C.c_int64()
    _check(load().qd_circuit_size(_P(c), C.byref(n), C.byref(g)))
    return int(n.value), int(g.value)


def qd_circuit_dims(c: int) -> list:
    n, _ = qd_circuit_size(c)
    out = (C.c_int32 * n)()
    _check(load().qd_circuit_dims(_P(c), out))
    return [int(x) for x in out]


def qd_circuit_name(c: int, q: int) -> str:
    buf = C.create_string_buffer(256)
    _check(load().qd_circuit_name(_P(c), int(q), buf, len(buf)))
    return buf.value.decode()


def qd_circuit_gate(c: int, i: int):
    """(kind, target, a, controls, control_values) of gate i."""
    kind, t, a, m = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    ctl, val = (C.c_int32 * 64)(), (C.c_int32 * 64)()
    _check(load().qd_circuit_gate(_P(c), int(i), C.byref(kind), C.byref(t), C.byref(a), C.byref(m), ctl, val))
    return int(kind.value), int(t.value), int(a.value), tuple(ctl[:m.value]), tuple(val[:m.value])


def qd_circuit_gates(c: int) -> list:
    return [qd_circuit_gate(c, i) for i in range(qd_circuit_size(c)[1])]


def qd_circuit_moments(c: int):
    """(moment of every gate, depth)."""
    _, g = qd_circuit_size(c)
    out = (C.c_int32 * max(1, g))()
    depth = C.c_int32()
    _check(load().qd_circuit_moments(_P(c), out, C.byref(depth)))
    return [int(x) for x in out[:g]], int(depth.value)


def qd_circuit_decompose(c: int) -> int:
    out = _P()
    _check(load().qd_circuit_decompose(_P(c), C.byref(out)))
    return out.value


def qd_circuit_apply(s: int, c: int) -> None:
    _check(load().qd_circuit_apply(_P(s), _P(c)))


def qd_circuit_free(c: int) -> None:
    load().qd_circuit_free(_P(c))


def qd_circuit_apply_sparse(sp: int, c: int) -> None:
    _check(load().qd_circuit_apply_sparse(_P(sp), _P(c)))


# ------------------------------------------------------------------------------ density matrices
def qd_density_init(dims, prec: int = QD_C128, stream: int = 0) -> int:
    out = _P()
    _check(load().qd_density_init(_i32(dims), len(dims), int(prec), _P(stream), C.byref(out)))
    return out.value


def qd_density_size(rho: int) -> int:
    n = C.c_int32()
    _check(load().qd_density_size(_P(rho), C.byref(n)))
    return int(n.value)


def qd_density_dims(rho: int):
    """The physical register (the first half of the doubled one)."""
    return qd_state_dims(rho)[:qd_density_size(rho)]


def qd_density_from_state(rho: int, psi: int) -> None:
    _check(load().qd_density_from_state(_P(rho), _P(psi)))


def qd_density_apply_gate(rho: int, targets, controls, control_values, U, flags: int = 0) -> None:
    Uc = _cplx(U)
    _check_shape(qd_density_dims(rho), targets, Uc)
    _check(load().qd_density_apply_gate(_P(rho), _i32(targets), len(targets), _i32(controls), _i32(control_values),
                                        len(controls), _dptr(Uc), int(flags)))


def apply_circuit_gate_density(rho: int, gate, dims, flags: int = 0):
    """qd_density_apply_gate for one gate record."""
    qd_density_apply_gate(rho, gate.targets, gate.controls, gate.cvals, gate_unitary(gate, dims), flags)


def qd_density_apply_channel(rho: int, targets, kraus, flags: int = 0) -> None:
    """Kraus operators (a list of d_T x d_T arrays) on the targets."""
    ks = [_cplx(K) for K in kraus]
    for K in ks:
        _check_shape(qd_density_dims(rho), targets, K)
    flat = np.ascontiguousarray(np.concatenate([K.reshape(-1) for K in ks])) if ks else np.zeros(1, np.complex128)
    _check(load().qd_density_apply_channel(_P(rho), _i32(targets), len(targets), _dptr(flat), len(ks), int(flags)))


def qd_density_apply_ops(rho: int, ops, flags: int = 0) -> None:
    """Operations in order: ("gate", gate record) or ("chan", targets, [Kraus matrices])."""
    dims = qd_density_dims(rho)
    arr = (_DensityOp * max(1, len(ops)))()
    keep = []
    for i, o in enumerate(ops):
        if o[0] == "gate":
            g = o[1]
            U = gate_unitary(g, dims)
            _check_shape(dims, g.targets, U)
            t, c, v = _i32(g.targets), _i32(g.controls), _i32(g.cvals)
            keep += [U, t, c, v]
            arr[i].kind, arr[i].k, arr[i].m, arr[i].nk = QD_OP_GATE, len(g.targets), len(g.controls), 1
            arr[i].targets, arr[i].controls, arr[i].control_values = C.cast(t, _I32P), C.cast(c, _I32P), C.cast(v, _I32P)
            arr[i].mats = _dptr(U)
        else:
            _, targets, kraus = o
            ks = [_cplx(K) for K in kraus]
            for K in ks:
                _check_shape(dims, targets, K)
            flat = np.ascontiguousarray(np.concatenate([K.reshape(-1) for K in ks]))
            t = _i32(targets)
            keep += [flat, t]
            arr[i].kind, arr[i].k, arr[i].m, arr[i].nk = QD_OP_CHANNEL, len(targets), 0, len(ks)
            arr[i].targets, arr[i].mats = C.cast(t, _I32P), _dptr(flat)
    _check(load().qd_density_apply_ops(_P(rho), arr, len(ops), int(flags)))


def qd_channel_kraus(kind: int, d: int, p: float) -> list:
    """The library's Kraus operators of a named one-qudit channel."""
    nk = C.c_int32()
    _check(load().qd_channel_kraus(int(kind), int(d), float(p), None, 0, C.byref(nk)))
    out = np.zeros(nk.value * d * d, dtype=np.complex128)
    _check(load().qd_channel_kraus(int(kind), int(d), float(p), _dptr(out), nk.value, C.byref(nk)))
    return [out[i * d * d:(i + 1) * d * d].reshape(d, d).copy() for i in range(nk.value)]


def qd_density_trace(rho: int) -> complex:
    re, im = C.c_double(), C.c_double()
    _check(load().qd_density_trace(_P(rho), C.byref(re), C.byref(im)))
    return complex(re.value, im.value)


def qd_density_probabilities(rho: int) -> np.ndarray:
    D = int(np.prod(qd_density_dims(rho)))
    out = np.empty(D, dtype=np.float64)
    _check(load().qd_density_probabilities(_P(rho), _dptr(out), 0))
    return out


def qd_density_purity(rho: int) -> float:
    v = C.c_double()
    _check(load().qd_density_purity(_P(rho), C.byref(v)))
    return float(v.value)


def qd_density_fidelity(rho: int, psi: int) -> float:
    v = C.c_double()
    _check(load().qd_density_fidelity(_P(rho), _P(psi), C.byref(v)))
    return float(v.value)


# ------------------------------------------------------------------------------ sparse state
_SPARSE_DIMS = {}   # handle -> register, for the argument-shape check before a raw pointer is passed


def qd_sparse_init(dims, capacity: int = 0, stream: int = 0) -> int:
    out = _P()
    _check(load().qd_sparse_init(_i32(dims), len(dims), int(capacity), _P(stream), C.byref(out)))
    _SPARSE_DIMS[out.value] = [int(d) for d in dims]
    return out.value


def qd_sparse_upload(sp: int, idx, amps) -> None:
    i = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    a = np.ascontiguousarray(np.asarray(amps, dtype=np.complex128))
    if i.shape != a.shape:
        raise ValueError("idx and amps must have the same length")
    _check(load().qd_sparse_upload(_P(sp), i.ctypes.data_as(_P), a.ctypes.data_as(_P), i.size))


def qd_sparse_set_basis(sp: int, values) -> None:
    _check(load().qd_sparse_set_basis(_P(sp), _i32(values)))


def qd_sparse_apply_gate(sp: int, targets, controls, control_values, U, flags: int = 0) -> None:
    Uc = _cplx(U)
    _check_shape(_SPARSE_DIMS[sp], targets, Uc)
    _check(load().qd_sparse_apply_gate(_P(sp), _i32(targets), len(targets), _i32(controls), _i32(control_values),
                                       len(controls), _dptr(Uc), int(flags)))


def apply_circuit_gate_sparse(sp: int, gate, dims, flags: int = 0):
    """qd_sparse_apply_gate for one gate record."""
    qd_sparse_apply_gate(sp, gate.targets, gate.controls, gate.cvals, gate_unitary(gate, dims), flags)


def qd_sparse_apply_gates(sp: int, gates, flags: int = 0) -> None:
    """Gate records applied in order (runs of monomial gates in one pass over the list)."""
    dims = _SPARSE_DIMS[sp]
    for g in gates:
        _check_shape(dims, g.targets, gate_unitary(g, dims))
    ga = GateArray(gates, lambda i: dims)
    _check(load().qd_sparse_apply_gates(_P(sp), ga.arr, ga.n, int(flags)))


def qd_sparse_count(sp: int) -> int:
    n = C.c_int64()
    _check(load().qd_sparse_count(_P(sp), C.byref(n)))
    return int(n.value)


def qd_sparse_download(sp: int):
    """The list in list order: (indices int64, amplitudes complex128)."""
    n = qd_sparse_count(sp)
    idx = np.empty(n, dtype=np.int64)
    amps = np.empty(n, dtype=np.complex128)
    cnt = C.c_int64()
    _check(load().qd_sparse_download(_P(sp), idx.ctypes.data_as(_P), amps.ctypes.data_as(_P), n, C.byref(cnt)))
    return idx, amps


def qd_sparse_device_lists(sp: int):
    """(device address of the indices, of the amplitudes, count)."""
    pi, pa, n = _P(), _P(), C.c_int64()
    _check(load().qd_sparse_device_lists(_P(sp), C.byref(pi), C.byref(pa), C.byref(n)))
    return pi.value, pa.value, int(n.value)


def qd_sparse_norm2(sp: int) -> float:
    v = C.c_double()
    _check(load().qd_sparse_norm2(_P(sp), C.byref(v)))
    return float(v.value)


def qd_sparse_probabilities(sp: int) -> np.ndarray:
    n = qd_sparse_count(sp)
    out = np.empty(n, dtype=np.float64)
    _check(load().qd_sparse_probabilities(_P(sp), out.ctypes.data_as(_P), 0, n))
    return out


def qd_sparse_to_dense(sp: int, s: int) -> None:
    _check(load().qd_sparse_to_dense(_P(sp), _P(s)))


def qd_sparse_updates(sp: int) -> int:
    n = C.c_int64()
    _check(load().qd_sparse_updates(_P(sp), C.byref(n)))
    return int(n.value)


def qd_sparse_sync(sp: int) -> None:
    _check(load().qd_sparse_sync(_P(sp)))


def qd_sparse_free(sp: int) -> None:
    _SPARSE_DIMS.pop(sp, None)
    load().qd_sparse_free(_P(sp))


# ------------------------------------------------------------------------------ batch
def qd_batch_create(dims_list, prec: int = QD_C64, stream: int = 0) -> int:
    n_per = [len(d) for d in dims_list]
    flat = [int(x) for d in dims_list for x in d]
    h = _P()
    _check(load().qd_batch_create(len(dims_list), _i32(n_per), _i32(flat), prec, _P(stream or None), C.byref(h)))
    return h.value


def qd_batch_size(b: int) -> int:
    v = C.c_int64()
    _check(load().qd_batch_size(_P(b), C.byref(v)))
    return int(v.value)


def qd_batch_offset(b: int, c: int) -> int:
    v = C.c_int64()
    _check(load().qd_batch_offset(_P(b), c, C.byref(v)))
    return int(v.value)


def qd_batch_reset(b: int):
    _check(load().qd_batch_reset(_P(b)))


def qd_batch_apply_layer(b: int, gates):
    """gates: a GateArray with one slot per circuit."""
    _check(load().qd_batch_apply_layer(_P(b), gates.arr))


def qd_batch_apply_layers(b: int, gates, nlayers: int, width: int = 0):
    """gates: a GateArray of nlayers x ncirc slots (layer-major); width 0 = the tuned fusion width."""
    _check(load().qd_batch_apply_layers(_P(b), gates.arr, int(nlayers), int(width)))


def qd_batch_compose_ms(b: int) -> float:
    """GPU time of the block compositions launched since the previous call (ms)."""
    v = C.c_double()
    _check(load().qd_batch_compose_ms(_P(b), C.byref(v)))
    return float(v.value)


def qd_batch_tune_key_set(key: int, spt: int):
    _check(load().qd_batch_tune_key_set(int(key), int(spt)))


def qd_batch_tune_key_get(key: int) -> int:
    v = C.c_int32()
    _check(load().qd_batch_tune_key_get(int(key), C.byref(v)))
    return int(v.value)


def qd_batch_autotune_layers(b: int, gates, nlayers: int):
    _check(load().qd_batch_autotune_layers(_P(b), gates.arr, int(nlayers)))


def qd_batch_capture(b: int, on: bool):
    _check(load().qd_batch_capture(_P(b), 1 if on else 0))


def qd_batch_replay(b: int):
    _check(load().qd_batch_replay(_P(b)))


def qd_batch_download(b: int, dtype=np.complex64) -> np.ndarray:
    out = np.empty(qd_batch_size(b), dtype=dtype)
    _check(load().qd_batch_download(_P(b), out.ctypes.data_as(_P), out.size))
    return out


def qd_batch_free(b: int):
    if b:
        load().qd_batch_free(_P(b))


# ------------------------------------------------------------------------------ tuning, calibration
def qd_tune_set(param: int, value: int):
    _check(load().qd_tune_set(param, value))


def qd_tune_get(param: int) -> int:
    v = C.c_int32()
    _check(load().qd_tune_get(param, C.byref(v)))
    return int(v.value)


def qd_autotune(scratch_state: int, path: Optional[str] = None):
    _check(load().qd_autotune(_P(scratch_state), path.encode() if path else None))


def qd_tune_load(path: str):
    _check(load().qd_tune_load(path.encode()))


def qd_tune_save(path: str):
    _check(load().qd_tune_save(path.encode()))


def qd_batch_autotune(b: int, gates):
    """gates: a GateArray with one slot per circuit (the layer to time)."""
    _check(load().qd_batch_autotune(_P(b), gates.arr))


def qd_stream_copy(dst: int, src: int, nbytes: int, stream: int = 0):
    _check(load().qd_stream_copy(_P(dst), _P(src), nbytes, _P(stream or None)))
