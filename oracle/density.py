"""Oracle for density matrices and noise channels. TEST INFRASTRUCTURE ONLY (tests, the smoke check
and the benchmark's CPU-baseline leg).

The paper keeps states as vectors and names density matrices (Sec. 3.3) and noise models (Sec. 7)
as the next representations; a channel acting on qudits of dimensions (d_1, .., d_k) has matrices
of the same size as a gate on them (Sec. 3.1). The definitions used here are the standard ones:

  * a pure state psi has density matrix rho = psi psi^dagger;
  * a gate G (the full D x D operator of oracle.qudit.gate_operator, controls included) maps
    rho -> G rho G^dagger;
  * a channel with Kraus operators K_1..K_r on targets T (sum_k K_k^dagger K_k = I) maps
    rho -> sum_k G_k rho G_k^dagger, G_k being K_k on T and the identity elsewhere.

Everything is computed with full D x D matrices and matrix products, so it is independent of any
vectorised form; tiny registers only (D up to a few hundred).

Named channels (readings; the paper defines none):
  * depolarizing(d, p): rho -> (1 - p) rho + p tr_t(rho) (x) I/d on one qudit; Kraus operators
    sqrt(1 - p + p/d^2) I and sqrt(p/d^2) X^a Z^b for (a, b) != (0, 0) (the d^2 Weyl operators);
  * dephasing(d, p): sqrt(1 - p) I and sqrt(p/(d-1)) Z^k, k = 1..d-1;
  * amplitude damping(d, g): K_0 = |0><0| + sqrt(1 - g) sum_{j>=1} |j><j|, K_j = sqrt(g) |j-1><j|,
    j = 1..d-1 (each excited level decays one step with probability g).
X and Z are the generalized shift and phase gates of Sec. 2.1 (oracle.qudit).
"""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

from .qudit import gate_operator, x_gate, z_gate

__all__ = ["from_state", "apply_unitary", "apply_channel", "depolarizing", "dephasing",
           "amplitude_damping", "kraus_complete", "trace", "purity", "fidelity", "probabilities"]


def from_state(psi: np.ndarray) -> np.ndarray:
    psi = np.asarray(psi, dtype=np.complex128)
    return np.outer(psi, psi.conj())


def apply_unitary(rho: np.ndarray, dims: Sequence[int], targets, controls, cvals, U) -> np.ndarray:
    G = gate_operator(dims, targets, controls, cvals, U)
    return G @ rho @ G.conj().T


def apply_channel(rho: np.ndarray, dims: Sequence[int], targets, kraus: Sequence[np.ndarray]) -> np.ndarray:
    out = np.zeros_like(rho)
    for K in kraus:
        G = gate_operator(dims, targets, (), (), K)
        out += G @ rho @ G.conj().T
    return out


def depolarizing(d: int, p: float) -> List[np.ndarray]:
    ks = []
    for a in range(d):
        for b in range(d):
            w = math.sqrt(1.0 - p + p / (d * d)) if (a, b) == (0, 0) else math.sqrt(p / (d * d))
            ks.append(w * (np.linalg.matrix_power(x_gate(d, 1), a) @ np.linalg.matrix_power(z_gate(d), b)))
    return ks


def dephasing(d: int, p: float) -> List[np.ndarray]:
    ks = [math.sqrt(1.0 - p) * np.eye(d, dtype=np.complex128)]
    for k in range(1, d):
        ks.append(math.sqrt(p / (d - 1)) * np.linalg.matrix_power(z_gate(d), k))
    return ks


def amplitude_damping(d: int, g: float) -> List[np.ndarray]:
    k0 = np.zeros((d, d), dtype=np.complex128)
    k0[0, 0] = 1.0
    for j in range(1, d):
        k0[j, j] = math.sqrt(1.0 - g)
    ks = [k0]
    for j in range(1, d):
        k = np.zeros((d, d), dtype=np.complex128)
        k[j - 1, j] = math.sqrt(g)
        ks.append(k)
    return ks


def kraus_complete(kraus: Sequence[np.ndarray]) -> float:
    """max |sum_k K_k^dagger K_k - I| (0 for a trace-preserving channel)."""
    s = sum(K.conj().T @ K for K in kraus)
    return float(np.max(np.abs(s - np.eye(s.shape[0]))))


def trace(rho: np.ndarray) -> complex:
    return complex(np.trace(rho))


def purity(rho: np.ndarray) -> float:
    return float(np.trace(rho @ rho).real)


def fidelity(rho: np.ndarray, psi: np.ndarray) -> float:
    psi = np.asarray(psi, dtype=np.complex128)
    return float((psi.conj() @ rho @ psi).real)


def probabilities(rho: np.ndarray) -> np.ndarray:
    return np.diagonal(rho).real.copy()
