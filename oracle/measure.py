"""Oracle for readout after the gates: computational-basis measurement, per-qudit marginals and the
list of basis states that carry probability. TEST INFRASTRUCTURE ONLY (tests, the smoke check and
the benchmark's CPU-baseline leg).

What the paper fixes:
  * a state's entries alpha_x are probability amplitudes, sum |alpha_x|^2 = 1 (Sec. 2.1.1, Eq. (1));
  * a measurement is in the computational basis and returns, for each qudit, an integer digit
    (Sec. 2.2); measuring every qudit (measure_all, Sec. 3.1) therefore returns a basis index x of
    the register with probability |alpha_x|^2;
  * run() outputs the basis states whose probability is not zero, as ket strings with their
    amplitude or their probability (Sec. 3.6, Sec. 3.8; the example of Sec. 3.9 prints |000> and
    |120> with amplitude 0.7071067811865475).

Readings (the paper is silent on how outcomes are drawn):
  * probabilities are FP64, p_x = re*re + im*im with both products rounded before the sum (no
    fused multiply-add), from the complex64 or complex128 entries promoted to FP64;
  * a shot is drawn by inverting the cumulative distribution of integer weights
    w_x = round-to-nearest-even(p_x * 2^62) (exact integers, so the cumulative sums do not depend
    on the order of summation): with W = sum w_x and a uniform 64-bit random word r supplied by the
    caller, t = floor(r * W / 2^64) (exact integer arithmetic, 0 <= t < W) and the outcome is the
    first x whose cumulative weight exceeds t. Probabilities below 2^-63 get weight 0 and are
    never drawn;
  * the marginal of qudit q is P_q(v) = sum of p_x over the x whose digit q is v;
  * the support at threshold eps is every x with p_x > eps, in ascending order (eps = 0: the
    states of non-zero probability).
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .qudit import digits_of, register_size

__all__ = ["exact_probabilities", "sample_weights", "sample", "marginals", "support", "ket_string"]

WEIGHT_SCALE = 2.0 ** 62


def exact_probabilities(psi: np.ndarray) -> np.ndarray:
    """p_x = |alpha_x|^2 in FP64 (Sec. 2.1.1, Eq. (1)): two rounded products, one rounded sum."""
    re = np.ascontiguousarray(psi.real, dtype=np.float64)
    im = np.ascontiguousarray(psi.imag, dtype=np.float64)
    a = re * re
    b = im * im
    return a + b


def sample_weights(psi: np.ndarray) -> np.ndarray:
    """Integer weights round(p_x * 2^62) (uint64). Raises when their sum would not fit in 64 bits
    (a state whose squared norm is about 4 or more)."""
    p = exact_probabilities(psi)
    if not np.all(np.isfinite(p)) or float(np.sum(p)) >= 3.999:
        raise ValueError("state too far from unit norm to sample")
    w = np.rint(p * WEIGHT_SCALE)
    out = w.astype(np.uint64)
    # exact total from the 32-bit halves (each half-sum fits in 64 bits for D < 2^32)
    hi = int(np.sum(out >> np.uint64(32), dtype=np.uint64))
    lo = int(np.sum(out & np.uint64(0xFFFFFFFF), dtype=np.uint64))
    if (hi << 32) + lo >= 2 ** 64:
        raise ValueError("weights overflow 64 bits")
    return out


def sample(psi: np.ndarray, r) -> np.ndarray:
    """Outcome index of each shot (measure_all, Sec. 3.1 and Sec. 2.2) for the uniform 64-bit
    random words r: inverse of the cumulative integer weights."""
    w = sample_weights(psi)
    cum = np.cumsum(w, dtype=np.uint64)
    total = int(cum[-1])
    if total == 0:
        raise ValueError("state has no weight")
    r = np.asarray(r, dtype=np.uint64)
    t = np.array([(int(x) * total) >> 64 for x in r.tolist()], dtype=np.uint64)
    return np.searchsorted(cum, t, side="right").astype(np.int64)


def marginals(psi: np.ndarray, dims: Sequence[int]) -> list:
    """Per-qudit outcome distributions: entry q is the length-d_q vector P_q(v) (Sec. 2.2)."""
    p = exact_probabilities(psi).reshape(tuple(dims))
    n = len(dims)
    return [p.sum(axis=tuple(a for a in range(n) if a != q)) for q in range(n)]


def support(psi: np.ndarray, eps: float = 0.0) -> np.ndarray:
    """Ascending basis indices whose probability exceeds eps (Sec. 3.6: the non-zero states)."""
    return np.flatnonzero(exact_probabilities(psi) > eps).astype(np.int64)


def ket_string(x: int, dims: Sequence[int]) -> str:
    """Ket label of basis index x, qudit 0 first (Sec. 3.9 prints |120> for q0 = 1, q1 = 2, q2 = 0).
    Digits are written side by side when every radix is at most 10, else separated by commas."""
    if not 0 <= x < register_size(dims):
        raise ValueError("index outside the register")
    digs = digits_of(x, dims)
    sep = "" if max(dims) <= 10 else ","
    return "|" + sep.join(str(d) for d in digs) + ">"
