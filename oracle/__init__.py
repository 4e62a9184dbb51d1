"""Reference oracle for the qudit gate-application path. TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct NumPy complex128 simulator written from the paper
(QuDiet, arXiv 2211.07918). Only the test-suite, the smoke check and the benchmark's CPU-baseline
leg may import it; the product library never does, and this package imports nothing from it.

Two independent forms of the same definition are provided:
  * O1 ``apply_gate``: per-gate tensor contraction on ``reshape(psi, dims)``;
  * O2 ``gate_operator`` / ``run_circuit_operator``: full D x D operators built by enumerating basis
    states, multiplied together and applied to the initial state at the end, which is the paper's
    own execution scheme (Sec. 3.6: Kronecker product per Moment, operator products, final
    matrix-vector product).

``oracle.measure`` holds the readout after the gates: shots of a computational-basis measurement,
per-qudit marginals and the list of states with non-zero probability (ket output).
``oracle.sparse`` holds the sparse state (the list of non-zero amplitudes) and its gate updates.
``oracle.density`` holds density matrices, gates on them and Kraus channels (full matrix products).
"""
from .qudit import *  # noqa: F401,F403
from .qudit import __all__  # noqa: F401
