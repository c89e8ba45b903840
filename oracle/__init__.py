"""Plain FP64 CPU oracle (test infrastructure only; see oracle.py)."""
from .oracle import (GATES, adjoint_jacobian, apply, apply_matrix, apply_pauli_sum, build, sample,  # noqa: F401
                     expval, gate_generator, gate_matrix, inner, num_threads, zero_state)
