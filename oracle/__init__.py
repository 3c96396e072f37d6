"""CPU FP64 oracle for the quantum-kernel Gram matrix (test infrastructure only).

This package is the independent checker of the GPU path.  It is plain, slow,
double-precision NumPy code that computes

    K(x_i, x_j) = |<psi(x_j)|psi(x_i)>|^2 ,   |psi(x)> = U(x)|0^n>

(paper §2, Eq. 3 and Eq. 4) in three unrelated ways:

* ``statevector``  (O1) -- the literal gate list applied to a dense 2^n state,
  n <= 20 (the state-vector method of §3.4.1, Alg. 1, in FP64 on the CPU);
* ``mps``          (O2) -- the same gate list applied to a matrix-product
  state gate by gate, with SVD splits that drop only numerical zeros, then the
  pairwise overlap swept site by site with a log-scale (the tensor-network
  method of §3.4.2 / Alg. 3, contracted in a fixed left-to-right order);
* ``closed_forms`` (O3) -- entanglement-free product states, the one-rep
  transfer-matrix sum and the one-qubit case;
* ``mlp`` -- FP64 forward, pair loss, backward and AdamW of the learned
  surrogate that stands in for K at large N.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, calls or links anything here, and nothing
here imports the product package: the two share no code.  Inputs are passed in
as arrays; the seeded generators live in a module of their own.
"""

from .feature_map import feature_map_gates, zz_angle
from .statevector import sv_state, sv_gram, sv_gram_rect
from .mps import mps_state, mps_overlap_log, mps_gram_pairs, mps_states
from .closed_forms import (
    single_qubit_state,
    k_one_qubit,
    k_product,
    k_reps1_transfer,
    k_reps1_bruteforce,
)
from .checks import check_gram, log_k_errors

__all__ = [
    "feature_map_gates",
    "zz_angle",
    "sv_state",
    "sv_gram",
    "sv_gram_rect",
    "mps_state",
    "mps_states",
    "mps_overlap_log",
    "mps_gram_pairs",
    "single_qubit_state",
    "k_one_qubit",
    "k_product",
    "k_reps1_transfer",
    "k_reps1_bruteforce",
    "check_gram",
    "log_k_errors",
]
