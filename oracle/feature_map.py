"""The data-encoding circuit U(x) as an explicit gate list (oracle side).

The paper (§3.2, Fig. ``pipeline``) encodes a feature vector with a
parameterised circuit whose qubits are entangled by CNOT gates on a linear
chain, but it does not print the gates, the depth or the number of
repetitions.  The circuit used throughout is the second-order ZZ feature map
of the quantum-kernel work the paper builds on (Havlicek et al., cited in §2)
with that linear chain.  One repetition is

    1. a Hadamard on every qubit;
    2. a phase gate P(2 x_k) on qubit k, for every k;
    3. for k = 0 .. n-2, in this order:
           CNOT(control k, target k+1),
           P(theta_k) on qubit k+1,
           CNOT(control k, target k+1),
       with theta_k = 2 (pi - x_k)(pi - x_{k+1}).

U(x) is ``reps`` repetitions of this block applied to |0...0>.  Feature k
drives qubit k.  P(lam) = diag(1, e^{i lam}); H = [[1, 1], [1, -1]] / sqrt 2.
"""

from __future__ import annotations

import math

import numpy as np

H_GATE = np.array([[1.0, 1.0], [1.0, -1.0]], dtype=np.complex128) / math.sqrt(2.0)

# CNOT on (control, target) in the basis |control target> = 00, 01, 10, 11.
CNOT_GATE = np.array(
    [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128
)


def p_gate(lam: float) -> np.ndarray:
    """Phase gate P(lam) = diag(1, e^{i lam})."""
    return np.array([[1.0, 0.0], [0.0, np.exp(1j * lam)]], dtype=np.complex128)


def zz_angle(xk: float, xk1: float) -> float:
    """Entangling angle theta_k = 2 (pi - x_k)(pi - x_{k+1}) of the ZZ block."""
    return 2.0 * (math.pi - float(xk)) * (math.pi - float(xk1))


def feature_map_gates(x, reps: int):
    """Return U(x) as a list of gates in application order.

    Each entry is ``("H", (k,), None)``, ``("P", (k,), lam)`` or
    ``("CX", (control, target), None)``.  The list is the literal circuit of
    one repetition (module docstring) repeated ``reps`` times.
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    if n < 1:
        raise ValueError("need at least one qubit")
    if reps < 1:
        raise ValueError("need at least one repetition")
    gates = []
    for _ in range(reps):
        for k in range(n):
            gates.append(("H", (k,), None))
        for k in range(n):
            gates.append(("P", (k,), 2.0 * float(x[k])))
        for k in range(n - 1):
            gates.append(("CX", (k, k + 1), None))
            gates.append(("P", (k + 1,), zz_angle(x[k], x[k + 1])))
            gates.append(("CX", (k, k + 1), None))
    return gates
