"""O3: closed forms of the kernel that need no circuit simulation.

Each function is a formula derived by hand from the feature map (see
``feature_map``) and the kernel definition K = |<psi(y)|psi(x)>|^2 (§2,
Eq. 3 and Eq. 4).  None of them shares code with the state-vector (O1) or MPS
(O2) simulators, so agreement pins those simulators.

* One qubit, any number of repetitions: |phi_r(x)> = (P(2x) H)^r |0>, a
  product of 2x2 matrices; K = |<phi_r(y)|phi_r(x)>|^2.
* Entanglement-free inputs: if x_k = pi for every even k, every
  theta_k = 2 (pi - x_k)(pi - x_{k+1}) vanishes, each ZZ block is the
  identity and U(x) factorises over qubits, so K = prod_k |f_r(x_k, y_k)|^2
  with f_r the one-qubit overlap.  For r = 1, |f_1|^2 = cos^2(x_k - y_k).
* One repetition with the entangling blocks switched on: U(x)|0^n> =
  D(x) H^n |0^n> with D diagonal, so
      <psi(y)|psi(x)> = 2^-n sum_b exp(i [Phi_x(b) - Phi_y(b)]),
      Phi_x(b) = sum_k 2 x_k b_k + sum_{k<n-1} theta_k (b_k XOR b_{k+1}),
  a one-dimensional sum evaluated either by brute force over the 2^n strings
  (small n) or as a product of 2x2 transfer matrices with a log-scale
  (any n).
"""

from __future__ import annotations

import itertools
import math

import numpy as np


def _theta(x: np.ndarray) -> np.ndarray:
    return 2.0 * (np.pi - x[:-1]) * (np.pi - x[1:])


def single_qubit_state(x: float, reps: int) -> np.ndarray:
    """|phi_r(x)> = (P(2x) H)^r |0> as a 2-vector."""
    h = np.array([[1.0, 1.0], [1.0, -1.0]], dtype=np.complex128) / math.sqrt(2.0)
    p = np.array([[1.0, 0.0], [0.0, np.exp(2j * x)]], dtype=np.complex128)
    v = np.array([1.0, 0.0], dtype=np.complex128)
    for _ in range(reps):
        v = p @ (h @ v)
    return v


def k_one_qubit(x: float, y: float, reps: int) -> float:
    """Kernel of the one-qubit circuit (n = 1: the chain has no CNOT)."""
    f = np.vdot(single_qubit_state(y, reps), single_qubit_state(x, reps))
    return float(abs(f) ** 2)


def k_product(x, y, reps: int) -> float:
    """Kernel of two entanglement-free inputs (x_k = y_k = pi on every even k).

    Raises ValueError when an entangling angle of either input is non-zero.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.shape[0] > 1 and (np.any(_theta(x) != 0.0) or np.any(_theta(y) != 0.0)):
        raise ValueError("inputs are not entanglement-free (some theta_k != 0)")
    log_k = 0.0
    for xk, yk in zip(x, y):
        kk = k_one_qubit(float(xk), float(yk), reps)
        if kk == 0.0:
            return 0.0
        log_k += math.log(kk)
    return math.exp(log_k)


def k_product_log(x, y, reps: int) -> float:
    """Natural log of ``k_product`` (-inf for an exact zero); no underflow."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.shape[0] > 1 and (np.any(_theta(x) != 0.0) or np.any(_theta(y) != 0.0)):
        raise ValueError("inputs are not entanglement-free (some theta_k != 0)")
    total = 0.0
    for xk, yk in zip(x, y):
        kk = k_one_qubit(float(xk), float(yk), reps)
        if kk == 0.0:
            return -math.inf
        total += math.log(kk)
    return total


def k_reps1_bruteforce(x, y) -> float:
    """One-repetition kernel by summing exp(i[Phi_x(b) - Phi_y(b)]) over all 2^n strings."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.shape[0]
    tx = _theta(x)
    ty = _theta(y)
    total = 0.0 + 0.0j
    for bits in itertools.product((0, 1), repeat=n):
        b = np.array(bits, dtype=np.float64)
        phi_x = np.sum(2.0 * x * b) + np.sum(tx * np.logical_xor(bits[:-1], bits[1:]))
        phi_y = np.sum(2.0 * y * b) + np.sum(ty * np.logical_xor(bits[:-1], bits[1:]))
        total += np.exp(1j * (phi_x - phi_y))
    amp = total / (2.0**n)
    return float(abs(amp) ** 2)


def k_reps1_transfer(x, y):
    """One-repetition kernel as a 2x2 transfer-matrix product, any n.

    u_k(b) collects the partial sum over b_0..b_{k-1} with b_k = b:
        u_0(b)     = e^{i d_0 b} / 2,
        u_{k+1}(c) = e^{i d_{k+1} c} / 2 * sum_b e^{i D_k (b XOR c)} u_k(b),
    with d_k = 2 (x_k - y_k) and D_k = theta^x_k - theta^y_k; the amplitude is
    u_{n-1}(0) + u_{n-1}(1).  After each step u is divided by its largest
    modulus and the log of the divisor is accumulated.

    Returns (log_k, k) with k = 0 where exp underflows.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.shape[0]
    d = 2.0 * (x - y)
    dd = _theta(x) - _theta(y) if n > 1 else np.zeros(0)
    u = np.array([0.5, 0.5 * np.exp(1j * d[0])], dtype=np.complex128)
    log_scale = 0.0
    for k in range(n - 1):
        e = np.exp(1j * dd[k])
        t = np.array([[1.0, e], [e, 1.0]], dtype=np.complex128)  # t[b, c]
        u = (u @ t) * np.array([0.5, 0.5 * np.exp(1j * d[k + 1])])
        m = np.max(np.abs(u))
        if m == 0.0:
            return -math.inf, 0.0
        u = u / m
        log_scale += math.log(m)
    amp = abs(u[0] + u[1])
    if amp == 0.0:
        return -math.inf, 0.0
    log_k = 2.0 * (log_scale + math.log(amp))
    return log_k, math.exp(log_k) if log_k > -745.0 else 0.0
