"""O1: FP64 dense state-vector simulation of the feature map (n <= 20).

This is the CPU, double-precision counterpart of the paper's state-vector
method (§3.4.1, Alg. 1): build |psi(x)> = U(x)|0^n> by applying every gate of
the circuit, one after the other, to a 2^n complex vector, then form
K_ij = |<psi(x_j)|psi(x_i)>|^2 (§2, Eq. 3).  Unlike Alg. 1, which assigns the
diagonal, every entry -- the diagonal included -- is computed.

Amplitude index convention: bit k of the basis-state index is qubit k.
"""

from __future__ import annotations

import numpy as np

from .feature_map import H_GATE, feature_map_gates

MAX_QUBITS = 20


def _apply_1q(psi: np.ndarray, n: int, k: int, g: np.ndarray) -> np.ndarray:
    # View the vector as (high bits, bit k, low bits) and act on the middle axis.
    v = psi.reshape(1 << (n - k - 1), 2, 1 << k)
    out = np.einsum("ij,ajb->aib", g, v)
    return out.reshape(-1)


def _apply_phase(psi: np.ndarray, n: int, k: int, lam: float) -> np.ndarray:
    v = psi.reshape(1 << (n - k - 1), 2, 1 << k).copy()
    v[:, 1, :] *= np.exp(1j * lam)
    return v.reshape(-1)


def _apply_cx(psi: np.ndarray, n: int, c: int, t: int) -> np.ndarray:
    # Flip bit t on every basis state whose bit c is 1.
    idx = np.arange(1 << n)
    src = np.where((idx >> c) & 1, idx ^ (1 << t), idx)
    return psi[src]


def sv_state(x, reps: int) -> np.ndarray:
    """|psi(x)> as a complex128 vector of length 2^n (gate list applied literally)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    if n > MAX_QUBITS:
        raise ValueError(f"state vector limited to {MAX_QUBITS} qubits")
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    for name, qubits, param in feature_map_gates(x, reps):
        if name == "H":
            psi = _apply_1q(psi, n, qubits[0], H_GATE)
        elif name == "P":
            psi = _apply_phase(psi, n, qubits[0], param)
        elif name == "CX":
            psi = _apply_cx(psi, n, qubits[0], qubits[1])
        else:  # pragma: no cover - the gate list has no other names
            raise AssertionError(name)
    return psi


def sv_states(X, reps: int) -> np.ndarray:
    """Rows are |psi(x_i)> for the rows x_i of X."""
    X = np.asarray(X, dtype=np.float64)
    return np.stack([sv_state(x, reps) for x in X])


def sv_gram_rect(Xa, Xb, reps: int) -> np.ndarray:
    """K[i, j] = |<psi(b_j)|psi(a_i)>|^2 for rows a_i of Xa and b_j of Xb."""
    Pa = sv_states(Xa, reps)
    Pb = sv_states(Xb, reps)
    amp = Pa @ Pb.conj().T  # amp[i, j] = sum_s conj(psi_b_j(s)) psi_a_i(s)
    return np.abs(amp) ** 2


def sv_gram(X, reps: int) -> np.ndarray:
    """Full symmetric Gram matrix of the rows of X, diagonal computed."""
    return sv_gram_rect(X, X, reps)
