"""Properties every exact quantum-kernel Gram matrix has.

K_ij = |<psi_j|psi_i>|^2 with normalised states (§2, Eq. 3) implies:
* K_ii = 1 and K_ij = K_ji;
* 0 <= K_ij <= 1 (Cauchy-Schwarz);
* K is positive semi-definite: with G_ij = <psi_j|psi_i>, K = G o conj(G)
  (elementwise product) and both factors are PSD Gram matrices, so the
  Schur product theorem applies.
"""

from __future__ import annotations

import numpy as np


def check_gram(K, tol: float = 1e-12, psd_tol: float | None = None) -> dict:
    """Return a dict of violations (empty when K passes every property)."""
    K = np.asarray(K, dtype=np.float64)
    bad = {}
    if K.ndim != 2 or K.shape[0] != K.shape[1]:
        return {"shape": K.shape}
    diag_err = float(np.max(np.abs(np.diag(K) - 1.0))) if K.size else 0.0
    if diag_err > tol:
        bad["diag"] = diag_err
    sym_err = float(np.max(np.abs(K - K.T))) if K.size else 0.0
    if sym_err > tol:
        bad["symmetry"] = sym_err
    lo = float(K.min()) if K.size else 0.0
    hi = float(K.max()) if K.size else 0.0
    if lo < -tol or hi > 1.0 + tol:
        bad["range"] = (lo, hi)
    if K.size:
        lam = float(np.linalg.eigvalsh(0.5 * (K + K.T)).min())
        limit = tol * K.shape[0] if psd_tol is None else psd_tol
        if lam < -limit:
            bad["psd"] = lam
    return bad


def log_k_errors(log_k_test, log_k_ref) -> np.ndarray:
    """|ln K_test - ln K_ref| elementwise, 0 where both are exact zeros."""
    a = np.asarray(log_k_test, dtype=np.float64)
    b = np.asarray(log_k_ref, dtype=np.float64)
    both_zero = np.isneginf(a) & np.isneginf(b)
    with np.errstate(invalid="ignore"):
        d = np.abs(a - b)
    return np.where(both_zero, 0.0, d)
