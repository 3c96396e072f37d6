"""O2: FP64 exact matrix-product-state simulation and pairwise overlaps.

The paper turns each kernel circuit into a tensor network and contracts it
(§3.1, §3.4.2, Alg. 2 and Alg. 3).  The oracle does the same job for the
linear-chain feature map without any shortcut taken by the GPU path:

1. ``mps_state`` starts from |0...0> as a bond-dimension-1 MPS and applies
   the literal gate list (``feature_map.feature_map_gates``) one gate at a
   time.  One-qubit gates are contracted into their site tensor.  Each CNOT
   merges its two sites, applies the 4x4 matrix and splits the result again
   with an SVD.  The MPS is kept in mixed-canonical form (orthogonality
   centre at the site the next CNOT touches), so the singular values are the
   Schmidt coefficients of the normalised state and dropping those below
   1e-14 of the largest removes numerical zeros only: the state is exact
   ("untruncated") to ~1e-14.
2. ``mps_overlap_log`` contracts <B|A> left to right, carrying the
   environment E <- sum_s B_s^dagger E A_s, dividing E by its largest modulus
   after every site and adding the logarithm of that divisor to a running
   FP64 log-scale, so 784-site overlaps of order 1e-400 do not underflow.
   The result is log|amp|; K = |amp|^2 = exp(2 log|amp|) (§2, Eq. 3).

Site tensors have shape (D_left, 2, D_right); the physical index is the qubit
value and qubit k is feature k.  Bond dimensions stay <= 2^reps.
"""

from __future__ import annotations

import math
from multiprocessing import get_context

import numpy as np

from .feature_map import CNOT_GATE, H_GATE, feature_map_gates, p_gate

SVD_ZERO_REL = 1e-14


def _one_site(t: np.ndarray, g: np.ndarray) -> np.ndarray:
    return np.einsum("ij,ajb->aib", g, t)


def _move_centre(sites, frm: int, to: int) -> None:
    """Shift the orthogonality centre from site ``frm`` to site ``to`` with QR steps."""
    k = frm
    while k > to:  # sites k..to+1 become right-isometries
        t = sites[k]
        dl, _, dr = t.shape
        q, r = np.linalg.qr(t.reshape(dl, 2 * dr).conj().T)  # t = r^H q^H
        sites[k] = q.conj().T.reshape(-1, 2, dr)
        sites[k - 1] = np.einsum("asb,bc->asc", sites[k - 1], r.conj().T)
        k -= 1
    while k < to:  # sites k..to-1 become left-isometries
        t = sites[k]
        dl, _, dr = t.shape
        q, r = np.linalg.qr(t.reshape(dl * 2, dr))
        sites[k] = q.reshape(dl, 2, -1)
        sites[k + 1] = np.einsum("ab,bsc->asc", r, sites[k + 1])
        k += 1


def _two_site(sites, k: int, g4: np.ndarray) -> None:
    """Apply a 4x4 gate to (k, k+1) and split back with an SVD (centre -> k+1)."""
    a, b = sites[k], sites[k + 1]
    dl, dr = a.shape[0], b.shape[2]
    theta = np.einsum("asb,btc->astc", a, b)
    theta = np.einsum("ijkl,aklc->aijc", g4.reshape(2, 2, 2, 2), theta)
    u, s, vh = np.linalg.svd(theta.reshape(dl * 2, 2 * dr), full_matrices=False)
    keep = s > SVD_ZERO_REL * s[0]
    sites[k] = u[:, keep].reshape(dl, 2, -1)
    sites[k + 1] = (s[keep, None] * vh[keep]).reshape(-1, 2, dr)


def mps_state(x, reps: int):
    """Exact MPS of |psi(x)> = U(x)|0^n>, built gate by gate (list of site tensors)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    sites = [np.zeros((1, 2, 1), dtype=np.complex128) for _ in range(n)]
    for t in sites:
        t[0, 0, 0] = 1.0
    gates = feature_map_gates(x, reps)
    centre = 0  # the product start state is canonical about any site
    for name, qubits, param in gates:
        if name == "H":
            sites[qubits[0]] = _one_site(sites[qubits[0]], H_GATE)
        elif name == "P":
            sites[qubits[0]] = _one_site(sites[qubits[0]], p_gate(param))
        elif name == "CX":
            c = qubits[0]
            if centre not in (c, c + 1):
                _move_centre(sites, centre, c)
            _two_site(sites, c, CNOT_GATE)
            centre = c + 1
        else:  # pragma: no cover
            raise AssertionError(name)
    limit = 1 << reps
    for t in sites:
        if t.shape[0] > limit or t.shape[2] > limit:
            raise AssertionError("bond dimension exceeded 2^reps")
    return sites


def mps_to_statevector(sites) -> np.ndarray:
    """Contract an MPS into the dense vector (bit k of the index = qubit k); small n only."""
    n = len(sites)
    v = sites[0][0]  # (2, D)
    for k in range(1, n):
        v = np.einsum("...a,asb->...sb", v, sites[k])
    v = v[..., 0]  # shape (2,)*n, axis k = qubit k
    # axis order (q0, q1, ...) -> flat index with q0 as the least significant bit
    return np.transpose(v, tuple(range(n - 1, -1, -1))).reshape(-1)


def mps_overlap_log(sites_a, sites_b):
    """log|<B|A>| and the unit phase of <B|A> for two MPS of the same length.

    Returns (log_abs_amp, phase); log_abs_amp = -inf when the overlap is zero.
    """
    e = np.ones((1, 1), dtype=np.complex128)
    log_scale = 0.0
    for a, b in zip(sites_a, sites_b):
        t = np.einsum("yx,xsu->ysu", e, a)
        e = np.einsum("ysv,ysu->vu", b.conj(), t)
        m = np.max(np.abs(e))
        if m == 0.0:
            return -math.inf, 0.0 + 0.0j
        e = e / m
        log_scale += math.log(m)
    amp = e[0, 0]
    if amp == 0:
        return -math.inf, 0.0 + 0.0j
    return log_scale + math.log(abs(amp)), amp / abs(amp)


def _state_worker(args):
    x, reps = args
    return mps_state(x, reps)


def mps_states(X, reps: int, processes: int = 1):
    """MPS of every row of X, zero-padded per bond to a common shape.

    Returns a list over sites of arrays (N, D_left, 2, D_right).  Zero padding
    of a bond index leaves every contraction unchanged.
    """
    X = np.asarray(X, dtype=np.float64)
    if processes > 1 and X.shape[0] > 1:
        with get_context("fork").Pool(processes) as pool:
            states = pool.map(_state_worker, [(x, reps) for x in X], chunksize=1)
    else:
        states = [mps_state(x, reps) for x in X]
    n = X.shape[1]
    out = []
    for k in range(n):
        dl = max(s[k].shape[0] for s in states)
        dr = max(s[k].shape[2] for s in states)
        arr = np.zeros((len(states), dl, 2, dr), dtype=np.complex128)
        for i, s in enumerate(states):
            t = s[k]
            arr[i, : t.shape[0], :, : t.shape[2]] = t
        out.append(arr)
    return out


def mps_gram_pairs(states_a, states_b, ia, jb, batch: int = 4096):
    """log K for the pairs (ia[p], jb[p]): K = |<psi(b_jb)|psi(a_ia)>|^2.

    ``states_a`` / ``states_b`` come from ``mps_states``.  Returns
    (log_k, k): natural-log kernel values (-inf for an exact zero) and the
    kernel values themselves (0 where exp underflows in FP64).
    """
    ia = np.asarray(ia, dtype=np.int64)
    jb = np.asarray(jb, dtype=np.int64)
    P = ia.shape[0]
    log_abs = np.empty(P, dtype=np.float64)
    for p0 in range(0, P, batch):
        i = ia[p0 : p0 + batch]
        j = jb[p0 : p0 + batch]
        e = np.ones((i.shape[0], 1, 1), dtype=np.complex128)
        log_scale = np.zeros(i.shape[0], dtype=np.float64)
        for a_k, b_k in zip(states_a, states_b):
            t = np.einsum("pyx,pxsu->pysu", e, a_k[i])
            e = np.einsum("pysv,pysu->pvu", b_k[j].conj(), t)
            m = np.max(np.abs(e), axis=(1, 2))
            safe = np.where(m > 0.0, m, 1.0)
            e = e / safe[:, None, None]
            log_scale += np.where(m > 0.0, np.log(safe), -np.inf)
        amp = np.abs(e[:, 0, 0])
        with np.errstate(divide="ignore"):
            log_abs[p0 : p0 + batch] = log_scale + np.log(amp)
    log_k = 2.0 * log_abs
    with np.errstate(under="ignore"):
        k = np.exp(log_k)
    return log_k, k
