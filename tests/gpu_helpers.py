"""Helpers for the GPU tests: run the HIP path through the C-ABI binding and
contract the MPS buffers it writes on the host (reading the documented layout
of include/qsvm.h, independently of the kernels)."""

from __future__ import annotations

import numpy as np

# Floating-point bars.  The kernel path carries the environment in FP32 and
# forms |amp|^2 in FP64.
#  * K_ABS_TOL: the absolute bar on kernel entries (1e-5), the contract.
#  * LOG_TOL_MAX / LOG_TOL_MEDIAN: bars on |ln K_gpu - ln K_oracle| for
#    entries far below 1e-5, where the absolute bar says nothing.  Each site
#    step rounds every environment entry a few times (relative 2^-24); over
#    n <= 784 sites this is a relative amplitude error of order
#    sqrt(10 n) 6e-8 ~ 5e-6, i.e. ~1e-5 in ln K -- the typical case, bounded
#    by LOG_TOL_MEDIAN.  An amplitude that is itself the result of
#    cancellation (a final sum ~10^3 times smaller than the entries it adds)
#    multiplies that relative error by the cancellation ratio; FP32 emulation
#    of both sweeps on 784-site pairs with K ~ 1e-80 shows up to 3e-4 (gauge
#    sweep) and 1.4e-3 (dense sweep).  LOG_TOL_MAX = 5e-3 (K within 0.5 %
#    relative) still exposes any algebraic mistake, which shows as O(1).
K_ABS_TOL = 1e-5
LOG_TOL_MAX = 5e-3
LOG_TOL_MEDIAN = 5e-5


def log_close(err):
    """True when an array of |ln K| errors meets both log-domain bars."""
    err = np.asarray(err, dtype=np.float64).ravel()
    return err.size == 0 or (float(np.max(err)) <= LOG_TOL_MAX and float(np.median(err)) <= LOG_TOL_MEDIAN)


def require_gpu():
    import torch

    assert torch.cuda.is_available(), "GPU test needs a visible MI355X"
    return torch.device("cuda:0")


def to_dev(X):
    import torch

    return torch.as_tensor(np.ascontiguousarray(X, dtype=np.float64), device="cuda:0")


def encode(X, reps, dense=False):
    from paper_2405_02630_amd import qsvm

    return qsvm.qsvm_encode_mps(to_dev(X), reps, dense=dense)


def gram_sym(X, reps, log=True, **kw):
    import torch
    from paper_2405_02630_amd import qsvm

    m = encode(X, reps, dense=kw.get("sweep") == qsvm.SWEEP_DENSE)
    K = torch.empty((m.N, m.N), dtype=torch.float64, device="cuda:0")
    L = torch.empty_like(K) if log else None
    qsvm.qsvm_gram_sym(m, K, log_k=L, **kw)
    torch.cuda.synchronize()
    return K.cpu().numpy(), (L.cpu().numpy() if log else None)


def gram_rect(Xa, Xb, reps, log=True, **kw):
    import torch
    from paper_2405_02630_amd import qsvm

    dense = kw.get("sweep") == qsvm.SWEEP_DENSE
    ma, mb = encode(Xa, reps, dense), encode(Xb, reps, dense)
    K = torch.empty((ma.N, mb.N), dtype=torch.float64, device="cuda:0")
    L = torch.empty_like(K) if log else None
    qsvm.qsvm_gram(ma, mb, K, log_k=L, **kw)
    torch.cuda.synchronize()
    return K.cpu().numpy(), (L.cpu().numpy() if log else None)


def mps_sections(m, residuals=False):
    """Host copies of the dense tensors (n, N, chi, chi complex; None unless
    encoded with dense=True) and of Section G (n, N, 4 float), and with
    residuals=True also Section L (n, N, 4 float)."""
    N, n, reps = m.N, m.n, m.reps
    chi = 1 << reps
    raw = m.buf.cpu().numpy()
    assert raw.size == n * N * 32  # the MPS buffer: Sections G and L only
    dense = None
    if m.dense is not None:
        dense = m.dense.cpu().numpy()[: n * N * chi * chi * 8].view(np.complex64).reshape(n, N, chi, chi)
    gen = raw[: n * N * 16].view(np.float32).reshape(n, N, 4)
    if residuals:
        lo = raw[n * N * 16 : n * N * 32].view(np.float32).reshape(n, N, 4)
        return dense, gen, lo
    return dense, gen


def _popcount(x):
    return bin(x).count("1")


def _sgn(beta, reps):
    c = beta
    return -1.0 if _popcount(c & (c >> 1)) % 2 else 1.0


def contract_dense(site_tensors, reps, right=None):
    """psi(s) = e_0^T A_0^{s_0} ... A_{n-1}^{s_{n-1}} r for one point.

    site_tensors: (n, chi, chi) complex; A^s[a, b] = A[a, b] if top bit of b == s.
    right: right boundary vector over b (default all ones).  Bit k of the
    returned index is qubit k."""
    n, chi, _ = site_tensors.shape
    top = np.array([(b >> (reps - 1)) & 1 for b in range(chi)])
    cur = site_tensors[0][0].astype(np.complex128)[None, :]  # (strings=1, b)
    cur = np.stack([np.where(top == s, cur[0], 0) for s in (0, 1)])  # (2, chi): s_0
    for k in range(1, n):
        nxt = cur @ site_tensors[k].astype(np.complex128)  # (2^k, chi)
        cur = np.concatenate([np.where(top == 0, nxt, 0), np.where(top == 1, nxt, 0)], axis=0)
    r = np.ones(chi) if right is None else right
    return cur @ r


def gauge_tensors(gen_point, reps):
    """Section G generators of one point -> (site tensors (n, chi, chi), right boundary)."""
    n = gen_point.shape[0]
    chi = 1 << reps
    scale = 2.0 ** (-reps / 2)
    T = np.zeros((n, chi, chi), dtype=np.complex128)
    for b in range(chi):
        T[0, :, b] = scale * _sgn(b, reps)  # every row; only row 0 is used
    for k in range(1, n):
        a = complex(gen_point[k, 0], gen_point[k, 1])
        bb = complex(gen_point[k, 2], gen_point[k, 3])
        C = np.array([[1.0, a], [1.0, bb]])  # C[new][old]
        for al in range(chi):
            for be in range(chi):
                v = scale * _sgn(be, reps)
                for l in range(reps):
                    v *= C[(be >> l) & 1, (al >> l) & 1]
                T[k, al, be] = v
    g = complex(gen_point[0, 0], gen_point[0, 1])
    right = np.array([g ** _popcount(b) for b in range(chi)])
    return T, right
