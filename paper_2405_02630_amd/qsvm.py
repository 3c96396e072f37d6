"""Python binding of libqsvm.so (argument marshalling only).

The functions ``qsvm_mps_bytes``, ``qsvm_encode_mps``, ``qsvm_gram`` and
``qsvm_gram_sym`` have the names and meaning of the C entry points declared
in include/qsvm.h; they take PyTorch CUDA tensors for device memory and launch
on the current PyTorch stream.  Every step of the computation runs in the HIP
kernels of the library: if the library cannot be loaded these functions raise
and there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsvm.so")

QSVM_OK = 0
QSVM_ERR_INVALID_ARG = -1
QSVM_ERR_UNSUPPORTED = -2
QSVM_ERR_HIP = -3
QSVM_ERR_SIZE = -4

SWEEP_AUTO = 0
SWEEP_BUTTERFLY = 1
SWEEP_DENSE = 2


class GramOpts(ctypes.Structure):
    """Mirror of qsvm_gram_opts."""

    _fields_ = [
        ("renorm_every", ctypes.c_int32),
        ("sweep", ctypes.c_int32),
        ("diag_mode", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("row_begin", ctypes.c_int64),
        ("row_end", ctypes.c_int64),
        ("log_k", ctypes.c_void_p),
        ("refine_above", ctypes.c_double),
        ("dense_a", ctypes.c_void_p),
        ("dense_b", ctypes.c_void_p),
    ]


class Job(ctypes.Structure):
    """Mirror of qsvm_job."""

    _fields_ = [
        ("mps", ctypes.c_void_p),
        ("N", ctypes.c_int64),
        ("n_qubits", ctypes.c_int32),
        ("reps", ctypes.c_int32),
        ("K", ctypes.c_void_p),
        ("ldk", ctypes.c_int64),
        ("log_k", ctypes.c_void_p),
    ]


class BatchOpts(ctypes.Structure):
    """Mirror of qsvm_batch_opts."""

    _fields_ = [
        ("renorm_every", ctypes.c_int32),
        ("diag_mode", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32),
        ("refine_above", ctypes.c_double),
        ("item_pi2", ctypes.c_int32),
        ("item_pi3", ctypes.c_int32),
    ]


class Mlp(ctypes.Structure):
    """Mirror of qsvm_mlp."""

    _fields_ = [
        ("d_in", ctypes.c_int32), ("d_h1", ctypes.c_int32), ("d_h2", ctypes.c_int32), ("d_out", ctypes.c_int32),
        ("W1", ctypes.c_void_p), ("b1", ctypes.c_void_p),
        ("W2", ctypes.c_void_p), ("b2", ctypes.c_void_p),
        ("W3", ctypes.c_void_p), ("b3", ctypes.c_void_p),
    ]


class MlpActs(ctypes.Structure):
    """Mirror of qsvm_mlp_acts."""

    _fields_ = [("H1", ctypes.c_void_p), ("A1", ctypes.c_void_p), ("H2", ctypes.c_void_p),
                ("A2", ctypes.c_void_p), ("E", ctypes.c_void_p), ("E16", ctypes.c_void_p)]


class MlpGrads(ctypes.Structure):
    """Mirror of qsvm_mlp_grads."""

    _fields_ = [("dW1", ctypes.c_void_p), ("db1", ctypes.c_void_p), ("dW2", ctypes.c_void_p),
                ("db2", ctypes.c_void_p), ("dW3", ctypes.c_void_p), ("db3", ctypes.c_void_p),
                ("dH1", ctypes.c_void_p), ("dH2", ctypes.c_void_p), ("ws", ctypes.c_void_p),
                ("ws_floats", ctypes.c_int64)]


class QsvmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libqsvm.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} not found: build it with `python -m paper_2405_02630_amd.build` "
            "(there is no fallback implementation)"
        )
    lib = ctypes.CDLL(path)
    i32, i64, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    lib.qsvm_mps_bytes.argtypes = [i64, i32, i32]
    lib.qsvm_mps_bytes.restype = sz
    lib.qsvm_encode_mps.argtypes = [vp, i64, i32, i32, vp, sz, vp]
    lib.qsvm_encode_mps.restype = i32
    lib.qsvm_dense_bytes.argtypes = [i64, i32, i32]
    lib.qsvm_dense_bytes.restype = sz
    lib.qsvm_encode_dense.argtypes = [vp, i64, i32, i32, vp, sz, vp]
    lib.qsvm_encode_dense.restype = i32
    lib.qsvm_auto_refine_threshold.argtypes = [i32]
    lib.qsvm_auto_refine_threshold.restype = ctypes.c_double
    lib.qsvm_gram.argtypes = [vp, i64, vp, i64, i32, i32, vp, i64, ctypes.POINTER(GramOpts), vp]
    lib.qsvm_gram.restype = i32
    lib.qsvm_gram_sym.argtypes = [vp, i64, i32, i32, vp, i64, ctypes.POINTER(GramOpts), vp]
    lib.qsvm_gram_sym.restype = i32
    lib.qsvm_gram_sym_noalloc.argtypes = [vp, i64, i32, i32, vp, i64, ctypes.POINTER(GramOpts), vp]
    lib.qsvm_gram_sym_noalloc.restype = i32
    lib.qsvm_status_string.argtypes = [i32]
    lib.qsvm_status_string.restype = ctypes.c_char_p
    lib.qsvm_last_error.argtypes = []
    lib.qsvm_last_error.restype = ctypes.c_char_p
    lib.qsvm_abi_version.argtypes = []
    lib.qsvm_abi_version.restype = i32
    lib.qsvm_batch_plan_create.argtypes = [ctypes.POINTER(Job), i32, ctypes.POINTER(BatchOpts), ctypes.POINTER(vp)]
    lib.qsvm_batch_plan_create.restype = i32
    lib.qsvm_batch_plan_launch.argtypes = [vp, vp]
    lib.qsvm_batch_plan_launch.restype = i32
    lib.qsvm_batch_plan_destroy.argtypes = [vp]
    lib.qsvm_batch_plan_destroy.restype = i32
    lib.qsvm_batch_plan_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.qsvm_batch_plan_info.restype = i32
    P = ctypes.POINTER
    f32 = ctypes.c_float
    lib.qsvm_gram_sym_tiles.argtypes = [vp, i64, i32, i32, vp, i64, vp, i64, P(GramOpts), vp]
    lib.qsvm_gram_sym_tiles.restype = i32
    lib.qsvm_gram_sym_tiles_dev.argtypes = [vp, i64, i32, i32, vp, vp, i64, vp, i64, P(GramOpts), vp]
    lib.qsvm_gram_sym_tiles_dev.restype = i32
    lib.qsvm_gram_sym_pairs_dev.argtypes = [vp, i64, i32, i32, vp, vp, i64, vp, i64, P(GramOpts), vp]
    lib.qsvm_gram_sym_pairs_dev.restype = i32
    lib.qsvm_gather_features.argtypes = [vp, i64, i32, vp, i64, i32, vp, vp]
    lib.qsvm_gather_features.restype = i32
    lib.qsvm_mlp_forward.argtypes = [P(Mlp), vp, i64, P(MlpActs), vp]
    lib.qsvm_mlp_forward.restype = i32
    lib.qsvm_pair_head.argtypes = [vp, i64, i32, vp, vp, i32, vp, vp, vp, vp]
    lib.qsvm_pair_head.restype = i32
    lib.qsvm_pair_head_log.argtypes = [vp, i32, vp, i32, i64, vp, vp, f32, vp, vp, vp, vp, vp]
    lib.qsvm_pair_head_log.restype = i32
    lib.qsvm_surrogate_gram_log.argtypes = [vp, i32, vp, i32, i64, i64, vp, vp, i64, vp, vp]
    lib.qsvm_surrogate_gram_log.restype = i32
    lib.qsvm_mlp_backward.argtypes = [P(Mlp), vp, P(MlpActs), vp, i64, P(MlpGrads), vp]
    lib.qsvm_mlp_backward.restype = i32
    lib.qsvm_mlp_workspace_floats.argtypes = [P(Mlp), i64]
    lib.qsvm_mlp_workspace_floats.restype = i64
    lib.qsvm_adamw.argtypes = [vp, vp, vp, vp, vp, i64, f32, f32, f32, f32, f32, i32, vp]
    lib.qsvm_adamw.restype = i32
    lib.qsvm_surrogate_gram.argtypes = [vp, i64, i64, i32, vp, vp, i64, vp, vp]
    lib.qsvm_surrogate_gram.restype = i32
    lib.qsvm_flag_tiles.argtypes = [vp, i32, f32, vp, vp, vp]
    lib.qsvm_flag_tiles.restype = i32
    lib.qsvm_flag_pairs.argtypes = [vp, i64, i64, vp, vp, i64, ctypes.c_double, i32, vp, vp, i64, vp, vp, vp]
    lib.qsvm_flag_pairs.restype = i32
    lib.qsvm_autotune.argtypes = [i32, i32, i64, vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float), i32]
    lib.qsvm_sv_bytes.argtypes = [i64, i32]
    lib.qsvm_sv_bytes.restype = ctypes.c_size_t
    lib.qsvm_encode_sv.argtypes = [vp, i64, i32, i32, vp, ctypes.c_size_t, vp]
    lib.qsvm_encode_sv.restype = i32
    lib.qsvm_sv_gram.argtypes = [vp, i64, vp, i64, i32, vp, i64, P(GramOpts), vp]
    lib.qsvm_sv_gram.restype = i32
    lib.qsvm_sv_gram_sym.argtypes = [vp, i64, i32, vp, i64, P(GramOpts), vp]
    lib.qsvm_sv_gram_sym.restype = i32
    lib.qsvm_autotune.restype = i32
    lib.qsvm_batch_plan_shape.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.qsvm_batch_plan_shape.restype = i32
    lib.qsvm_autotune_save.argtypes = []
    lib.qsvm_autotune_save.restype = i32
    lib.qsvm_autotune_cache_path.argtypes = []
    lib.qsvm_autotune_cache_path.restype = ctypes.c_char_p
    lib.qsvm_get_tuned_variant.argtypes = [i32, i32, i64]
    lib.qsvm_get_tuned_variant.restype = i32
    lib.qsvm_set_tuned_variant.argtypes = [i32, i32, i64, i32]
    lib.qsvm_set_tuned_variant.restype = i32
    _lib = lib
    return lib


def _check(status: int) -> None:
    if status != QSVM_OK:
        lib = load_library()
        msg = lib.qsvm_last_error().decode() or lib.qsvm_status_string(status).decode()
        raise QsvmError(status, msg)


def _stream_ptr(stream):
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _device_ptr(t, name, dtype=None):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class MPS:
    """Device MPS buffer written by qsvm_encode_mps (layout in include/qsvm.h),
    with the dense site tensors of qsvm_encode_dense when they were asked for
    (only the dense sweep reads them)."""

    buf: "object"  # torch.uint8 CUDA tensor
    N: int
    n: int
    reps: int
    dense: "object" = None  # torch.uint8 CUDA tensor or None


def qsvm_mps_bytes(N: int, n_qubits: int, reps: int) -> int:
    return int(load_library().qsvm_mps_bytes(N, n_qubits, reps))


def qsvm_dense_bytes(N: int, n_qubits: int, reps: int) -> int:
    return int(load_library().qsvm_dense_bytes(N, n_qubits, reps))


def qsvm_encode_dense(X, reps: int, out=None, stream=None):
    """Dense site tensors of the rows of X (a uint8 CUDA tensor of qsvm_dense_bytes)."""
    import torch

    lib = load_library()
    N, n = int(X.shape[0]), int(X.shape[1])
    if out is None:
        out = torch.empty(max(1, lib.qsvm_dense_bytes(N, n, reps)), dtype=torch.uint8, device=X.device)
    _check(lib.qsvm_encode_dense(_device_ptr(X, "X", torch.float64), N, n, reps, _device_ptr(out, "out"), out.numel(),
                                 _stream_ptr(stream)))
    return out


def qsvm_encode_mps(X, reps: int, out=None, stream=None, dense: bool = False) -> MPS:
    """Encode the rows of X (CUDA float64, N x n) as exact MPS; with dense=True
    also write the dense site tensors (for the dense sweep) into m.dense."""
    import torch

    lib = load_library()
    if X.dim() != 2:
        raise ValueError("X must be 2-D (N x n_qubits)")
    N, n = int(X.shape[0]), int(X.shape[1])
    need = lib.qsvm_mps_bytes(N, n, reps)
    if out is None:
        if need == 0:
            # let the library produce the precise error
            _check(lib.qsvm_encode_mps(_device_ptr(X, "X", torch.float64), N, n, reps, None, 0, _stream_ptr(stream)))
        out = torch.empty(need, dtype=torch.uint8, device=X.device)
    st = lib.qsvm_encode_mps(
        _device_ptr(X, "X", torch.float64), N, n, reps, _device_ptr(out, "out"), out.numel(), _stream_ptr(stream)
    )
    _check(st)
    return MPS(out, N, n, reps, qsvm_encode_dense(X, reps, stream=stream) if dense else None)


N_VARIANTS = 4


def qsvm_autotune_cache_path() -> str:
    return load_library().qsvm_autotune_cache_path().decode()


def qsvm_autotune_save() -> None:
    _check(load_library().qsvm_autotune_save())


def qsvm_autotune(reps: int, n_qubits: int, N: int, stream=None):
    """Time every butterfly variant on a synthetic (N, n_qubits, reps) Gram and
    record the fastest for later launches.  Returns (best, [ms per variant])."""
    lib = load_library()
    best = ctypes.c_int32(0)
    ms = (ctypes.c_float * N_VARIANTS)()
    _check(lib.qsvm_autotune(reps, n_qubits, N, _stream_ptr(stream), ctypes.byref(best), ms, N_VARIANTS))
    return int(best.value), [float(x) for x in ms]


def qsvm_get_tuned_variant(reps: int, n_qubits: int, N: int) -> int:
    return int(load_library().qsvm_get_tuned_variant(reps, n_qubits, N))


def qsvm_set_tuned_variant(reps: int, n_qubits: int, N: int, variant: int) -> None:
    _check(load_library().qsvm_set_tuned_variant(reps, n_qubits, N, variant))


def _opts(renorm_every, sweep, diag_mode, rows, log_k, variant=0, refine_above=0.0, dense_a=None, dense_b=None):
    o = GramOpts()
    o.dense_a = None if dense_a is None else dense_a.data_ptr()
    o.dense_b = None if dense_b is None else dense_b.data_ptr()
    o.refine_above = refine_above
    o.variant = variant
    o.renorm_every = renorm_every
    o.sweep = sweep
    o.diag_mode = diag_mode
    if rows is not None:
        o.row_begin, o.row_end = int(rows[0]), int(rows[1])
    o.log_k = None if log_k is None else log_k.data_ptr()
    return o


def qsvm_auto_refine_threshold(n_qubits: int) -> float:
    """Threshold of the automatic FP64 refinement for n_qubits (>= 1: none)."""
    return float(load_library().qsvm_auto_refine_threshold(n_qubits))


def qsvm_gram(mps_a: MPS, mps_b: MPS, K=None, *, log_k=None, renorm_every: int = 0,
              sweep: int = SWEEP_AUTO, rows=None, variant: int = 0, refine_above: float = 0.0, stream=None):
    """K[i, j] = |<psi(b_j)|psi(a_i)>|^2 (CUDA float64, Na x Nb).  Returns K.
    refine_above: tiles with an entry above it are recomputed in FP64 (0 =
    automatic from n_qubits, negative = off)."""
    import torch

    lib = load_library()
    if mps_a.n != mps_b.n or mps_a.reps != mps_b.reps:
        raise ValueError("both MPS sets need the same n_qubits and reps")
    if K is None:
        K = torch.empty((mps_a.N, mps_b.N), dtype=torch.float64, device=mps_a.buf.device)
    if K.dim() != 2 or K.shape[0] < mps_a.N or K.stride(1) != 1:
        raise ValueError("K must be 2-D with unit column stride and at least Na rows")
    if log_k is not None and (log_k.shape != K.shape or log_k.stride() != K.stride() or log_k.dtype != torch.float64):
        raise ValueError("log_k must match K's shape, strides and dtype")
    o = _opts(renorm_every, sweep, 0, rows, log_k, variant, refine_above, mps_a.dense, mps_b.dense)
    st = lib.qsvm_gram(
        _device_ptr(mps_a.buf, "mps_a"), mps_a.N, _device_ptr(mps_b.buf, "mps_b"), mps_b.N, mps_a.n, mps_a.reps,
        ctypes.c_void_p(K.data_ptr()), K.stride(0), ctypes.byref(o), _stream_ptr(stream),
    )
    _check(st)
    return K


def qsvm_gram_sym(mps: MPS, K=None, *, log_k=None, renorm_every: int = 0, sweep: int = SWEEP_AUTO,
                  diag_mode: int = 0, rows=None, variant: int = 0, refine_above: float = 0.0, stream=None):
    """Symmetric Gram of one set: pairs i < j contracted, mirrored, K[i, i] = 1
    (diag_mode 0) or computed (diag_mode 1).  Returns K."""
    import torch

    lib = load_library()
    if K is None:
        K = torch.empty((mps.N, mps.N), dtype=torch.float64, device=mps.buf.device)
    if K.dim() != 2 or K.shape[0] < mps.N or K.stride(1) != 1:
        raise ValueError("K must be 2-D with unit column stride and at least N rows")
    if log_k is not None and (log_k.shape != K.shape or log_k.stride() != K.stride() or log_k.dtype != torch.float64):
        raise ValueError("log_k must match K's shape, strides and dtype")
    o = _opts(renorm_every, sweep, diag_mode, rows, log_k, variant, refine_above, mps.dense)
    st = lib.qsvm_gram_sym(
        _device_ptr(mps.buf, "mps"), mps.N, mps.n, mps.reps, ctypes.c_void_p(K.data_ptr()), K.stride(0),
        ctypes.byref(o), _stream_ptr(stream),
    )
    _check(st)
    return K


NOALLOC_SCRATCH_ENTRIES = 1 << 20  # QSVM_NOALLOC_SCRATCH_ENTRIES


def qsvm_gram_sym_noalloc(mps: MPS, K, *, log_k=None, renorm_every: int = 0, sweep: int = SWEEP_AUTO,
                          diag_mode: int = 0, rows=None, variant: int = 0, refine_above: float = 0.0,
                          stream=None):
    """qsvm_gram_sym without any device allocation by the library: the
    refinement's tile list lives in a static per-device array.  K (and log_k)
    must be supplied by the caller.  Calls overlapping on one device race."""
    import torch

    lib = load_library()
    if K is None or K.dim() != 2 or K.shape[0] < mps.N or K.stride(1) != 1 or K.dtype != torch.float64:
        raise ValueError("K must be a float64 2-D tensor with unit column stride and at least N rows")
    if log_k is not None and (log_k.shape != K.shape or log_k.stride() != K.stride() or log_k.dtype != torch.float64):
        raise ValueError("log_k must match K's shape, strides and dtype")
    o = _opts(renorm_every, sweep, diag_mode, rows, log_k, variant, refine_above, mps.dense)
    st = lib.qsvm_gram_sym_noalloc(
        _device_ptr(mps.buf, "mps"), mps.N, mps.n, mps.reps, ctypes.c_void_p(K.data_ptr()), K.stride(0),
        ctypes.byref(o), _stream_ptr(stream),
    )
    _check(st)
    return K


@dataclass
class SV:
    """Device states written by qsvm_encode_sv (N x 2^n complex128)."""

    buf: "object"  # torch.complex128 CUDA tensor, N x 2^n
    N: int
    n: int
    reps: int


def qsvm_sv_bytes(N: int, n_qubits: int) -> int:
    return int(load_library().qsvm_sv_bytes(N, n_qubits))


def qsvm_encode_sv(X, reps: int, out=None, stream=None) -> SV:
    """Full state vectors of the rows of X (CUDA float64, N x n), n <= 30."""
    import torch

    lib = load_library()
    if X.dim() != 2:
        raise ValueError("X must be 2-D (N x n_qubits)")
    N, n = int(X.shape[0]), int(X.shape[1])
    need = lib.qsvm_sv_bytes(N, n)
    if out is None:
        if need == 0:
            _check(lib.qsvm_encode_sv(_device_ptr(X, "X", torch.float64), N, n, reps, None, 0, _stream_ptr(stream)))
        out = torch.empty((N, 1 << n), dtype=torch.complex128, device=X.device)
    st = lib.qsvm_encode_sv(_device_ptr(X, "X", torch.float64), N, n, reps, _device_ptr(out, "out"),
                            out.numel() * out.element_size(), _stream_ptr(stream))
    _check(st)
    return SV(out, N, n, reps)


def _check_k(K, rows, log_k):
    import torch

    if K.dim() != 2 or K.shape[0] < rows or K.stride(1) != 1:
        raise ValueError("K must be 2-D with unit column stride and enough rows")
    if log_k is not None and (log_k.shape != K.shape or log_k.stride() != K.stride() or log_k.dtype != torch.float64):
        raise ValueError("log_k must match K's shape, strides and dtype")


def qsvm_sv_gram(sa: SV, sb: SV, K=None, *, log_k=None, rows=None, stream=None):
    """K[i, j] = |<psi(b_j)|psi(a_i)>|^2 from full states.  Returns K."""
    import torch

    lib = load_library()
    if sa.n != sb.n:
        raise ValueError("both state sets need the same n_qubits")
    if K is None:
        K = torch.empty((sa.N, sb.N), dtype=torch.float64, device=sa.buf.device)
    _check_k(K, sa.N, log_k)
    o = _opts(0, SWEEP_AUTO, 0, rows, log_k)
    _check(lib.qsvm_sv_gram(_device_ptr(sa.buf, "sv_a"), sa.N, _device_ptr(sb.buf, "sv_b"), sb.N, sa.n,
                            ctypes.c_void_p(K.data_ptr()), K.stride(0), ctypes.byref(o), _stream_ptr(stream)))
    return K


def qsvm_sv_gram_sym(s: SV, K=None, *, log_k=None, diag_mode: int = 0, rows=None, stream=None):
    """Symmetric Gram from full states (pairs i < j, mirrored).  Returns K."""
    import torch

    lib = load_library()
    if K is None:
        K = torch.empty((s.N, s.N), dtype=torch.float64, device=s.buf.device)
    _check_k(K, s.N, log_k)
    o = _opts(0, SWEEP_AUTO, diag_mode, rows, log_k)
    _check(lib.qsvm_sv_gram_sym(_device_ptr(s.buf, "sv"), s.N, s.n, ctypes.c_void_p(K.data_ptr()), K.stride(0),
                                ctypes.byref(o), _stream_ptr(stream)))
    return K


class BatchPlan:
    """A qsvm_batch_plan over symmetric Gram jobs [(MPS, K, log_k or None), ...].

    Holds references to every job buffer for its lifetime; ``launch`` enqueues
    one execution on the current PyTorch stream."""

    def __init__(self, jobs, *, renorm_every: int = 0, diag_mode: int = 0, use_graph: bool = True,
                 grid_blocks: int = 0, refine_above: float = 0.0, item_pi2: int = 0, item_pi3: int = 0):
        lib = load_library()
        self._keep = list(jobs)
        arr = (Job * len(jobs))()
        for q, (m, K, L) in enumerate(jobs):
            if K.dim() != 2 or K.shape[0] < m.N or K.shape[1] < m.N or K.stride(1) != 1:
                raise ValueError(f"job {q}: K must be at least N x N with unit column stride")
            arr[q].mps = _device_ptr(m.buf, f"job {q} mps").value
            arr[q].N = m.N
            arr[q].n_qubits = m.n
            arr[q].reps = m.reps
            arr[q].K = K.data_ptr()
            arr[q].ldk = K.stride(0)
            arr[q].log_k = None if L is None else L.data_ptr()
        o = BatchOpts(renorm_every, diag_mode, 1 if use_graph else 0, grid_blocks, refine_above, item_pi2, item_pi3)
        h = ctypes.c_void_p()
        _check(lib.qsvm_batch_plan_create(arr, len(jobs), ctypes.byref(o), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(load_library().qsvm_batch_plan_launch(self._h, _stream_ptr(stream)))

    def info(self):
        t = ctypes.c_int64()
        g = ctypes.c_int32()
        u = ctypes.c_int32()
        _check(load_library().qsvm_batch_plan_info(self._h, ctypes.byref(t), ctypes.byref(g), ctypes.byref(u)))
        return int(t.value), int(g.value), bool(u.value)

    def shape(self):
        """(ket points per lane of the reps = 2 items, of the reps = 3 items)."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(load_library().qsvm_batch_plan_shape(self._h, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def close(self):
        if self._h:
            load_library().qsvm_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# Surrogate building blocks (tensors are CUDA; bf16 buffers are torch.bfloat16)
# --------------------------------------------------------------------------

def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def qsvm_gram_sym_tiles(mps: MPS, tiles, n_tiles: int, K, *, log_k=None, renorm_every: int = 0,
                        sweep: int = SWEEP_AUTO, diag_mode: int = 0, variant: int = 0, refine_above: float = 0.0,
                        stream=None):
    """Exact symmetric Gram on a device list of (ti, tj) tiles (int32 tensor)."""
    o = _opts(renorm_every, sweep, diag_mode, None, log_k, variant, refine_above, mps.dense)
    _check(load_library().qsvm_gram_sym_tiles(
        _device_ptr(mps.buf, "mps"), mps.N, mps.n, mps.reps, _p(tiles), n_tiles, _p(K), K.stride(0),
        ctypes.byref(o), _stream_ptr(stream)))
    return K


def qsvm_gram_sym_tiles_dev(mps: MPS, tiles, tile_count, max_tiles: int, K, *, log_k=None, renorm_every: int = 0,
                            diag_mode: int = 0, variant: int = 0, refine_above: float = 0.0, stream=None):
    """qsvm_gram_sym_tiles with the list length in device memory (tile_count:
    1-element int32 tensor, read by the kernels, clamped to [0, max_tiles])."""
    o = _opts(renorm_every, SWEEP_AUTO, diag_mode, None, log_k, variant, refine_above)
    _check(load_library().qsvm_gram_sym_tiles_dev(
        _device_ptr(mps.buf, "mps"), mps.N, mps.n, mps.reps, _p(tiles), _p(tile_count), max_tiles, _p(K),
        K.stride(0), ctypes.byref(o), _stream_ptr(stream)))
    return K


def qsvm_gram_sym_pairs_dev(mps: MPS, pairs, pair_count, max_pairs: int, K, *, log_k=None, renorm_every: int = 0,
                            diag_mode: int = 0, stream=None):
    """FP64 entries of the listed pairs (pairs: int32 (i, j) rows; pair_count:
    1-element int32 tensor read by the kernels, clamped to [0, max_pairs])."""
    o = _opts(renorm_every, SWEEP_AUTO, diag_mode, None, log_k)
    _check(load_library().qsvm_gram_sym_pairs_dev(
        _device_ptr(mps.buf, "mps"), mps.N, mps.n, mps.reps, _p(pairs), _p(pair_count), max_pairs, _p(K),
        K.stride(0), ctypes.byref(o), _stream_ptr(stream)))
    return K


def qsvm_gather_features(X, idx, d_pad: int, out, stream=None):
    _check(load_library().qsvm_gather_features(
        _p(X), X.shape[0], X.shape[1], _p(idx), idx.shape[0], d_pad, _p(out), _stream_ptr(stream)))
    return out


def qsvm_mlp_forward(net: Mlp, X16, rows: int, acts: MlpActs, stream=None):
    _check(load_library().qsvm_mlp_forward(ctypes.byref(net), _p(X16), rows, ctypes.byref(acts), _stream_ptr(stream)))


LOSS_MSE = 0
LOSS_BCE = 1


def qsvm_pair_head(E, pairs: int, d: int, target, alpha_beta, dE16, partial, out3, loss_kind: int = LOSS_BCE,
                   stream=None):
    _check(load_library().qsvm_pair_head(_p(E), pairs, d, _p(target), _p(alpha_beta), loss_kind, _p(dE16),
                                         _p(partial), _p(out3), _stream_ptr(stream)))


def qsvm_pair_head_log(X16, E, pairs: int, target, head, scale: float, dE16, partial, out3, pred=None,
                       stream=None):
    """Log-domain pair head on [X16 row, E row] (see include/qsvm.h)."""
    d_in = 0 if X16 is None else X16.shape[1]
    _check(load_library().qsvm_pair_head_log(_p(X16) if d_in else None, d_in, _p(E), E.shape[1], pairs, _p(target), _p(head),
                                             float(scale), _p(dE16), _p(partial), _p(out3),
                                             None if pred is None else _p(pred), _stream_ptr(stream)))


def qsvm_surrogate_gram_log(X16, E16, N: int, head, K, tile_max, stream=None):
    """K = exp(ln K_hat) of all pairs of rows of [X16, E16]; per-tile max ln K_hat."""
    if X16 is not None and X16.shape[0] != E16.shape[0]:
        raise ValueError("X16 and E16 need the same (padded) row count")
    d_in = 0 if X16 is None else X16.shape[1]
    _check(load_library().qsvm_surrogate_gram_log(_p(X16) if d_in else None, d_in, _p(E16), E16.shape[1], N,
                                                  E16.shape[0],
                                                  _p(head), _p(K), K.stride(0), _p(tile_max), _stream_ptr(stream)))
    return K


def qsvm_mlp_backward(net: Mlp, X16, acts: MlpActs, dE16, rows: int, grads: MlpGrads, stream=None):
    _check(load_library().qsvm_mlp_backward(ctypes.byref(net), _p(X16), ctypes.byref(acts), _p(dE16), rows,
                                            ctypes.byref(grads), _stream_ptr(stream)))


def qsvm_mlp_workspace_floats(net: Mlp, rows: int) -> int:
    return int(load_library().qsvm_mlp_workspace_floats(ctypes.byref(net), rows))


def qsvm_adamw(w, grad, m, v, w16, lr, beta1, beta2, eps, weight_decay, step, stream=None):
    _check(load_library().qsvm_adamw(_p(w), _p(grad), _p(m), _p(v), _p(w16), w.numel(), lr, beta1, beta2, eps,
                                     weight_decay, step, _stream_ptr(stream)))


def qsvm_surrogate_gram(E16, N: int, alpha_beta, K, tile_max, stream=None):
    _check(load_library().qsvm_surrogate_gram(_p(E16), N, E16.shape[0], E16.shape[1], _p(alpha_beta), _p(K),
                                              K.stride(0), _p(tile_max), _stream_ptr(stream)))
    return K


def qsvm_flag_tiles(tile_max, T: int, tau: float, tile_list, count, stream=None):
    _check(load_library().qsvm_flag_tiles(_p(tile_max), T, tau, _p(tile_list), _p(count), _stream_ptr(stream)))


def qsvm_flag_pairs(K, N: int, tiles, tile_count, max_tiles: int, cut: float, cap_per_tile: int, pairs, pair_count,
                    max_pairs: int, dense_tiles, dense_count, stream=None):
    """Pairs of the listed tiles with K >= cut (at most cap_per_tile per tile,
    else the tile goes to dense_tiles); counts written to the 1-element int32
    tensors pair_count and dense_count."""
    _check(load_library().qsvm_flag_pairs(_p(K), N, K.stride(0), _p(tiles), _p(tile_count), max_tiles, cut,
                                          cap_per_tile, _p(pairs), _p(pair_count), max_pairs, _p(dense_tiles),
                                          _p(dense_count), _stream_ptr(stream)))
