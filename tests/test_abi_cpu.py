"""The C-ABI library on a machine without a GPU: it loads, exports every
symbol include/qsvm.h declares, and rejects bad arguments on the host before
any HIP call (so every branch here runs with fake, never-dereferenced
pointers).  The injected launch failure shows the error path that a real
launch failure takes."""

import ctypes
import os
import re

import pytest

from paper_2405_02630_amd import qsvm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qsvm.h")

FAKE = ctypes.c_void_p(0x100000)  # 16-byte aligned, never dereferenced on these paths
FAKE2 = ctypes.c_void_p(0x200000)


@pytest.fixture(scope="module")
def lib():
    return qsvm.load_library()


@pytest.fixture
def no_inject(monkeypatch):
    monkeypatch.delenv("QSVM_FAULT_INJECT", raising=False)


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qsvm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_three_paper_calls():
    names = declared_functions()
    for f in ("qsvm_encode_mps", "qsvm_gram", "qsvm_gram_sym", "qsvm_mps_bytes"):
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_abi_version(lib):
    assert lib.qsvm_abi_version() == 2


def test_opts_struct_layout():
    # int32 x4, int64 x2, pointer, double, pointer x2: 64 bytes
    assert ctypes.sizeof(qsvm.GramOpts) == 64
    assert qsvm.GramOpts.log_k.offset == 32
    assert qsvm.GramOpts.refine_above.offset == 40
    assert qsvm.GramOpts.dense_a.offset == 48 and qsvm.GramOpts.dense_b.offset == 56


@pytest.mark.parametrize("N,n,reps", [(1, 1, 1), (32, 8, 2), (4096, 784, 2), (1024, 784, 3), (7, 3, 1), (1024, 784, 4),
                                     (1024, 784, 5), (9, 3, 6)])
def test_mps_bytes_formula(N, n, reps):
    # Sections G and L only (16 bytes each per site and point, any reps); the
    # dense tensors have their own buffer, written for reps <= 4 only
    chi = 2**reps
    assert qsvm.qsvm_mps_bytes(N, n, reps) == n * N * 32
    assert qsvm.qsvm_dense_bytes(N, n, reps) == (n * N * chi * chi * 8 if reps <= 4 else 0)


@pytest.mark.parametrize("N,n,reps", [(0, 8, 2), (8, 0, 2), (8, 8, 0), (8, 8, 7), (-1, 8, 2), (8, 65536, 2), (2**31, 8, 2)])
def test_mps_bytes_rejects(N, n, reps):
    assert qsvm.qsvm_mps_bytes(N, n, reps) == 0
    assert qsvm.qsvm_dense_bytes(N, n, reps) == 0


def test_encode_dense_validation(lib, no_inject):
    def enc(X=FAKE, N=8, n=4, reps=2, d=FAKE2, nbytes=None):
        nbytes = max(qsvm.qsvm_dense_bytes(N, n, reps), 1) if nbytes is None else nbytes
        return lib.qsvm_encode_dense(X, N, n, reps, d, nbytes, None)

    assert enc(X=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert enc(d=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert enc(d=ctypes.c_void_p(0x100008)) == qsvm.QSVM_ERR_INVALID_ARG
    assert enc(reps=5) == qsvm.QSVM_ERR_UNSUPPORTED  # dense tensors up to reps 4
    assert b"reps <= 4" in lib.qsvm_last_error()
    assert enc(reps=7) == qsvm.QSVM_ERR_UNSUPPORTED
    assert enc(nbytes=qsvm.qsvm_dense_bytes(8, 4, 2) - 1) == qsvm.QSVM_ERR_SIZE


def test_dense_sweep_needs_dense_tensors(lib, no_inject):
    o = qsvm.GramOpts()
    o.sweep = qsvm.SWEEP_DENSE
    assert _sym(lib, opts=o) == qsvm.QSVM_ERR_INVALID_ARG
    assert b"dense_a" in lib.qsvm_last_error()
    assert _rect(lib, opts=o) == qsvm.QSVM_ERR_INVALID_ARG
    o.dense_a = 0x300008  # misaligned
    assert _sym(lib, opts=o) == qsvm.QSVM_ERR_INVALID_ARG
    o.dense_a = 0x300000
    os.environ["QSVM_FAULT_INJECT"] = "launch"
    try:
        assert _sym(lib, opts=o) == qsvm.QSVM_ERR_HIP  # accepted: dense_b defaults to dense_a
        assert _rect(lib, opts=o) == qsvm.QSVM_ERR_HIP
    finally:
        del os.environ["QSVM_FAULT_INJECT"]
    # the butterfly sweep needs no dense tensors
    os.environ["QSVM_FAULT_INJECT"] = "launch"
    try:
        assert _sym(lib, opts=qsvm.GramOpts()) == qsvm.QSVM_ERR_HIP
    finally:
        del os.environ["QSVM_FAULT_INJECT"]


def test_status_strings(lib):
    for s in (0, -1, -2, -3, -4):
        assert lib.qsvm_status_string(s).startswith(b"QSVM_")
    assert lib.qsvm_status_string(17) == b"unknown qsvm_status"


def _enc(lib, X=FAKE, N=8, n=4, reps=2, mps=FAKE2, nbytes=None):
    if nbytes is None:
        nbytes = max(qsvm.qsvm_mps_bytes(N, n, reps), 1)
    return lib.qsvm_encode_mps(X, N, n, reps, mps, nbytes, None)


def test_encode_validation(lib, no_inject):
    assert _enc(lib, X=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert _enc(lib, mps=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert _enc(lib, N=0) == qsvm.QSVM_ERR_INVALID_ARG
    assert _enc(lib, n=0) == qsvm.QSVM_ERR_INVALID_ARG
    assert _enc(lib, n=70000) == qsvm.QSVM_ERR_INVALID_ARG
    assert _enc(lib, reps=0) == qsvm.QSVM_ERR_INVALID_ARG
    assert _enc(lib, reps=7) == qsvm.QSVM_ERR_UNSUPPORTED
    assert b"reps = 7" in lib.qsvm_last_error()
    assert _enc(lib, mps=ctypes.c_void_p(0x100008)) == qsvm.QSVM_ERR_INVALID_ARG  # misaligned
    assert _enc(lib, X=ctypes.c_void_p(0x100004)) == qsvm.QSVM_ERR_INVALID_ARG
    need = qsvm.qsvm_mps_bytes(8, 4, 2)
    assert _enc(lib, nbytes=need - 1) == qsvm.QSVM_ERR_SIZE


def _sym(lib, mps=FAKE, N=100, n=8, reps=2, K=FAKE2, ldk=None, opts=None):
    ldk = N if ldk is None else ldk
    return lib.qsvm_gram_sym(mps, N, n, reps, K, ldk, ctypes.byref(opts) if opts is not None else None, None)


def _rect(lib, a=FAKE, Na=50, b=FAKE2, Nb=70, n=8, reps=2, K=FAKE2, ldk=None, opts=None):
    ldk = Nb if ldk is None else ldk
    return lib.qsvm_gram(a, Na, b, Nb, n, reps, K, ldk, ctypes.byref(opts) if opts is not None else None, None)


def test_gram_sym_validation(lib, no_inject):
    assert _sym(lib, mps=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert _sym(lib, K=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert _sym(lib, N=0) == qsvm.QSVM_ERR_INVALID_ARG
    assert _sym(lib, n=0) == qsvm.QSVM_ERR_INVALID_ARG
    assert _sym(lib, reps=7) == qsvm.QSVM_ERR_UNSUPPORTED
    assert _sym(lib, ldk=99) == qsvm.QSVM_ERR_INVALID_ARG
    assert _sym(lib, mps=ctypes.c_void_p(0x100004)) == qsvm.QSVM_ERR_INVALID_ARG


def _sym_noalloc(lib, N=100, n=784, reps=2, ldk=None, opts=None, mps=FAKE, K=FAKE2):
    ldk = N if ldk is None else ldk
    return lib.qsvm_gram_sym_noalloc(mps, N, n, reps, K, ldk, ctypes.byref(opts) if opts is not None else None, None)


def _tiles_upper(N):
    T = -(-N // 64)
    return T * (T + 1) // 2


def test_gram_sym_noalloc_validation(lib, no_inject):
    assert _sym_noalloc(lib, mps=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert _sym_noalloc(lib, K=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert _sym_noalloc(lib, ldk=99) == qsvm.QSVM_ERR_INVALID_ARG
    assert _sym_noalloc(lib, reps=7) == qsvm.QSVM_ERR_UNSUPPORTED
    # the refinement's list needs one entry per tile plus the count: the
    # largest N whose upper triangle fits the static array, and the next one
    # that does not, are told apart before any HIP call
    cap = qsvm.NOALLOC_SCRATCH_ENTRIES
    N_ok = max(N for N in range(64, 200000, 64) if _tiles_upper(N) + 1 <= cap)
    assert _tiles_upper(N_ok + 64) + 1 > cap
    assert _sym_noalloc(lib, N=N_ok + 1) == qsvm.QSVM_ERR_SIZE
    assert b"static workspace" in lib.qsvm_last_error()
    # a row range narrows the tiles the call needs
    o = qsvm.GramOpts()
    o.row_begin, o.row_end = 0, 64
    os.environ["QSVM_FAULT_INJECT"] = "launch"
    try:
        assert _sym_noalloc(lib, N=N_ok + 1, opts=o) == qsvm.QSVM_ERR_HIP
        assert _sym_noalloc(lib, N=N_ok) == qsvm.QSVM_ERR_HIP  # passes validation
        # refinement off: no workspace, no size limit
        o2 = qsvm.GramOpts()
        o2.refine_above = -1.0
        assert _sym_noalloc(lib, N=4 * N_ok, opts=o2) == qsvm.QSVM_ERR_HIP
        # at n <= 50 the automatic threshold switches the refinement off
        assert _sym_noalloc(lib, N=4 * N_ok, n=50) == qsvm.QSVM_ERR_HIP
    finally:
        del os.environ["QSVM_FAULT_INJECT"]
    assert _sym_noalloc(lib, N=4 * N_ok, n=51) == qsvm.QSVM_ERR_SIZE


def test_gram_rect_validation(lib, no_inject):
    assert _rect(lib, a=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert _rect(lib, b=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert _rect(lib, K=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert _rect(lib, Na=0) == qsvm.QSVM_ERR_INVALID_ARG
    assert _rect(lib, Nb=-3) == qsvm.QSVM_ERR_INVALID_ARG
    assert _rect(lib, ldk=69) == qsvm.QSVM_ERR_INVALID_ARG
    assert _rect(lib, reps=7) == qsvm.QSVM_ERR_UNSUPPORTED


# One row of 64 x 64 tiles must fit one launch of at most 2^24 - 8 blocks:
# 16 blocks per tile (1048575 tiles, 67108800 points), 32 at reps = 4
# (524287 tiles), 128 at reps = 5 (131071 tiles), 512 at reps = 6 (32767
# tiles).  Validation fails before any HIP call.
@pytest.mark.parametrize("reps,nb_max", [(2, 64 * 1048575), (4, 64 * 524287), (5, 64 * 131071), (6, 64 * 32767)])
def test_gram_rejects_a_tile_row_wider_than_one_launch(lib, no_inject, reps, nb_max):
    opts = qsvm.GramOpts()
    opts.row_begin, opts.row_end = 5, 5  # empty range: a valid Nb returns before launching
    assert _rect(lib, Na=64, Nb=nb_max, n=4, reps=reps, opts=opts) == qsvm.QSVM_OK
    assert _rect(lib, Na=64, Nb=nb_max + 1, n=4, reps=reps, opts=opts) == qsvm.QSVM_ERR_UNSUPPORTED
    assert b"exceeds one launch" in lib.qsvm_last_error()


@pytest.mark.parametrize("n,expect", [(1, None), (50, None), (51, 0.992), (64, 0.897), (784, 0.0645), (65535, 1.4464e-5)])
def test_auto_refine_threshold(n, expect):
    # (5e-6 / (4e-6 + 2e-8 n))^2: >= 1 (no refinement) up to 50 qubits
    t = qsvm.qsvm_auto_refine_threshold(n)
    if expect is None:
        assert t >= 1.0
    else:
        assert t == pytest.approx(expect, rel=2e-3)
    assert qsvm.qsvm_auto_refine_threshold(0) == 0.0


def test_refine_above_nan_is_rejected(lib, no_inject):
    o = qsvm.GramOpts()
    o.refine_above = float("nan")
    assert _sym(lib, opts=o) == qsvm.QSVM_ERR_INVALID_ARG
    assert _rect(lib, opts=o) == qsvm.QSVM_ERR_INVALID_ARG
    assert b"refine_above" in lib.qsvm_last_error()
    b = qsvm.BatchOpts()
    b.refine_above = float("nan")
    st, h = _plan(lib, [_job()], b)
    assert st == qsvm.QSVM_ERR_INVALID_ARG and not h.value


def test_dense_sweep_rejects_reps_4(lib, no_inject):
    opts = qsvm.GramOpts()
    opts.sweep = qsvm.SWEEP_DENSE
    opts.dense_a = 0x300000
    assert _sym(lib, reps=4, opts=opts) == qsvm.QSVM_ERR_UNSUPPORTED
    assert b"dense sweep" in lib.qsvm_last_error()
    assert _rect(lib, reps=4, opts=opts) == qsvm.QSVM_ERR_UNSUPPORTED


def _tiles(lib, dev, mps=FAKE, N=150, n=8, reps=2, tiles=FAKE2, count=FAKE, n_tiles=3, K=FAKE2, ldk=None,
           opts=None):
    ldk = N if ldk is None else ldk
    if dev:
        return lib.qsvm_gram_sym_tiles_dev(mps, N, n, reps, tiles, count, n_tiles, K, ldk, opts, None)
    return lib.qsvm_gram_sym_tiles(mps, N, n, reps, tiles, n_tiles, K, ldk, opts, None)


@pytest.mark.parametrize("dev", [False, True])
def test_tile_list_validation(lib, no_inject, dev):
    bad = qsvm.QSVM_ERR_INVALID_ARG
    assert _tiles(lib, dev, mps=None) == bad
    assert _tiles(lib, dev, tiles=None) == bad
    assert _tiles(lib, dev, K=None) == bad
    assert _tiles(lib, dev, ldk=149) == bad
    assert _tiles(lib, dev, mps=ctypes.c_void_p(0x100008)) == bad
    assert _tiles(lib, dev, n_tiles=-1) == bad
    assert _tiles(lib, dev, n_tiles=7) == bad  # 150 points: 3 tile rows, 6 upper-triangular tiles
    o = qsvm.GramOpts()
    o.row_begin, o.row_end = 0, 64
    assert _tiles(lib, dev, opts=o) == bad
    assert b"row ranges" in lib.qsvm_last_error()
    assert _tiles(lib, dev, reps=7) == qsvm.QSVM_ERR_UNSUPPORTED
    assert _tiles(lib, dev, n_tiles=0) == qsvm.QSVM_OK  # nothing to launch
    assert _tiles(lib, dev, N=(1 << 31) - 1, n_tiles=1 << 31) == qsvm.QSVM_ERR_UNSUPPORTED


def test_tile_list_with_device_count_validation(lib, no_inject):
    assert _tiles(lib, True, count=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert b"tile_count" in lib.qsvm_last_error()
    assert _tiles(lib, True, reps=4) == qsvm.QSVM_ERR_UNSUPPORTED
    assert b"butterfly" in lib.qsvm_last_error()
    o = qsvm.GramOpts()
    o.sweep = qsvm.SWEEP_DENSE
    o.dense_a = 0x300000
    assert _tiles(lib, True, opts=o) == qsvm.QSVM_ERR_UNSUPPORTED
    # a list too long for the refinement's one-launch scan of a device count
    assert _tiles(lib, True, N=370752, n_tiles=1 << 24) == qsvm.QSVM_ERR_UNSUPPORTED
    assert _tiles(lib, True, N=370752, n_tiles=0) == qsvm.QSVM_OK


@pytest.mark.parametrize(
    "field,value",
    [("renorm_every", -1), ("renorm_every", 17), ("sweep", 3), ("sweep", -1), ("diag_mode", 2), ("variant", 5), ("variant", -1)],
)
def test_gram_opts_validation(lib, no_inject, field, value):
    o = qsvm.GramOpts()
    setattr(o, field, value)
    assert _sym(lib, opts=o) == qsvm.QSVM_ERR_INVALID_ARG
    assert _rect(lib, opts=o) == qsvm.QSVM_ERR_INVALID_ARG


@pytest.mark.parametrize("rb,re_", [(-1, 5), (5, 4), (0, 101), (10, 200)])
def test_gram_row_range_validation(lib, no_inject, rb, re_):
    o = qsvm.GramOpts()
    o.row_begin, o.row_end = rb, re_
    assert _sym(lib, N=100, opts=o) == qsvm.QSVM_ERR_INVALID_ARG


def test_empty_row_range_is_a_no_op(lib, no_inject):
    # an empty range returns OK without launching (pointers are fake)
    o = qsvm.GramOpts()
    o.row_begin, o.row_end = 7, 7
    assert _sym(lib, N=100, opts=o) == qsvm.QSVM_OK
    assert _rect(lib, Na=50, opts=o) == qsvm.QSVM_OK


def test_injected_launch_failure(lib, monkeypatch):
    monkeypatch.setenv("QSVM_FAULT_INJECT", "launch")
    assert _enc(lib) == qsvm.QSVM_ERR_HIP
    assert b"injected" in lib.qsvm_last_error()
    assert _sym(lib) == qsvm.QSVM_ERR_HIP
    assert _rect(lib) == qsvm.QSVM_ERR_HIP
    # validation still comes first
    assert _sym(lib, N=0) == qsvm.QSVM_ERR_INVALID_ARG


def test_python_binding_raises_with_the_library_message(monkeypatch):
    monkeypatch.setenv("QSVM_FAULT_INJECT", "launch")
    with pytest.raises(qsvm.QsvmError) as ei:
        qsvm._check(qsvm.load_library().qsvm_gram_sym(FAKE, 8, 8, 2, FAKE2, 8, None, None))
    assert ei.value.status == qsvm.QSVM_ERR_HIP
    assert "injected" in str(ei.value)


def test_missing_library_raises(tmp_path):
    saved = qsvm._lib
    try:
        qsvm._lib = None
        with pytest.raises(RuntimeError, match="no fallback"):
            qsvm.load_library(str(tmp_path / "libqsvm.so"))
    finally:
        qsvm._lib = saved


# --------------------------------------------------------------------------
# Batched plans: validation happens before any HIP call
# --------------------------------------------------------------------------

def _job(mps=0x100000, N=100, n=8, reps=2, K=0x200000, ldk=100, log_k=None):
    j = qsvm.Job()
    j.mps, j.N, j.n_qubits, j.reps, j.K, j.ldk, j.log_k = mps, N, n, reps, K, ldk, log_k
    return j


def _plan(lib, jobs, opts=None):
    arr = (qsvm.Job * len(jobs))(*jobs)
    h = ctypes.c_void_p()
    st = lib.qsvm_batch_plan_create(arr, len(jobs), ctypes.byref(opts) if opts else None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize(
    "kw",
    [dict(mps=None), dict(K=None), dict(N=0), dict(n=0), dict(reps=0), dict(ldk=99), dict(mps=0x100008)],
)
def test_batch_plan_rejects_bad_job(lib, no_inject, kw):
    st, h = _plan(lib, [_job(), _job(**kw)])
    assert st == qsvm.QSVM_ERR_INVALID_ARG and not h.value
    assert b"job 1" in lib.qsvm_last_error()


def test_batch_plan_unsupported_reps(lib, no_inject):
    st, h = _plan(lib, [_job(reps=4)])
    assert st == qsvm.QSVM_ERR_UNSUPPORTED and not h.value


@pytest.mark.parametrize(
    "field,value",
    [("renorm_every", 17), ("diag_mode", 3), ("use_graph", 2), ("grid_blocks", -1), ("grid_blocks", 1 << 24)],
)
def test_batch_plan_rejects_bad_opts(lib, no_inject, field, value):
    o = qsvm.BatchOpts()
    setattr(o, field, value)
    st, _ = _plan(lib, [_job()], o)
    assert st == qsvm.QSVM_ERR_INVALID_ARG


def test_batch_plan_null_arguments(lib, no_inject):
    assert lib.qsvm_batch_plan_create(None, 0, None, None) == qsvm.QSVM_ERR_INVALID_ARG
    h = ctypes.c_void_p()
    assert lib.qsvm_batch_plan_create(None, 3, None, ctypes.byref(h)) == qsvm.QSVM_ERR_INVALID_ARG
    assert lib.qsvm_batch_plan_launch(None, None) == qsvm.QSVM_ERR_INVALID_ARG
    assert lib.qsvm_batch_plan_info(None, None, None, None) == qsvm.QSVM_ERR_INVALID_ARG
    assert lib.qsvm_batch_plan_destroy(None) == qsvm.QSVM_OK


def test_batch_plan_injected_failure(lib, monkeypatch):
    monkeypatch.setenv("QSVM_FAULT_INJECT", "launch")
    st, h = _plan(lib, [_job(), _job(reps=3, n=5)])
    assert st == qsvm.QSVM_ERR_HIP and not h.value


def test_tuned_variant_table(lib, no_inject):
    assert lib.qsvm_set_tuned_variant(2, 300, 1000, 4) == qsvm.QSVM_ERR_INVALID_ARG
    assert lib.qsvm_set_tuned_variant(7, 300, 1000, 1) == qsvm.QSVM_ERR_UNSUPPORTED
    assert lib.qsvm_set_tuned_variant(2, 300, 0, 1) == qsvm.QSVM_ERR_INVALID_ARG
    assert lib.qsvm_set_tuned_variant(2, 300, 1000, 3) == qsvm.QSVM_OK
    assert lib.qsvm_get_tuned_variant(2, 300, 1000) == 3
    assert lib.qsvm_get_tuned_variant(2, 511, 600) == 3  # same log2 buckets (n 8, N 9)
    assert lib.qsvm_get_tuned_variant(2, 512, 1000) == 0  # untuned n bucket -> default
    # other N buckets of the same n bucket: only the tuned buckets answer
    assert lib.qsvm_set_tuned_variant(2, 300, 8192, 1) == qsvm.QSVM_OK
    assert lib.qsvm_get_tuned_variant(2, 300, 9000) == 1     # bucket 13
    assert lib.qsvm_get_tuned_variant(2, 300, 100) == 0      # bucket 6: untuned -> default
    assert lib.qsvm_get_tuned_variant(2, 300, 5000) == 0     # bucket 12: untuned -> default
    assert lib.qsvm_get_tuned_variant(2, 300, 1 << 20) == 0
    for N in (1000, 8192):
        assert lib.qsvm_set_tuned_variant(2, 300, N, 0) == qsvm.QSVM_OK


@pytest.mark.parametrize("field,value", [("item_pi2", 3), ("item_pi2", 1), ("item_pi3", 2), ("item_pi3", -1)])
def test_batch_plan_rejects_bad_item_shape(lib, no_inject, field, value):
    o = qsvm.BatchOpts()
    setattr(o, field, value)
    st, _ = _plan(lib, [_job()], o)
    assert st == qsvm.QSVM_ERR_INVALID_ARG
    assert b"item_pi" in lib.qsvm_last_error()


def _run_py(code, env):
    import subprocess
    import sys

    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    return r.stdout.strip()


def test_tune_cache_persists_across_processes(tmp_path):
    # without a GPU the architecture key is "unknown"; the file format and the
    # merge of entries across processes are what is checked here
    path = tmp_path / "sub" / "tune.txt"
    env = dict(os.environ, QSVM_TUNE_CACHE=str(path))
    env.pop("QSVM_FAULT_INJECT", None)
    pre = "from paper_2405_02630_amd import qsvm; "
    _run_py(pre + "qsvm.qsvm_set_tuned_variant(3, 784, 4096, 2); qsvm.qsvm_autotune_save(); "
                  "print(qsvm.qsvm_autotune_cache_path())", env)
    lines = [ln for ln in path.read_text().splitlines() if not ln.startswith("#")]
    assert lines == ["unknown 3 9 12 2"]
    out = _run_py(pre + "print(qsvm.qsvm_get_tuned_variant(3, 784, 4096), qsvm.qsvm_get_tuned_variant(3, 1100, 4096), "
                        "qsvm.qsvm_get_tuned_variant(2, 784, 4096)); qsvm.qsvm_set_tuned_variant(2, 64, 100, 1); "
                        "qsvm.qsvm_autotune_save()", env)
    assert out == "2 0 0"  # 1100 qubits is in another log2 bucket
    lines = sorted(ln for ln in path.read_text().splitlines() if not ln.startswith("#"))
    assert lines == ["unknown 2 6 6 1", "unknown 3 9 12 2"]  # merged, not overwritten
    # malformed lines are skipped
    path.write_text(path.read_text() + "garbage line\nunknown 2 6\nunknown 9 1 1 1\n")
    assert _run_py(pre + "print(qsvm.qsvm_get_tuned_variant(2, 64, 100))", env) == "1"
    # an empty QSVM_TUNE_CACHE switches persistence off
    env["QSVM_TUNE_CACHE"] = ""
    assert _run_py(pre + "print(repr(qsvm.qsvm_autotune_cache_path()), qsvm.qsvm_get_tuned_variant(3, 784, 4096))",
                   env) == "'' 0"


def test_autotune_validation(lib, no_inject):
    ms = (ctypes.c_float * 2)()
    assert lib.qsvm_autotune(7, 10, 100, None, None, None, 0) == qsvm.QSVM_ERR_UNSUPPORTED
    assert lib.qsvm_autotune(2, 10, 70000, None, None, None, 0) == qsvm.QSVM_ERR_INVALID_ARG
    assert lib.qsvm_autotune(2, 10, 100, None, None, ms, 2) == qsvm.QSVM_ERR_SIZE


# --------------------------------------------------------------------------
# State-vector engine
# --------------------------------------------------------------------------

@pytest.mark.parametrize("N,n", [(1, 1), (32, 8), (1024, 20), (3, 30)])
def test_sv_bytes_formula(N, n):
    assert qsvm.qsvm_sv_bytes(N, n) == N * 2**n * 16


@pytest.mark.parametrize("N,n", [(0, 8), (-1, 8), (8, 0), (8, 31), (2**40, 30)])
def test_sv_bytes_rejects(N, n):
    assert qsvm.qsvm_sv_bytes(N, n) == 0


def test_encode_sv_validation(lib, no_inject):
    nb = qsvm.qsvm_sv_bytes(8, 4)
    assert lib.qsvm_encode_sv(FAKE, 8, 31, 2, FAKE2, nb, None) == qsvm.QSVM_ERR_UNSUPPORTED
    assert lib.qsvm_encode_sv(FAKE, 8, 4, 0, FAKE2, nb, None) == qsvm.QSVM_ERR_INVALID_ARG
    assert lib.qsvm_encode_sv(FAKE, 8, 4, 17, FAKE2, nb, None) == qsvm.QSVM_ERR_INVALID_ARG
    assert lib.qsvm_encode_sv(FAKE, 0, 4, 2, FAKE2, nb, None) == qsvm.QSVM_ERR_INVALID_ARG
    assert lib.qsvm_encode_sv(None, 8, 4, 2, FAKE2, nb, None) == qsvm.QSVM_ERR_INVALID_ARG
    assert lib.qsvm_encode_sv(FAKE, 8, 4, 2, None, nb, None) == qsvm.QSVM_ERR_INVALID_ARG
    assert lib.qsvm_encode_sv(FAKE, 8, 4, 2, ctypes.c_void_p(0x200008), nb, None) == qsvm.QSVM_ERR_INVALID_ARG
    assert lib.qsvm_encode_sv(FAKE, 8, 4, 2, FAKE2, nb - 1, None) == qsvm.QSVM_ERR_SIZE


def test_sv_gram_validation(lib, no_inject):
    o = qsvm.GramOpts()
    assert lib.qsvm_sv_gram(None, 5, FAKE2, 7, 4, FAKE, 7, None, None) == qsvm.QSVM_ERR_INVALID_ARG
    assert lib.qsvm_sv_gram(FAKE, 5, FAKE2, 7, 4, None, 7, None, None) == qsvm.QSVM_ERR_INVALID_ARG
    assert lib.qsvm_sv_gram(FAKE, 5, FAKE2, 7, 31, FAKE, 7, None, None) == qsvm.QSVM_ERR_UNSUPPORTED
    assert lib.qsvm_sv_gram(FAKE, 5, FAKE2, 7, 4, FAKE, 6, None, None) == qsvm.QSVM_ERR_INVALID_ARG
    assert lib.qsvm_sv_gram(FAKE, 0, FAKE2, 7, 4, FAKE, 7, None, None) == qsvm.QSVM_ERR_INVALID_ARG
    assert lib.qsvm_sv_gram(ctypes.c_void_p(0x100008), 5, FAKE2, 7, 4, FAKE, 7, None, None) == qsvm.QSVM_ERR_INVALID_ARG
    o.row_begin, o.row_end = 3, 9
    assert lib.qsvm_sv_gram_sym(FAKE, 5, 4, FAKE2, 5, ctypes.byref(o), None) == qsvm.QSVM_ERR_INVALID_ARG
    o.row_begin, o.row_end = 2, 2  # empty range: nothing to do
    assert lib.qsvm_sv_gram_sym(FAKE, 5, 4, FAKE2, 5, ctypes.byref(o), None) == qsvm.QSVM_OK
    o = qsvm.GramOpts()
    o.diag_mode = 2
    assert lib.qsvm_sv_gram_sym(FAKE, 5, 4, FAKE2, 5, ctypes.byref(o), None) == qsvm.QSVM_ERR_INVALID_ARG


def test_sv_gram_rejects_a_tile_row_wider_than_one_launch(lib, no_inject):
    # one block per 64 x 64 tile: at most 2^24 - 8 tiles, 64 (2^24 - 8) points, in a row
    o = qsvm.GramOpts()
    o.row_begin, o.row_end = 2, 2
    nb = 64 * ((1 << 24) - 8)
    assert lib.qsvm_sv_gram(FAKE, 5, FAKE2, nb, 1, FAKE, nb, ctypes.byref(o), None) == qsvm.QSVM_OK
    assert lib.qsvm_sv_gram(FAKE, 5, FAKE2, nb + 1, 1, FAKE, nb + 1, ctypes.byref(o), None) == qsvm.QSVM_ERR_UNSUPPORTED
    assert b"exceeds one launch" in lib.qsvm_last_error()


def test_sv_injected_launch_failure(lib, monkeypatch):
    monkeypatch.setenv("QSVM_FAULT_INJECT", "launch")
    nb = qsvm.qsvm_sv_bytes(8, 4)
    assert lib.qsvm_encode_sv(FAKE, 8, 4, 2, FAKE2, nb, None) == qsvm.QSVM_ERR_HIP
    assert lib.qsvm_sv_gram_sym(FAKE, 8, 4, FAKE2, 8, None, None) == qsvm.QSVM_ERR_HIP
    assert b"injected" in lib.qsvm_last_error()


def _net():
    return qsvm.Mlp(832, 512, 512, 256, 0x100000, 0x110000, 0x120000, 0x130000, 0x140000, 0x150000)


def test_mlp_forward_validation(lib, no_inject):
    net = _net()
    full = qsvm.MlpActs(0x200000, 0x210000, 0x220000, 0x230000, 0x240000, 0x250000)
    part = qsvm.MlpActs(0x200000, 0x210000, None, 0x230000, 0x240000, 0x250000)  # H2 missing
    infer = qsvm.MlpActs(None, 0x210000, None, 0x230000, None, 0x250000)
    nobf16 = qsvm.MlpActs(0x200000, None, 0x220000, 0x230000, 0x240000, 0x250000)
    f = lib.qsvm_mlp_forward
    assert f(None, FAKE, 64, ctypes.byref(full), None) == qsvm.QSVM_ERR_INVALID_ARG
    assert f(ctypes.byref(net), FAKE, 100, ctypes.byref(full), None) == qsvm.QSVM_ERR_INVALID_ARG  # rows % 64
    assert f(ctypes.byref(net), FAKE, 64, ctypes.byref(part), None) == qsvm.QSVM_ERR_INVALID_ARG
    assert b"all given or all NULL" in lib.qsvm_last_error()
    assert f(ctypes.byref(net), FAKE, 64, ctypes.byref(nobf16), None) == qsvm.QSVM_ERR_INVALID_ARG
    os.environ["QSVM_FAULT_INJECT"] = "launch"
    try:  # both forms pass validation
        assert f(ctypes.byref(net), FAKE, 64, ctypes.byref(full), None) == qsvm.QSVM_ERR_HIP
        assert f(ctypes.byref(net), FAKE, 64, ctypes.byref(infer), None) == qsvm.QSVM_ERR_HIP
    finally:
        del os.environ["QSVM_FAULT_INJECT"]


def _roctx_probe(env_value):
    """In a fresh process: one entry-point call that fails validation, then
    whether the marker library is mapped."""
    import subprocess
    import sys

    code = (
        "import ctypes\n"
        "from paper_2405_02630_amd import qsvm\n"
        "lib = qsvm.load_library()\n"
        "st = lib.qsvm_gram_sym(None, 100, 8, 2, ctypes.c_void_p(0x200000), 100, None, None)\n"
        "maps = open('/proc/self/maps').read()\n"
        "print(st, 'rocprofiler-sdk-roctx' in maps)\n"
    )
    env = dict(os.environ)
    env.pop("QSVM_ROCTX", None)
    if env_value is not None:
        env["QSVM_ROCTX"] = env_value
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    return r.stdout.split()


def test_roctx_ranges_are_opt_in():
    # QSVM_ROCTX=1: the marker library is opened on the first entry-point call
    # (the call itself behaves as without it); otherwise it is never loaded
    st, mapped = _roctx_probe("1")
    assert int(st) == qsvm.QSVM_ERR_INVALID_ARG and mapped == "True"
    st, mapped = _roctx_probe(None)
    assert int(st) == qsvm.QSVM_ERR_INVALID_ARG and mapped == "False"
    st, mapped = _roctx_probe("0")
    assert mapped == "False"


def test_pair_fallback_validation(lib, no_inject):
    o = qsvm.GramOpts()

    def pairs_dev(mps=FAKE, N=100, n=8, reps=2, pairs=FAKE2, count=FAKE2, maxp=10, K=FAKE2, ldk=100, opts=None):
        return lib.qsvm_gram_sym_pairs_dev(mps, N, n, reps, pairs, count, maxp, K, ldk,
                                           ctypes.byref(opts) if opts is not None else None, None)

    assert pairs_dev(mps=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert pairs_dev(pairs=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert pairs_dev(count=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert pairs_dev(ldk=99) == qsvm.QSVM_ERR_INVALID_ARG
    assert pairs_dev(maxp=-1) == qsvm.QSVM_ERR_INVALID_ARG
    assert pairs_dev(reps=7) == qsvm.QSVM_ERR_UNSUPPORTED
    assert pairs_dev(mps=ctypes.c_void_p(0x100008)) == qsvm.QSVM_ERR_INVALID_ARG
    o.row_begin, o.row_end = 0, 50
    assert pairs_dev(opts=o) == qsvm.QSVM_ERR_INVALID_ARG
    assert pairs_dev(maxp=0) == qsvm.QSVM_OK  # nothing to do, nothing launched

    def flag(K=FAKE, N=100, ldk=100, tiles=FAKE2, tcount=FAKE2, maxt=10, cut=1e-6, cap=64, pairs=FAKE2,
             pcount=FAKE2, maxp=100, dense=FAKE2, dcount=FAKE2):
        return lib.qsvm_flag_pairs(K, N, ldk, tiles, tcount, maxt, cut, cap, pairs, pcount, maxp, dense, dcount, None)

    assert flag(K=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert flag(dense=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert flag(N=0) == qsvm.QSVM_ERR_INVALID_ARG
    assert flag(ldk=50) == qsvm.QSVM_ERR_INVALID_ARG
    assert flag(cap=4097) == qsvm.QSVM_ERR_INVALID_ARG
    assert flag(maxt=1 << 20, cap=4096) == qsvm.QSVM_ERR_INVALID_ARG  # reservations could pass 2^31
    assert flag(maxp=-1) == qsvm.QSVM_ERR_INVALID_ARG


def test_surrogate_gram_log_validation(lib, no_inject):
    head = FAKE2

    def gram(X16=FAKE, d_in=832, E16=FAKE, d=256, N=100, N_pad=128, K=FAKE2, ldk=100, tmax=FAKE2):
        return lib.qsvm_surrogate_gram_log(X16, d_in, E16, d, N, N_pad, head, K, ldk, tmax, None)

    assert gram(E16=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert gram(K=None) == qsvm.QSVM_ERR_INVALID_ARG
    assert gram(X16=None) == qsvm.QSVM_ERR_INVALID_ARG  # an input part needs its rows
    assert gram(N_pad=96) == qsvm.QSVM_ERR_INVALID_ARG  # N_pad % 64
    assert gram(N_pad=192) == qsvm.QSVM_ERR_INVALID_ARG  # N_pad >= N + 64
    assert gram(d_in=48) == qsvm.QSVM_ERR_INVALID_ARG
    assert gram(d=16) == qsvm.QSVM_ERR_INVALID_ARG
    assert gram(ldk=99) == qsvm.QSVM_ERR_INVALID_ARG
    big = (1 << 19) + 64  # one block per 128 x 128 piece of the upper triangle: N_pad <= 2^19
    assert gram(N=big, N_pad=big, ldk=big) == qsvm.QSVM_ERR_UNSUPPORTED
    os.environ["QSVM_FAULT_INJECT"] = "launch"
    try:  # valid arguments, without and with the input part, reach the launch
        assert gram() == qsvm.QSVM_ERR_HIP
        assert gram(X16=None, d_in=0) == qsvm.QSVM_ERR_HIP
        assert gram(N=1 << 19, N_pad=1 << 19, ldk=1 << 19) == qsvm.QSVM_ERR_HIP
    finally:
        del os.environ["QSVM_FAULT_INJECT"]
