"""GPU: the state-vector engine (full FP64 states, Gram on the FP64 matrix
cores) against the FP64 state-vector oracle, and against the MPS path.

Both this engine and the oracle are FP64 end to end, so the bar against the
oracle is 1e-12 absolute on K (rounding of a 2^n-term FP64 sum, n <= 14
here); against the FP32 MPS sweep the parity bars of tests/gpu_helpers.py."""

import math

import numpy as np
import pytest

import oracle
from oracle import statevector
from paper_2405_02630_amd import qsvm, synth

from gpu_helpers import K_ABS_TOL, encode, log_close, require_gpu, to_dev

pytestmark = pytest.mark.gpu

SV_TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


def _states(X, reps):
    return qsvm.qsvm_encode_sv(to_dev(X), reps)


def _sym(X, reps, **kw):
    import torch

    s = _states(X, reps)
    K = torch.empty((s.N, s.N), dtype=torch.float64, device="cuda:0")
    L = torch.empty_like(K)
    qsvm.qsvm_sv_gram_sym(s, K, log_k=L, **kw)
    torch.cuda.synchronize()
    return K.cpu().numpy(), L.cpu().numpy()


@pytest.mark.parametrize("reps", [1, 2, 3, 4])
@pytest.mark.parametrize("n", [1, 2, 5, 10, 14])
def test_states_match_the_oracle(n, reps):
    X = synth.uniform_features(3, n, seed=5000 + 10 * n + reps)
    s = _states(X, reps).buf.cpu().numpy()
    for i in range(3):
        assert np.max(np.abs(s[i] - statevector.sv_state(X[i], reps))) < 1e-13


@pytest.mark.parametrize("reps", [1, 2, 3])
@pytest.mark.parametrize("n,N", [(1, 5), (3, 66), (8, 130), (12, 67)])
def test_sym_gram_vs_oracle(n, N, reps):
    X = synth.uniform_features(N, n, seed=5100 + n + reps)
    ref = statevector.sv_gram(X, reps)
    K, L = _sym(X, reps, diag_mode=1)
    assert np.max(np.abs(K - ref)) <= SV_TOL
    assert np.array_equal(K, K.T)
    assert np.max(np.abs(L - np.log(ref))) <= 1e-9
    K0, _ = _sym(X, reps)
    assert np.all(np.diag(K0) == 1.0)


def test_rect_gram_and_rows_vs_oracle():
    import torch

    Xa = synth.uniform_features(70, 9, seed=5200)
    Xb = synth.uniform_features(131, 9, seed=5201)
    ref = statevector.sv_gram_rect(Xa, Xb, 2)
    sa, sb = _states(Xa, 2), _states(Xb, 2)
    big = torch.full((70, 140), -3.0, dtype=torch.float64, device="cuda:0")
    K = big[:, :131]
    qsvm.qsvm_sv_gram(sa, sb, K, rows=(5, 69))
    torch.cuda.synchronize()
    b = big.cpu().numpy()
    assert np.all(b[:, 131:] == -3.0) and np.all(b[:5] == -3.0) and np.all(b[69:] == -3.0)
    assert np.max(np.abs(b[5:69, :131] - ref[5:69])) <= SV_TOL


def test_state_vector_and_mps_engines_agree_at_20_qubits():
    """The two GPU engines on 20 qubits, 96 points: the FP64 state-vector
    Gram against the FP32 MPS sweep, to the MPS path's parity bars."""
    import torch

    X = synth.uniform_features(96, 20, seed=5300)
    Ksv, Lsv = _sym(X, 2)
    m = encode(X, 2)
    Km = torch.empty((96, 96), dtype=torch.float64, device="cuda:0")
    Lm = torch.empty_like(Km)
    qsvm.qsvm_gram_sym(m, Km, log_k=Lm)
    torch.cuda.synchronize()
    Km, Lm = Km.cpu().numpy(), Lm.cpu().numpy()
    assert np.max(np.abs(Ksv - Km)) <= K_ABS_TOL
    off = ~np.eye(96, dtype=bool)
    assert log_close(oracle.log_k_errors(Lm[off], Lsv[off]))
    # and a few entries against the oracle itself
    pts = np.array([0, 17, 95])
    ref = statevector.sv_gram(X[pts], 2)
    assert np.max(np.abs(Ksv[np.ix_(pts, pts)] - ref)) <= SV_TOL


def test_near_duplicates_reach_the_diagonal():
    base = synth.uniform_features(4, 12, seed=5400)
    X = np.vstack([base, np.clip(base + 1e-4, 0, math.pi)])
    K, _ = _sym(X, 3, diag_mode=1)
    ref = statevector.sv_gram(X, 3)
    assert np.max(np.abs(K - ref)) <= SV_TOL
    assert min(K[i, i + 4] for i in range(4)) > 0.99


def test_maximum_qubits_entanglement_free():
    """n = 30 (the largest supported): two points, 2 x 2^30 FP64 amplitudes
    (34 GB), inner dimension 2^30 split across 1024 blocks; entanglement-free
    inputs against the product closed form."""
    import torch

    from oracle import closed_forms

    n = 30
    X = synth.pin_even_features(synth.uniform_features(2, n, seed=5500))
    s = _states(X, 2)
    K = torch.empty((2, 2), dtype=torch.float64, device="cuda:0")
    L = torch.empty_like(K)
    qsvm.qsvm_sv_gram_sym(s, K, log_k=L, diag_mode=1)
    torch.cuda.synchronize()
    Kh, Lh = K.cpu().numpy(), L.cpu().numpy()
    del s
    torch.cuda.empty_cache()
    ref = closed_forms.k_product_log(X[0], X[1], 2)
    assert abs(Lh[0, 1] - ref) <= 1e-9 * max(1.0, abs(ref))
    assert abs(Kh[0, 0] - 1.0) <= SV_TOL and abs(Kh[1, 1] - 1.0) <= SV_TOL


def test_empty_row_range_leaves_k_untouched():
    import torch

    X = synth.uniform_features(10, 6, seed=5600)
    s = _states(X, 2)
    K = torch.full((10, 10), -7.0, dtype=torch.float64, device="cuda:0")
    qsvm.qsvm_sv_gram_sym(s, K, rows=(4, 4))
    torch.cuda.synchronize()
    assert torch.all(K == -7.0)
