"""GPU test of qsvm_gram_sym_noalloc, the symmetric Gram that allocates no
device memory (the FP64 refinement's tile list lives in a static per-device
array).  Two calls in a row, the second on a smaller input, are checked
against qsvm_gram_sym on the same inputs (bit for bit: the same kernels run)
and, where the refinement must have run through the static list, against the
FP64 MPS oracle.  The inputs are 784-qubit images with near-duplicate copies,
so tiles hold entries near 1 and the refinement lists them."""

import numpy as np
import pytest

from oracle import mps as omps
from paper_2405_02630_amd import qsvm, synth

from gpu_helpers import K_ABS_TOL, encode, require_gpu

pytestmark = pytest.mark.gpu

REFINED_TOL = 1e-9


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


def _near_duplicate_set(seed, n_base):
    base, Xp, idx, eps = synth.image_near_duplicates(seed=seed, n_base=n_base)
    X = np.concatenate([base, Xp])
    # pair (base row b, its copy at row n_base + r) for every perturbed row r
    pairs = np.stack([idx, n_base + np.arange(Xp.shape[0])], axis=1)
    return X, pairs


def _noalloc(m, diag_mode):
    import torch

    K = torch.full((m.N, m.N), -7.0, dtype=torch.float64, device="cuda:0")
    L = torch.full_like(K, -7.0)
    qsvm.qsvm_gram_sym_noalloc(m, K, log_k=L, diag_mode=diag_mode)
    return K, L


def test_noalloc_matches_gram_sym_on_two_calls_second_smaller():
    import torch

    X1, pairs1 = _near_duplicate_set(seed=51, n_base=40)   # 240 points: 4 tile rows, 10 tiles
    X2, pairs2 = _near_duplicate_set(seed=52, n_base=16)   # 96 points: 2 tile rows, 3 tiles
    print(f"noalloc: n=784 reps=2 N={X1.shape[0]} then N={X2.shape[0]}", flush=True)
    m1, m2 = encode(X1, 2), encode(X2, 2)
    K1, L1 = _noalloc(m1, diag_mode=1)
    K2, L2 = _noalloc(m2, diag_mode=1)
    R1 = qsvm.qsvm_gram_sym(m1, diag_mode=1, log_k=(Lr1 := torch.empty((m1.N, m1.N), dtype=torch.float64, device="cuda:0")))
    R2 = qsvm.qsvm_gram_sym(m2, diag_mode=1, log_k=(Lr2 := torch.empty((m2.N, m2.N), dtype=torch.float64, device="cuda:0")))
    torch.cuda.synchronize()
    for K, L, R, Lr in ((K1, L1, R1, Lr1), (K2, L2, R2, Lr2)):
        assert np.array_equal(K.cpu().numpy(), R.cpu().numpy())
        assert np.array_equal(L.cpu().numpy(), Lr.cpu().numpy())
    # the self-overlaps reach FP64 accuracy only through the refinement, whose
    # tile list is the static array on this path
    for K in (K1, K2):
        d = np.abs(np.diag(K.cpu().numpy()) - 1.0)
        assert d.max() <= REFINED_TOL
    # near-duplicate pairs against the FP64 oracle
    for X, pairs, K in ((X1, pairs1, K1), (X2, pairs2, K2)):
        S = omps.mps_states(X, 2, processes=5)
        _, kk = omps.mps_gram_pairs(S, S, pairs[:, 0], pairs[:, 1])
        got = K.cpu().numpy()[pairs[:, 0], pairs[:, 1]]
        assert (kk > 0.1).sum() >= 8
        assert np.abs(got - kk)[kk > 0.1].max() <= REFINED_TOL
        assert np.abs(got - kk).max() <= K_ABS_TOL


def test_noalloc_refinement_off_and_row_range():
    import torch

    X, _ = _near_duplicate_set(seed=53, n_base=24)  # 144 points
    m = encode(X, 2)
    K = torch.zeros((m.N, m.N), dtype=torch.float64, device="cuda:0")
    R = torch.zeros_like(K)
    qsvm.qsvm_gram_sym_noalloc(m, K, refine_above=-1.0)
    qsvm.qsvm_gram_sym(m, R, refine_above=-1.0)
    K2 = torch.zeros_like(K)
    R2 = torch.zeros_like(K)
    qsvm.qsvm_gram_sym_noalloc(m, K2, rows=(64, 144))
    qsvm.qsvm_gram_sym(m, R2, rows=(64, 144))
    torch.cuda.synchronize()
    assert np.array_equal(K.cpu().numpy(), R.cpu().numpy())
    assert np.array_equal(K2.cpu().numpy(), R2.cpu().numpy())


def test_noalloc_rejects_sizes_beyond_the_static_list():
    # 92,736 points need 1,050,525 tiles + 1 > 2^20 list entries: rejected on
    # the host before anything is enqueued (no buffer of that size is made)
    import ctypes

    lib = qsvm.load_library()
    st = lib.qsvm_gram_sym_noalloc(ctypes.c_void_p(0x100000), 92736, 784, 2, ctypes.c_void_p(0x200000), 92736,
                                   None, None)
    assert st == qsvm.QSVM_ERR_SIZE
