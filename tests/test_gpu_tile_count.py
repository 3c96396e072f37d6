"""GPU tests of qsvm_gram_sym_tiles_dev: the tile-list Gram whose list length
is read on the device (the surrogate's fallback without a host round trip).

Bars: the entries of the first *count listed tiles match the oracle within the
1e-5 contract and equal qsvm_gram_sym_tiles over the same entries bit for bit
(the same per-item code runs in a persistent loop); entries outside those
tiles keep the caller's sentinel; the count is clamped to [0, max_tiles]."""

import numpy as np
import pytest

from oracle import mps as omps
from paper_2405_02630_amd import qsvm, synth

from gpu_helpers import K_ABS_TOL, encode, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


def _upper_tiles(T, seed):
    lst = np.array([(i, j) for i in range(T) for j in range(i, T)], dtype=np.int32)
    return lst[np.random.default_rng(seed).permutation(len(lst))]


def _covered(lst, N):
    cov = np.zeros((N, N), dtype=bool)
    for ti, tj in lst:
        cov[ti * 64:(ti + 1) * 64, tj * 64:(tj + 1) * 64] = True
        cov[tj * 64:(tj + 1) * 64, ti * 64:(ti + 1) * 64] = True
    return cov


def _run(m, lst, count, cap=None, dev=True, **kw):
    import torch

    cap = len(lst) if cap is None else cap
    tiles = torch.as_tensor(lst.reshape(-1), device="cuda:0")
    K = torch.full((m.N, m.N), -7.0, dtype=torch.float64, device="cuda:0")
    if dev:
        c = torch.tensor([count], dtype=torch.int32, device="cuda:0")
        qsvm.qsvm_gram_sym_tiles_dev(m, tiles, c, cap, K, **kw)
    else:
        qsvm.qsvm_gram_sym_tiles(m, tiles, count, K, **kw)
    torch.cuda.synchronize()
    return K.cpu().numpy()


@pytest.mark.parametrize("reps,n,N", [(1, 10, 300), (2, 8, 300), (3, 6, 230)])
def test_device_count_matches_host_count_and_oracle(reps, n, N):
    X = synth.uniform_features(N, n, seed=50 + reps)
    m = encode(X, reps)
    T = (N + 63) // 64
    lst = _upper_tiles(T, seed=reps)
    count = len(lst) - 4  # a prefix of the shuffled list: some diagonal and ragged tiles left out
    K = _run(m, lst, count, diag_mode=1)
    Kh = _run(m, lst[:count], count, dev=False, diag_mode=1)
    assert np.array_equal(K, Kh)
    cov = _covered(lst[:count], N)
    assert np.all(K[~cov] == -7.0)
    S = omps.mps_states(X, reps)
    ii, jj = np.nonzero(np.triu(cov))
    _, kk = omps.mps_gram_pairs(S, S, ii, jj)
    assert np.max(np.abs(K[ii, jj] - kk)) <= K_ABS_TOL


@pytest.mark.parametrize("count,expect", [(0, 0), (-3, 0), (99, 6), (6, 6), (2, 2)])
def test_device_count_is_clamped(count, expect):
    X = synth.uniform_features(150, 8, seed=60)
    m = encode(X, 2)
    lst = _upper_tiles(3, seed=7)
    K = _run(m, lst, count, cap=6)
    cov = _covered(lst[:expect], 150)
    assert np.all(K[~cov] == -7.0)
    assert np.all(K[cov] != -7.0)
    if expect:
        full = _run(m, lst, 6, dev=False)
        assert np.array_equal(K[cov], full[cov])


def test_device_count_refines_like_the_host_count():
    # near-duplicate 784-pixel images: the listed tiles hold entries near 1,
    # so the FP64 refinement runs on the device-count list as well
    base, Xp, _, _ = synth.image_near_duplicates(seed=61, n_base=40)
    X = np.concatenate([base, Xp[:110]])  # 150 points
    m = encode(X, 2)
    lst = _upper_tiles(3, seed=9)
    K = _run(m, lst, 5, diag_mode=1)
    Kh = _run(m, lst[:5], 5, dev=False, diag_mode=1)
    assert np.array_equal(K, Kh)
    K32 = _run(m, lst, 5, diag_mode=1, refine_above=-1.0)
    cov = _covered(lst[:5], 150)
    assert np.max(np.abs(K[cov] - K32[cov])) > 0.0  # the refinement changed some entries
    assert np.max(np.abs(K[cov] - K32[cov])) <= K_ABS_TOL


def test_flag_then_recompute_without_host_sync():
    """qsvm_flag_tiles feeds qsvm_gram_sym_tiles_dev on one stream; the result
    equals the exact Gram on the flagged tiles."""
    import torch

    X = synth.uniform_features(200, 10, seed=62)
    m = encode(X, 2)
    exact = qsvm.qsvm_gram_sym(m).cpu().numpy()
    T = 4
    tm = np.full((T, T), -np.inf, dtype=np.float32)
    flagged = [(0, 0), (0, 3), (1, 2), (3, 3)]
    for ti, tj in flagged:
        tm[ti, tj] = 1.0
    tile_max = torch.as_tensor(tm.reshape(-1), device="cuda:0")
    tiles = torch.empty(T * (T + 1), dtype=torch.int32, device="cuda:0")
    count = torch.empty(1, dtype=torch.int32, device="cuda:0")
    K = torch.full((200, 200), -7.0, dtype=torch.float64, device="cuda:0")
    qsvm.qsvm_flag_tiles(tile_max, T, 0.5, tiles, count)
    qsvm.qsvm_gram_sym_tiles_dev(m, tiles, count, T * (T + 1) // 2, K)
    torch.cuda.synchronize()
    assert int(count.item()) == len(flagged)
    Kh = K.cpu().numpy()
    cov = _covered(np.array(flagged), 200)
    assert np.array_equal(Kh[cov], exact[cov])
    assert np.all(Kh[~cov] == -7.0)


@pytest.mark.parametrize("reps", [1, 2, 3])
def test_device_count_ignores_the_variant_hint(reps):
    X = synth.uniform_features(200, 9, seed=63 + reps)
    m = encode(X, reps)
    lst = _upper_tiles(4, seed=11)
    ref = _run(m, lst, 7, dev=False)
    for v in range(1, 5):
        assert np.array_equal(_run(m, lst, 7, variant=v), ref)
