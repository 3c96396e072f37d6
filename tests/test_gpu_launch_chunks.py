"""GPU tests of Gram calls whose tiles need more than one kernel launch.

A dispatch holds at most 2^24 - 8 blocks of 256 threads, so the library
issues large tile sets as several launches (whole rows of tiles, or stretches
of a tile list).  These tests take tile sets just above one launch, check
that every entry is written, and check entries that only the second launch
writes against the oracle: the tail of a shuffled list of a whole triangle of
tiles, and the last tile rows of a rectangular Gram.  Bars as in the other parity
tests (|dK| <= 1e-5)."""

import numpy as np
import pytest

from oracle import statevector
from paper_2405_02630_amd import qsvm, synth

from gpu_helpers import K_ABS_TOL, encode, require_gpu, to_dev

pytestmark = pytest.mark.gpu

MAX_GRID_BLOCKS = (1 << 24) - 8


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


# (reps, sweep, blocks per tile of that sweep, tiles per side: the smallest
# triangle T (T + 1) / 2 above one launch's 2^24 - 8 blocks)
@pytest.mark.parametrize("reps,sweep,bpt,T", [(4, qsvm.SWEEP_AUTO, 32, 1024), (2, qsvm.SWEEP_DENSE, 16, 1449)])
def test_tile_list_longer_than_one_launch(reps, sweep, bpt, T):
    import torch

    cap = MAX_GRID_BLOCKS // bpt  # tiles per launch
    assert T * (T + 1) // 2 > cap
    n = 2
    N = 64 * T - 9  # ragged last tile
    X = synth.uniform_features(N, n, seed=5100 + reps)
    m = encode(X, reps, dense=sweep == qsvm.SWEEP_DENSE)
    ti, tj = np.triu_indices(T)
    order = np.random.default_rng(5110 + reps).permutation(ti.size)
    lst = np.stack([ti[order], tj[order]], axis=1).astype(np.int32)
    # the ragged corner tiles (0, T-1) and (T-1, T-1) go last
    corner = (lst[:, 1] == T - 1) & ((lst[:, 0] == 0) | (lst[:, 0] == T - 1))
    lst = np.concatenate([lst[~corner], lst[corner]])
    tiles = torch.as_tensor(lst, device="cuda:0")
    K = torch.full((N, N), float("nan"), dtype=torch.float64, device="cuda:0")
    qsvm.qsvm_gram_sym_tiles(m, tiles, len(lst), K, sweep=sweep, diag_mode=1)
    torch.cuda.synchronize()
    assert not bool(torch.isnan(K).any())
    # tiles of the second launch (beyond the first `cap` list entries)
    second = lst[cap:]
    pick = list(second[:6]) + list(second[-2:])
    for a, b in pick:
        r = np.arange(64 * a, min(64 * a + 64, N))
        c = np.arange(64 * b, min(64 * b + 64, N))
        got = K[64 * a : 64 * a + r.size, 64 * b : 64 * b + c.size].cpu().numpy()
        ref = statevector.sv_gram_rect(X[r], X[c], reps)
        assert np.max(np.abs(got - ref)) <= K_ABS_TOL, (a, b)


def test_rect_rows_split_across_launches():
    import torch

    reps, n = 4, 2
    Na, Nb = 64 * 65, 1 << 19  # 65 x 8192 tiles at 32 blocks each: two launches
    assert Na // 64 * (Nb // 64) * 32 > MAX_GRID_BLOCKS
    Xa = synth.uniform_features(Na, n, seed=5200)
    Xb = synth.uniform_features(Nb, n, seed=5201)
    ma, mb = encode(Xa, reps), encode(Xb, reps)
    K = torch.full((Na, Nb), float("nan"), dtype=torch.float64, device="cuda:0")
    qsvm.qsvm_gram(ma, mb, K)
    torch.cuda.synchronize()
    assert not bool(torch.isnan(K).any())
    # rows on both sides of the first launch's last tile row, and the last rows
    rows = np.r_[4000:4040, 4090:4100, Na - 8 : Na]
    rng = np.random.default_rng(5202)
    cols = np.sort(np.r_[0, 63, 64, Nb - 1, rng.choice(Nb, 200, replace=False)])
    got = K[to_dev(rows).long()][:, to_dev(cols).long()].cpu().numpy()
    ref = statevector.sv_gram_rect(Xa[rows], Xb[cols], reps)
    assert np.max(np.abs(got - ref)) <= K_ABS_TOL
