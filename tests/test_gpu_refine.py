"""GPU tests of the FP64 refinement of large Gram entries.

The FP32 sweep's error in K is relative and biased low: at 784 qubits an
entry near 1 (a self-overlap, a near-duplicate pair) comes out 1e-5 or more
below its exact value (reps 2 to 4).  With refinement (the default: an
automatic threshold from n, 0.064 at 784 qubits) every entry above it is
recomputed with an FP64 environment from FP64 generators (the tiles holding
such entries are listed, and within them only those entries are
recomputed).  Bars: refined entries within 1e-9 of the FP64 oracle (its own
error is ~1e-12), every entry within the 1e-5 contract; untouched entries are
bitwise what the FP32 sweep wrote."""

import numpy as np
import pytest

from oracle import mps as omps
from paper_2405_02630_amd import qsvm, synth

from gpu_helpers import K_ABS_TOL, encode, require_gpu, to_dev

pytestmark = pytest.mark.gpu

REFINED_TOL = 1e-9


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


@pytest.mark.parametrize("reps", [1, 2, 3, 4])
def test_self_overlaps_784_qubits_are_exact(reps):
    import torch

    wl = synth.images784(seed=21, n_train=150, n_test=0, reps=reps)  # 3 tiles, ragged
    m = encode(wl.X, reps)
    K = qsvm.qsvm_gram_sym(m, diag_mode=1)
    K32 = qsvm.qsvm_gram_sym(m, diag_mode=1, refine_above=-1.0)
    torch.cuda.synchronize()
    d = np.abs(np.diag(K.cpu().numpy()) - 1.0)
    d32 = np.abs(np.diag(K32.cpu().numpy()) - 1.0)
    assert d.max() <= REFINED_TOL
    assert d32.max() > 1e-8  # the FP32 sweep's error that the refinement removes
    # off-diagonal tiles hold only tiny entries: not refined, bitwise unchanged
    Kh, K32h = K.cpu().numpy(), K32.cpu().numpy()
    off = np.ones_like(Kh, dtype=bool)
    for t in range(3):
        off[t * 64:(t + 1) * 64, t * 64:(t + 1) * 64] = False
    assert np.array_equal(Kh[off], K32h[off])


@pytest.mark.parametrize("reps,n_base", [(2, 40), (3, 40), (4, 8)])
def test_near_duplicates_784_qubits_vs_oracle(reps, n_base):
    base, Xp, _, _ = synth.image_near_duplicates(seed=31, n_base=n_base)  # n_base x 5 n_base pairs, K up to ~1
    ma, mb = encode(base, reps), encode(Xp, reps)
    K_auto = qsvm.qsvm_gram(ma, mb).cpu().numpy()  # automatic threshold: 0.064 at 784 qubits
    K_1e3 = qsvm.qsvm_gram(ma, mb, refine_above=1e-3).cpu().numpy()
    Sa = omps.mps_states(base, reps, processes=5)
    Sb = omps.mps_states(Xp, reps, processes=5)
    ii, jj = np.meshgrid(np.arange(base.shape[0]), np.arange(Xp.shape[0]), indexing="ij")
    _, kk = omps.mps_gram_pairs(Sa, Sb, ii.ravel(), jj.ravel())
    assert (kk > 0.1).sum() >= n_base
    d = np.abs(K_1e3.ravel() - kk)
    assert d[kk > 1e-3].max() <= REFINED_TOL  # every entry above the threshold is refined
    d = np.abs(K_auto.ravel() - kk)
    assert d[kk > 0.1].max() <= REFINED_TOL
    assert d.max() <= 5e-6  # the automatic threshold's budget for entries left in FP32


def test_no_refinement_where_the_fp32_error_is_small():
    # 16 qubits: the FP32 error (< 4.3e-6 at K = 1) needs no refinement, so
    # the automatic threshold skips it and the result equals refine_above < 0
    import torch

    m = encode(synth.uniform_features(300, 16, seed=43), 2)
    K = qsvm.qsvm_gram_sym(m, diag_mode=1).cpu().numpy()
    K32 = qsvm.qsvm_gram_sym(m, diag_mode=1, refine_above=-1.0).cpu().numpy()
    K64 = qsvm.qsvm_gram_sym(m, diag_mode=1, refine_above=1e-3).cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(K, K32)
    assert np.max(np.abs(np.diag(K64) - 1.0)) <= REFINED_TOL
    assert np.max(np.abs(K - K64)) <= 5e-6


def test_every_variant_and_the_dense_sweep_agree_after_refinement():
    import torch

    base, Xp, _, _ = synth.image_near_duplicates(seed=33, n_base=30)
    X = np.concatenate([base, Xp[:60]])  # 90 points, near-duplicate pairs inside
    m = encode(X, 2, dense=True)
    Ks = [qsvm.qsvm_gram_sym(m, variant=v).cpu().numpy() for v in range(1, 5)]
    torch.cuda.synchronize()
    for K in Ks[1:]:
        assert np.array_equal(K, Ks[0])
    Kd = qsvm.qsvm_gram_sym(m, sweep=qsvm.SWEEP_DENSE).cpu().numpy()
    big = Ks[0] > 0.1  # above the automatic threshold at 784 qubits (0.064): always refined
    # refined tiles: both sweeps end in the same FP64 recomputation
    assert np.max(np.abs(Kd[big] - Ks[0][big])) <= REFINED_TOL
    assert np.max(np.abs(Kd - Ks[0])) <= K_ABS_TOL


def test_tile_list_is_refined_like_the_full_gram():
    import torch

    base, Xp, _, _ = synth.image_near_duplicates(seed=35, n_base=50)
    X = np.concatenate([base, Xp[:100]])  # 150 points, 3 tiles
    m = encode(X, 2)
    full = qsvm.qsvm_gram_sym(m, diag_mode=1).cpu().numpy()
    T = 3
    lst = [(i, j) for i in range(T) for j in range(i, T)]
    tiles = torch.tensor(lst, dtype=torch.int32, device="cuda:0").reshape(-1)
    K = torch.full((150, 150), -2.0, dtype=torch.float64, device="cuda:0")
    qsvm.qsvm_gram_sym_tiles(m, tiles, len(lst), K, diag_mode=1)
    torch.cuda.synchronize()
    assert np.array_equal(K.cpu().numpy(), full)


def test_row_range_refines_only_its_rows():
    import torch

    base, Xp, _, _ = synth.image_near_duplicates(seed=37, n_base=40)
    ma, mb = encode(np.concatenate([base, base]), 2), encode(Xp, 2)  # 80 x 200
    full = qsvm.qsvm_gram(ma, mb).cpu().numpy()
    K = torch.full((80, 200), -3.0, dtype=torch.float64, device="cuda:0")
    qsvm.qsvm_gram(ma, mb, K, rows=(64, 80))
    torch.cuda.synchronize()
    Kh = K.cpu().numpy()
    assert np.all(Kh[:64] == -3.0)
    assert np.array_equal(Kh[64:80], full[64:80])


def test_batch_plan_is_refined_like_one_launch_per_job():
    import torch

    base, Xp, _, _ = synth.image_near_duplicates(seed=39, n_base=30)
    sets = [np.concatenate([base, Xp[:40]]), synth.images784(seed=40, n_train=70, n_test=0, reps=3).X,
            synth.uniform_features(100, 16, seed=41)]
    reps = [2, 3, 2]
    jobs, ref = [], []
    for X, r in zip(sets, reps):
        m = encode(X, r)
        K = torch.empty((m.N, m.N), dtype=torch.float64, device="cuda:0")
        jobs.append((m, K, None))
        ref.append(qsvm.qsvm_gram_sym(m, diag_mode=1).cpu().numpy())
    plan = qsvm.BatchPlan(jobs, diag_mode=1, use_graph=True)
    for _ in range(2):  # graph replays
        for _, K, _ in jobs:
            K.fill_(-1.0)
        plan.launch()
        torch.cuda.synchronize()
        for (_, K, _), R in zip(jobs, ref):
            assert np.array_equal(K.cpu().numpy(), R)
    plan.close()
    assert np.max(np.abs(np.diag(ref[0]) - 1.0)) <= REFINED_TOL


def test_refined_entries_carry_log_k_and_respect_ldk_padding():
    import torch

    base, Xp, _, _ = synth.image_near_duplicates(seed=45, n_base=24)
    ma, mb = encode(base, 2), encode(Xp[:70], 2)  # 24 x 70, rows padded to ldk = 96
    Kp = torch.full((24, 96), -5.0, dtype=torch.float64, device="cuda:0")
    Lp = torch.full((24, 96), -5.0, dtype=torch.float64, device="cuda:0")
    K, L = Kp[:, :70], Lp[:, :70]
    qsvm.qsvm_gram(ma, mb, K, log_k=L, refine_above=1e-3)
    ref = qsvm.qsvm_gram(ma, mb, refine_above=1e-3).cpu().numpy()
    torch.cuda.synchronize()
    Kh, Lh = K.cpu().numpy(), L.cpu().numpy()
    assert np.array_equal(Kh, ref)
    assert np.all(Kp.cpu().numpy()[:, 70:] == -5.0) and np.all(Lp.cpu().numpy()[:, 70:] == -5.0)
    big = Kh > 1e-3
    assert big.sum() >= 24
    assert np.max(np.abs(Lh[big] - np.log(Kh[big]))) <= 1e-12  # log K written by the FP64 pass too
