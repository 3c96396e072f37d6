"""GPU: batched persistent launches and kernel variants.

Every pair's arithmetic is the same sequence of FP32 operations whichever
kernel variant or launch shape computes it, so the batched persistent kernel
(with or without a hipGraph) and every autotuner variant must reproduce one
launch per job bit for bit."""

import numpy as np
import pytest

import oracle
from oracle import mps, statevector
from paper_2405_02630_amd import qsvm, synth

from gpu_helpers import K_ABS_TOL, encode, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


def _jobs(specs, seed=0):
    import torch

    out = []
    for q, (n, N, reps) in enumerate(specs):
        X = synth.uniform_features(N, n, seed=seed + q)
        m = encode(X, reps)
        K = torch.full((N, N), -5.0, dtype=torch.float64, device="cuda:0")
        L = torch.full((N, N), -5.0, dtype=torch.float64, device="cuda:0")
        out.append((X, m, K, L))
    return out


def _reference(jobs):
    import torch

    refs = []
    for X, m, _, _ in jobs:
        K = torch.empty((m.N, m.N), dtype=torch.float64, device="cuda:0")
        L = torch.empty_like(K)
        qsvm.qsvm_gram_sym(m, K, log_k=L)
        refs.append((K, L))
    torch.cuda.synchronize()
    return refs


SPECS = [(16, 64, 2), (64, 130, 3), (196, 300, 2), (8, 70, 1), (100, 65, 3), (33, 200, 1), (400, 129, 2)]


@pytest.mark.parametrize("use_graph", [True, False], ids=["graph", "stream"])
def test_batched_equals_one_launch_per_job(use_graph):
    import torch

    jobs = _jobs(SPECS)
    refs = _reference(jobs)
    plan = qsvm.BatchPlan([(m, K, L) for _, m, K, L in jobs], use_graph=use_graph)
    total, grid, g = plan.info()
    assert g == use_graph and grid > 0 and total > 0
    plan.launch()
    torch.cuda.synchronize()
    for (X, m, K, L), (Kr, Lr) in zip(jobs, refs):
        assert torch.equal(K, Kr), (m.n, m.N, m.reps)
        assert torch.equal(L, Lr)
    plan.close()


def test_graph_replays_match_eager_each_time():
    import torch

    jobs = _jobs(SPECS[:4], seed=50)
    refs = _reference(jobs)
    plan = qsvm.BatchPlan([(m, K, L) for _, m, K, L in jobs], use_graph=True)
    for replay in range(3):
        for _, _, K, L in jobs:  # eager work between replays
            K.fill_(float(replay) - 9.0)
            L.zero_()
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for (_, m, K, L), (Kr, Lr) in zip(jobs, refs):
            assert torch.equal(K, Kr), (replay, m.n, m.N)
            assert torch.equal(L, Lr)
    plan.close()


def test_batched_small_grid_still_drains_the_queue():
    import torch

    jobs = _jobs(SPECS[:3], seed=70)
    refs = _reference(jobs)
    plan = qsvm.BatchPlan([(m, K, L) for _, m, K, L in jobs], use_graph=False, grid_blocks=3)
    plan.launch()
    torch.cuda.synchronize()
    for (_, _, K, L), (Kr, Lr) in zip(jobs, refs):
        assert torch.equal(K, Kr) and torch.equal(L, Lr)
    plan.close()


def test_batched_jobs_against_the_oracle():
    import torch

    specs = [(9, 70, 2), (10, 40, 3), (7, 66, 1)]
    jobs = _jobs(specs, seed=90)
    plan = qsvm.BatchPlan([(m, K, L) for _, m, K, L in jobs], diag_mode=1)
    plan.launch()
    torch.cuda.synchronize()
    for (X, m, K, L) in jobs:
        ref = statevector.sv_gram(X, m.reps)
        Kh = K.cpu().numpy()
        assert np.max(np.abs(Kh - ref)) <= K_ABS_TOL
        assert oracle.check_gram(Kh, tol=K_ABS_TOL) == {}
    plan.close()


def test_uneven_jobs_workload_bitwise():
    """The 64-job uneven workload (n in {16..784}, N in [64, 2048], reps 2/3)."""
    import torch

    wl = synth.uneven_jobs(seed=0)
    jobs = []
    for w in wl:
        m = encode(w.X, w.reps)
        K = torch.empty((m.N, m.N), dtype=torch.float64, device="cuda:0")
        jobs.append((w.X, m, K, None))
    plan = qsvm.BatchPlan([(m, K, None) for _, m, K, _ in jobs], use_graph=True)
    plan.launch()
    torch.cuda.synchronize()
    for q, (X, m, K, _) in enumerate(jobs):
        Kr = qsvm.qsvm_gram_sym(m)
        torch.cuda.synchronize()
        assert torch.equal(K, Kr), q
    # spot-check two jobs against the oracle
    for q in (0, 7):
        X, m, K, _ = jobs[q]
        pts = np.array([0, 1, 63, m.N - 1])
        S = mps.mps_states(X[pts], m.reps)
        ia, jb = np.triu_indices(len(pts), 1)
        lk, kk = mps.mps_gram_pairs(S, S, ia, jb)
        Kh = K.cpu().numpy()
        assert np.max(np.abs(Kh[pts[ia], pts[jb]] - kk)) <= K_ABS_TOL
    plan.close()


@pytest.mark.parametrize("reps", [1, 2, 3])
def test_every_variant_is_bitwise_identical(reps):
    import torch

    X = synth.uniform_features(150, 40, seed=reps)
    m = encode(X, reps)
    outs = []
    for v in range(1, qsvm.N_VARIANTS + 1):
        K = torch.empty((150, 150), dtype=torch.float64, device="cuda:0")
        L = torch.empty_like(K)
        qsvm.qsvm_gram_sym(m, K, log_k=L, variant=v)
        outs.append((K, L))
    torch.cuda.synchronize()
    for K, L in outs[1:]:
        assert torch.equal(K, outs[0][0]) and torch.equal(L, outs[0][1])


@pytest.mark.parametrize("pi2", [2, 4])
def test_batched_item_shapes_are_bitwise_identical(pi2):
    import torch

    jobs = _jobs(SPECS, seed=40)
    refs = _reference(jobs)
    plan = qsvm.BatchPlan([(m, K, L) for _, m, K, L in jobs], use_graph=True, item_pi2=pi2, item_pi3=1)
    assert plan.shape() == (pi2, 1)
    plan.launch()
    torch.cuda.synchronize()
    for (X, m, K, L), (Kr, Lr) in zip(jobs, refs):
        assert torch.equal(K, Kr), (pi2, m.n, m.N, m.reps)
        assert torch.equal(L, Lr)
    plan.close()


def test_plan_takes_its_item_shape_from_the_tuned_table():
    # the costliest job (N^2 n) of each reps decides: 196 qubits for reps = 2,
    # 64 qubits for reps = 3
    n2, N2, _ = max((s for s in SPECS if s[2] == 2), key=lambda s: s[1] ** 2 * s[0])
    n3, N3, _ = max((s for s in SPECS if s[2] == 3), key=lambda s: s[1] ** 2 * s[0])
    assert (n2, n3) == (196, 64)
    jobs = _jobs(SPECS, seed=41)
    old2, old3 = qsvm.qsvm_get_tuned_variant(2, n2, N2), qsvm.qsvm_get_tuned_variant(3, n3, N3)
    try:
        qsvm.qsvm_set_tuned_variant(2, n2, N2, 1)  # 4 ket points per lane
        qsvm.qsvm_set_tuned_variant(3, n3, N3, 1)  # 2 per lane: beyond the batched kernel's registers
        plan = qsvm.BatchPlan([(m, K, L) for _, m, K, L in jobs], use_graph=False)
        assert plan.shape() == (4, 1)
        plan.close()
        qsvm.qsvm_set_tuned_variant(2, n2, N2, 0)
        plan = qsvm.BatchPlan([(m, K, L) for _, m, K, L in jobs], use_graph=False)
        assert plan.shape() == (2, 1)
        plan.close()
    finally:
        qsvm.qsvm_set_tuned_variant(2, n2, N2, old2)
        qsvm.qsvm_set_tuned_variant(3, n3, N3, old3)


def test_autotune_persists_for_this_architecture():
    import os
    import subprocess
    import sys

    best, _ = qsvm.qsvm_autotune(3, 40, 256)
    path = qsvm.qsvm_autotune_cache_path()
    assert path and os.path.exists(path)
    rows = [ln.split() for ln in open(path) if not ln.startswith("#")]
    assert ["gfx950", "3", "5", "8", str(best)] in rows
    code = ("from paper_2405_02630_amd import qsvm; import torch; torch.zeros(1, device='cuda:0'); "
            "print(qsvm.qsvm_get_tuned_variant(3, 40, 256))")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                       cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == str(best)


def test_autotune_records_a_variant():
    best, ms = qsvm.qsvm_autotune(2, 64, 512)
    assert 0 <= best < qsvm.N_VARIANTS
    assert all(t > 0 for t in ms) and ms[best] == min(ms)
    assert qsvm.qsvm_get_tuned_variant(2, 64, 512) == best
    assert qsvm.qsvm_get_tuned_variant(2, 127, 1000) == best
