"""Benchmark: quantum-kernel Gram entries per second on one MI355X.

Workload (default): 784-qubit (28x28) synthetic images, reps = 2 (bond
dimension 4), 4096 training points; one step = encode the 4096 feature vectors
as MPS + the symmetric Gram (N(N-1)/2 = 8,386,560 contracted pairs), with the
features already resident in HBM.  value = contracted pairs per second.

Prints one JSON line with the timing, a roofline entry for the dominant
kernel (the overlap sweep; launch durations from HIP events on the launch
stream) and, on rank 0, a CPU baseline: the FP64 oracle timed on the host
cores on a bounded sample of the same workload.  Legs (--legs, all by
default) add their own objects to the line:
  exact        -- the workload's second Gram, 1024 test images x the 4096
                  training images (`test_by_train`: encode of the test MPS +
                  rectangular Gram per step);
  reps3        -- both Grams again at reps = 3 (bond dimension 8);
  mixture64    -- 1024 points of a 10-class Gaussian mixture in R^64, reps = 2:
                  encode + symmetric Gram (the refinement recomputes the
                  entries above the 64-qubit threshold);
  deep         -- the split sweep at reps 4, 5 and 6 (bond dimensions 16, 32,
                  64): symmetric Grams of 2048, 1024 and 512 images;
  refine_worst -- 4096 near-identical images, every tile refined in FP64,
                  against the FP32 sweep alone;
  mlp          -- the surrogate's MLP at 784 (832) -> 512 -> 512 -> 256: the
                  forward pass of 32768 rows and one 8192-pair training step;
  surrogate    -- 32768 synthetic 784-pixel images with 2048 near-duplicate
                  copies, reps = 2: the log-domain surrogate trained on exact
                  entries of ~2 % of the tiles, calibrated on ~0.5 %, judged
                  on ~1 % held out (trained, untrained and constant
                  predictors), its whole-set Gram with exact fallback for the
                  flagged tiles timed against the exact whole-set Gram, and
                  one-vs-rest SVM accuracy on a 4096-point subset;
  batched      -- 64 independent Gram jobs of uneven n, N and reps in one
                  persistent hipGraph launch (default and tuned work-item
                  shape) against one launch per job;
  sv           -- the state-vector engine against the MPS engine on 512
                  points at 12, 16 and 20 qubits: times, agreement, and the
                  FP64 matrix-core rate of the state-vector Gram.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--reps 1..6]
                       [--sweep butterfly|dense] [--legs exact,reps3,deep,...]
                       [--no-cpu-baseline] [--cpu-sample P] [--copy-calibration MiB]
                       [--surrogate-gram-only N]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3  # MI355X FP32 vector: 256 CU x 2.4 GHz x 256 flop/clk

# HBM bytes per sweep launch from two rocprofv3 counter passes (FETCH_SIZE,
# WRITE_SIZE), each scaled by what the counter reads for a 1 GiB copy; valid
# only for the kernel and configuration they were taken on (sweep, reps,
# points, qubits) -- any other configuration reports null.
MEASURED_TRAFFIC = {
    ("butterfly", 2, 4096, 784): (3.4178e9, "profiles/sweep_butterfly_images784_r2_hbm_counters.md"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sweep_flops_per_pair(n: int, reps: int, sweep: str) -> int:
    """Executed floating-point operations of one pair's sweep.

    butterfly: per site k >= 1, (2r-1) bit axes x 2^(2r-2) butterflies x 2
    complex multiply-adds (8 flops each) + 2 complex products for the shared
    axis coefficients (6 flops each).
    dense: per site chi^3 complex multiply-adds (8 flops each).
    The FP64 closure and the renormalisation (max / ldexp) are not counted.
    """
    if sweep == "butterfly":
        per_site = (2 * reps - 1) * (1 << (2 * reps - 2)) * 2 * 8 + 12
        return (n - 1) * per_site
    chi = 1 << reps
    return n * chi**3 * 8


def cpu_baseline(X, reps, K_gpu, sample_points: int, cores: int):
    """Time the FP64 MPS oracle on the first `sample_points` points (all pairs)."""
    import numpy as np
    from multiprocessing import get_context

    import oracle
    from oracle import mps as omps

    Xs = X[:sample_points]
    ia, jb = np.triu_indices(sample_points, 1)
    t0 = time.perf_counter()
    states = omps.mps_states(Xs, reps, processes=cores)
    t1 = time.perf_counter()
    chunks = np.array_split(np.arange(ia.shape[0]), cores)
    global _BENCH_STATES
    _BENCH_STATES = states
    with get_context("fork").Pool(cores) as pool:
        parts = pool.map(_pair_chunk, [(ia[c], jb[c]) for c in chunks])
    t2 = time.perf_counter()
    lk = np.concatenate([p[0] for p in parts])
    kk = np.concatenate([p[1] for p in parts])
    pairs = ia.shape[0]
    Kg = K_gpu[ia, jb]
    max_dk = float(np.max(np.abs(Kg - kk)))
    return {
        "value": pairs / (t2 - t0),
        "unit": "entries/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"first {sample_points} points of the workload, all {pairs} pairs i<j: "
        f"gate-by-gate FP64 MPS build ({t1 - t0:.1f} s) + FP64 overlap sweeps ({t2 - t1:.1f} s), "
        f"{cores} worker processes",
        "seconds": t2 - t0,
        "sample_max_abs_dK_vs_gpu": max_dk,
        "sample_max_log_err_vs_gpu": None,
        "_lk": lk,
        "_pairs": (ia, jb),
    }


def refine_worst_accuracy(samples, cores: int):
    """CPU-baseline step for the refine_worst leg: the FP64 oracle on the pairs
    i <= j of its first 64 points against the GPU values kept there (with the
    refinement and without)."""
    import numpy as np

    from oracle import mps as omps

    S = omps.mps_states(samples["X"], samples["reps"], processes=cores)
    ia, jb = np.triu_indices(samples["X"].shape[0])
    _, kk = omps.mps_gram_pairs(S, S, ia, jb)
    out = {"K_oracle_min_sample": float(kk.min())}
    for tag in ("refined", "fp32_only"):
        out[f"{tag}_sample_max_abs_dK"] = float(np.max(np.abs(samples[tag] - kk)))
    return out


def near_duplicate_check(reps: int, cores: int, n_base: int = 8):
    """The bar where it bites: near-duplicate 784-pixel images (K up to ~1),
    GPU rectangular Gram of n_base base images x their eps-perturbed copies
    in the default launch configuration against the FP64 MPS oracle."""
    import numpy as np
    import torch

    from oracle import mps as omps
    from paper_2405_02630_amd import qsvm, synth

    base, Xp, _, eps = synth.image_near_duplicates(seed=3, n_base=n_base)
    dev = torch.device("cuda:0")
    ma = qsvm.qsvm_encode_mps(torch.as_tensor(base, device=dev), reps)
    mb = qsvm.qsvm_encode_mps(torch.as_tensor(Xp, device=dev), reps)
    K = qsvm.qsvm_gram(ma, mb).cpu().numpy()
    S = omps.mps_states(base, reps, processes=cores)
    Sp = omps.mps_states(Xp, reps, processes=cores)
    ii, jj = np.meshgrid(np.arange(base.shape[0]), np.arange(Xp.shape[0]), indexing="ij")
    _, kk = omps.mps_gram_pairs(S, Sp, ii.ravel(), jj.ravel())
    d = np.abs(K.ravel() - kk)
    return {
        "pairs": int(kk.size),
        "eps": sorted(set(float(e) for e in eps)),
        "K_oracle_max": float(kk.max()),
        "pairs_with_K_above_1e-3": int(np.sum(kk > 1e-3)),
        "max_abs_dK": float(d.max()),
        "max_abs_dK_where_K_above_1e-3": float(d[kk > 1e-3].max()) if np.any(kk > 1e-3) else None,
    }


_BENCH_STATES = None


def _pair_chunk(args):
    from oracle import mps as omps

    ia, jb = args
    return omps.mps_gram_pairs(_BENCH_STATES, _BENCH_STATES, ia, jb)


def _events(n):
    import torch

    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def test_by_train_leg(reps, n_train, train_buf, Xtrain, sweep, args):
    """Rectangular Gram of 1024 test images against the training images (the
    second Gram of the 784-pixel workload); encode + Gram timed per step."""
    import numpy as np
    import torch
    from paper_2405_02630_amd import qsvm, synth

    dev = torch.device("cuda:0")
    n_test = 1024
    wl = synth.images784(seed=0, n_train=n_train, n_test=n_test, reps=reps)
    Xt = torch.as_tensor(wl.X_test, dtype=torch.float64, device=dev)
    mb = qsvm.qsvm_encode_mps(Xtrain, reps, out=train_buf)
    K = torch.empty((n_test, n_train), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        ma = qsvm.qsvm_encode_mps(Xt, reps)
        if ev is not None:
            ev[0].record(stream)
        qsvm.qsvm_gram(ma, mb, K, sweep=sweep, renorm_every=args.renorm_every)
        if ev is not None:
            ev[1].record(stream)

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(evs[s])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    sweep_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    pairs = n_test * n_train
    flops = sweep_flops_per_pair(Xt.shape[1], reps, args.sweep) * pairs
    log(f"test x train {n_test} x {n_train}: {ms:.3f} ms/step, sweep {sweep_ms:.3f} ms, "
        f"{pairs / (ms / 1e3):.4e} entries/s")
    return {
        "workload": f"images-n{Xt.shape[1]}-r{reps}-test{n_test}-train{n_train}-rect",
        "pairs_per_step": pairs,
        "ms_per_step": ms,
        "value": pairs / (ms / 1e3),
        "unit": "entries/s",
        "sweep_ms": round(sweep_ms, 4),
        "sweep_frac_of_fp32_peak": round(flops / (sweep_ms / 1e3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS, 4),
        "step": "encode test MPS + rectangular Gram against the resident training MPS",
    }


def exact_reps_leg(reps, n_train, args, kinds=("sym", "test_by_train"), steps=None):
    """The 784-pixel image workload at another depth: the symmetric Gram of the
    training images (encode + Gram per step) and the 1024 x n_train test-by-train
    Gram, each with its sweep's fraction of the FP32 vector peak."""
    steps = args.steps if steps is None else steps
    import numpy as np
    import torch
    from paper_2405_02630_amd import qsvm, synth

    dev = torch.device("cuda:0")
    wl = synth.images784(seed=0, n_train=n_train, n_test=1024, reps=reps)
    n = wl.X.shape[1]
    X = torch.as_tensor(wl.X, dtype=torch.float64, device=dev)
    Xt = torch.as_tensor(wl.X_test, dtype=torch.float64, device=dev)
    buf = torch.empty(qsvm.qsvm_mps_bytes(n_train, n, reps), dtype=torch.uint8, device=dev)
    K = torch.empty((n_train, n_train), dtype=torch.float64, device=dev)
    Kr = torch.empty((Xt.shape[0], n_train), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    out = {}
    for kind in kinds:
        def step(ev=None):
            m = qsvm.qsvm_encode_mps(X, reps, out=buf)
            if kind == "sym":
                if ev is not None:
                    ev[0].record(stream)
                qsvm.qsvm_gram_sym(m, K)
            else:
                ma = qsvm.qsvm_encode_mps(Xt, reps)
                if ev is not None:
                    ev[0].record(stream)
                qsvm.qsvm_gram(ma, m, Kr)
            if ev is not None:
                ev[1].record(stream)

        for _ in range(max(1, args.warmup)):
            step()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = time.perf_counter()
        for st in range(steps):
            step(evs[st])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        sweep_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        pairs = n_train * (n_train - 1) // 2 if kind == "sym" else Xt.shape[0] * n_train
        flops = sweep_flops_per_pair(n, reps, "butterfly") * pairs
        out[kind] = {
            "workload": (f"images-n{n}-r{reps}-train{n_train}-sym" if kind == "sym"
                         else f"images-n{n}-r{reps}-test{Xt.shape[0]}-train{n_train}-rect"),
            "pairs_per_step": pairs,
            "ms_per_step": ms,
            "value": pairs / (ms / 1e3),
            "unit": "entries/s",
            "sweep_ms": round(sweep_ms, 4),
            "sweep_tflops": round(flops / (sweep_ms / 1e3) / 1e12, 3),
            "sweep_frac_of_fp32_peak": round(flops / (sweep_ms / 1e3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS, 4),
            "step": ("encode MPS + symmetric Gram" if kind == "sym"
                     else "encode both MPS sets + rectangular Gram (the sweep time covers the Gram only)"),
        }
        log(f"reps={reps} {kind}: {ms:.3f} ms/step, sweep {sweep_ms:.3f} ms "
            f"({out[kind]['sweep_frac_of_fp32_peak']:.3f} of peak), {out[kind]['value']:.4e} entries/s")
    del K, Kr, buf
    torch.cuda.empty_cache()
    return out


def mixture64_leg(args, steps=None):
    """The 64-qubit workload: 1024 points of the 10-class Gaussian mixture in
    R^64 (reps = 2), encode + symmetric Gram per step, the sweep's fraction of
    the FP32 vector peak, the entries the refinement recomputed (K above the
    64-qubit threshold), and, outside the timed region, max|dK| against the
    same Gram with every entry recomputed in FP64 (refine_above = 1e-300;
    the parity tests check this workload against the oracle)."""
    steps = args.steps if steps is None else steps
    import numpy as np
    import torch

    from paper_2405_02630_amd import qsvm, synth

    dev = torch.device("cuda:0")
    wl = synth.mixture64(seed=0)
    N, n = wl.X.shape
    X = torch.as_tensor(wl.X, dtype=torch.float64, device=dev)
    buf = torch.empty(qsvm.qsvm_mps_bytes(N, n, wl.reps), dtype=torch.uint8, device=dev)
    K = torch.empty((N, N), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        m = qsvm.qsvm_encode_mps(X, wl.reps, out=buf)
        if ev is not None:
            ev[0].record(stream)
        qsvm.qsvm_gram_sym(m, K)
        if ev is not None:
            ev[1].record(stream)

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for st in range(steps):
        step(evs[st])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    gram_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    pairs = N * (N - 1) // 2
    flops = sweep_flops_per_pair(n, wl.reps, "butterfly") * pairs
    Kh = K.cpu().numpy()
    thresh = qsvm.qsvm_auto_refine_threshold(n)
    iu = np.triu_indices(N, 1)
    K64 = qsvm.qsvm_gram_sym(qsvm.qsvm_encode_mps(X, wl.reps), refine_above=1e-300).cpu().numpy()
    res = {
        "workload": f"mixture-n{n}-r{wl.reps}-N{N}-sym (10-class Gaussian mixture in R^64)",
        "pairs_per_step": pairs,
        "ms_per_step": ms,
        "value": pairs / (ms / 1e3),
        "unit": "entries/s",
        "gram_ms": round(gram_ms, 4),
        "gram_frac_of_fp32_peak": round(flops / (gram_ms / 1e3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS, 4),
        "K_max_offdiag": float(np.max(Kh[iu])),
        "entries_above_refine_threshold": int(np.count_nonzero(Kh[iu] > thresh)),
        "refine_threshold": thresh,
        "max_abs_dK_vs_fp64_sweep": float(np.max(np.abs(Kh[iu] - K64[iu]))),
        "step": "encode MPS + symmetric Gram (sweep, tile scan and FP64 refinement of the entries above the threshold)",
    }
    log(f"mixture64: {ms:.3f} ms/step, Gram {gram_ms:.3f} ms ({res['gram_frac_of_fp32_peak']:.3f} of peak in "
        f"sweep flops), {res['value']:.4e} entries/s; {res['entries_above_refine_threshold']} entries above "
        f"{thresh:.3f} refined; max|dK| vs the FP64 sweep {res['max_abs_dK_vs_fp64_sweep']:.2e}")
    del K, buf
    torch.cuda.empty_cache()
    return res


def refine_worst_leg(args, reps: int = 2, N: int = 4096, cores: int = 8):
    """Worst case of the FP64 refinement: 4096 near-identical 784-pixel images,
    so every 64 x 64 tile holds entries near 1 and is recomputed with an FP64
    environment.  Times the symmetric Gram with the automatic refinement and
    with the refinement off; the pairs of the first 64 points (self-overlaps
    computed, diag_mode 1) are kept for the CPU-baseline step, which compares
    both with the FP64 oracle (refine_worst_accuracy)."""
    import numpy as np
    import torch

    from paper_2405_02630_amd import qsvm, synth

    dev = torch.device("cuda:0")
    Xh = synth.near_identical_images(N, seed=9)
    X = torch.as_tensor(Xh, device=dev)
    m = qsvm.qsvm_encode_mps(X, reps)
    K = torch.empty((N, N), dtype=torch.float64, device=dev)
    res = {"workload": f"near-identical images-n{Xh.shape[1]}-r{reps}-N{N}-sym (one image + 4e-4 N(0,1) pixel noise)",
           "_samples": {"X": Xh[:64], "reps": reps}}
    ia, jb = np.triu_indices(64)
    for tag, ra in (("refined", 0.0), ("fp32_only", -1.0)):
        qsvm.qsvm_gram_sym(m, K, refine_above=ra, diag_mode=1)
        torch.cuda.synchronize()
        ev = _events(2)
        ev[0].record()
        for _ in range(3):
            qsvm.qsvm_gram_sym(m, K, refine_above=ra, diag_mode=1)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / 3
        res["_samples"][tag] = K[:64, :64].cpu().numpy()[ia, jb]
        res[tag] = {"ms": ms, "value": N * (N + 1) // 2 / (ms / 1e3), "unit": "entries/s"}
        log(f"refine worst case ({tag}): {ms:.2f} ms")
    res["refined_over_fp32_time"] = res["refined"]["ms"] / res["fp32_only"]["ms"]
    del K
    torch.cuda.empty_cache()
    return res


def _tile_pairs(tiles, N):
    """Pairs (i, j), i < j, of the listed 64 x 64 tiles of an N-point upper triangle."""
    import numpy as np

    a = np.arange(64)
    I, J = [], []
    for ti, tj in tiles:
        ii = ti * 64 + a[:, None].repeat(64, 1)
        jj = tj * 64 + a[None, :].repeat(64, 0)
        m = (ii < jj) & (jj < N)
        I.append(ii[m])
        J.append(jj[m])
    return np.concatenate(I), np.concatenate(J)


def surrogate_leg(args, exact_rate):
    """Train, time and judge the learned surrogate on 32768 784-pixel images
    (reps = 2) of which 2048 are near-duplicate copies (K up to ~1).

    Training, calibration and judging pairs are the pairs of uniformly drawn
    64 x 64 tiles of the upper triangle: 2 %, 0.5 % and 1 % of the tiles,
    disjoint, with exact K and ln K from the tile-list Gram.  Reports the
    held-out log-domain error of the trained network, the untrained network
    (same head fitted to the same targets) and the best constant predictor,
    on all pairs and on the close pairs (ln K > -100); the tiles each of
    them would have to send to the exact fallback at the tau = 1e-6 bar; the
    timed whole Gram with fallback against the exact Gram; and the largest
    |dK| over every held-out pair."""
    import numpy as np
    import torch

    from paper_2405_02630_amd import qsvm, synth
    from paper_2405_02630_amd.surrogate import Surrogate, SurrogateConfig

    dev = torch.device("cuda:0")
    N = args.sur_points
    reps = 2
    n_copies = N // 16
    Xh, labels, base_of_row = synth.images784_with_near_duplicates(N, n_copies, seed=5)
    X = torch.as_tensor(Xh, dtype=torch.float64, device=dev)
    n = Xh.shape[1]
    T = (N + 63) // 64
    upper = [(a, b) for a in range(T) for b in range(a, T)]
    rng = np.random.default_rng(17)
    perm = rng.permutation(len(upper))
    n_tr, n_cal, n_ho = (int(round(f * len(upper))) for f in (0.02, 0.005, 0.01))
    sets = {"train": perm[:n_tr], "cal": perm[n_tr:n_tr + n_cal], "held": perm[n_tr + n_cal:n_tr + n_cal + n_ho]}
    mps_all = qsvm.qsvm_encode_mps(X, reps)
    Kex = torch.full((N, N), -1.0, dtype=torch.float64, device=dev)
    Lex = torch.full((N, N), -1.0, dtype=torch.float64, device=dev)
    pairs = {}
    t0 = time.perf_counter()
    for name, sel in sets.items():
        tl = np.array([upper[u] for u in sel], dtype=np.int32)
        qsvm.qsvm_gram_sym_tiles(mps_all, torch.as_tensor(tl.reshape(-1), device=dev), len(tl), Kex, log_k=Lex)
        I, J = _tile_pairs(tl, N)
        It, Jt = torch.as_tensor(I, device=dev), torch.as_tensor(J, device=dev)
        pairs[name] = (I, J, Lex[It, Jt].cpu().numpy(), Kex[It, Jt].cpu().numpy())
    torch.cuda.synchronize()
    t_targets = time.perf_counter() - t0
    log(f"surrogate: N={N} ({n_copies} near duplicates), exact targets on "
        f"{n_tr}/{n_cal}/{n_ho} tiles: {len(pairs['train'][0])} train, {len(pairs['cal'][0])} calibration, "
        f"{len(pairs['held'][0])} held-out pairs ({t_targets:.2f} s)")
    Itr, Jtr, Ltr, _ = pairs["train"]
    Ica, Jca, Lca, _ = pairs["cal"]
    Iho, Jho, Lho, Kho = pairs["held"]

    cfg = SurrogateConfig()
    sur = Surrogate(n, cfg)
    pick = rng.choice(Itr.size, min(65536, Itr.size), replace=False)
    sur.init_head(X, Itr[pick], Jtr[pick], Ltr[pick])
    tau = cfg.tau
    lt = math.log(tau)
    const = float(np.median(Ltr))

    def margin_for(lh_cal):
        # the margin Surrogate.calibrate sets, for the predictions lh_cal
        near = Lca >= lt - 20.0
        under = Lca - lh_cal
        return max(0.0, float(np.max(under[near])) if near.any() else float(np.max(under))) + 1.0

    def judge(lh):
        e = np.abs(lh - Lho)
        close = Lho > -100.0
        return {"mean_abs_dlnK": float(e.mean()), "median_abs_dlnK": float(np.median(e)),
                "close_pairs_mean_abs_dlnK": float(e[close].mean()) if close.any() else None,
                "close_pairs_max_abs_dlnK": float(e[close].max()) if close.any() else None}

    lh0_ho, _ = sur.predict_pairs(X, Iho, Jho)
    lh0_ca, _ = sur.predict_pairs(X, Ica, Jca)
    margin0 = margin_for(lh0_ca)
    _, cnt0 = sur.gram(X, None, margin=margin0)
    untrained_flagged = int(cnt0.item())
    rep = sur.fit(X, Itr, Jtr, Ltr, steps=args.sur_steps, log_every=max(1, args.sur_steps // 5))
    log(f"surrogate: trained {rep.steps} steps in {rep.seconds:.2f} s, loss {rep.loss_history}")
    lh1_ho, _ = sur.predict_pairs(X, Iho, Jho)
    margin = sur.calibrate(X, Ica, Jca, Lca)
    untrained, trained = judge(lh0_ho), judge(lh1_ho)
    constant = judge(np.full_like(Lho, const))
    near_c = Lca >= lt - 20.0
    const_margin = max(0.0, float(np.max(Lca[near_c] - const)) if near_c.any() else float(np.max(Lca - const))) + 1.0
    constant_flagged = len(upper) if const >= lt - const_margin else 0

    Kall = torch.empty((N, N), dtype=torch.float64, device=dev)
    sur.gram(X, mps_all, K=Kall)  # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        _, flagged = sur.gram(X, mps_all, K=Kall)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    flagged = int(flagged.item())
    fb = [int(v) for v in sur.fallback.cpu()] if sur.fallback is not None else [None, None]
    sur_s = float(np.median(times))
    It, Jt = torch.as_tensor(Iho, device=dev), torch.as_tensor(Jho, device=dev)
    Ks_ho = Kall[It, Jt].cpu().numpy()
    dk = np.abs(Ks_ho - Kho)
    big = Kho > 1e-3
    # SVM on a 4096-point subset with the exact and the surrogate Gram
    svm_pts = np.sort(rng.choice(N, 4096, replace=False))
    sp = torch.as_tensor(svm_pts, device=dev)
    Ks_svm = Kall[sp][:, sp].cpu().numpy()
    m_svm = qsvm.qsvm_encode_mps(X[sp].contiguous(), reps)
    Ke_svm = qsvm.qsvm_gram_sym(m_svm).cpu().numpy()
    acc_exact, acc_sur = svm_accuracies(Ke_svm, Ks_svm, labels[svm_pts])
    # exact whole-set Gram for the speedup (same N, same buffer)
    ev = _events(2)
    ev[0].record()
    qsvm.qsvm_gram_sym(mps_all, Kall)
    ev[1].record()
    torch.cuda.synchronize()
    exact_s = ev[0].elapsed_time(ev[1]) / 1e3
    n_pairs = N * (N - 1) // 2
    c_head, s_head = sur.head_values()
    res = {
        "workload": f"images-n{n}-r{reps}-N{N}-sym, {n_copies} near-duplicate copies (eps 1e-3..1e-1), shuffled",
        "value": n_pairs / sur_s,
        "unit": "entries/s",
        "seconds": sur_s,
        "exact_seconds": exact_s,
        "exact_value": n_pairs / exact_s,
        "speedup_vs_exact": exact_s / sur_s,
        "fallback_pairs": fb[0],
        "fallback_whole_tiles": fb[1],
        "tau": tau,
        "margin_nats": margin,
        "flagged_tiles": flagged,
        "tiles": len(upper),
        "untrained_flagged_tiles": untrained_flagged,
        "constant_flagged_tiles": constant_flagged,
        "held_out_pairs": int(dk.size),
        "held_out_pairs_K_above_1e-3": int(big.sum()),
        "held_out_max_abs_dK": float(dk.max()),
        "held_out_max_abs_dK_where_K_above_1e-3": float(dk[big].max()) if big.any() else None,
        "held_out_mean_abs_dK": float(dk.mean()),
        "held_out_log_domain": {"trained": trained, "untrained": untrained, "constant_median": constant,
                                "close_pairs": int((Lho > -100.0).sum())},
        "trained_over_constant_mean_abs_dlnK": constant["mean_abs_dlnK"] / trained["mean_abs_dlnK"],
        "trained_over_constant_close_pairs": (constant["close_pairs_mean_abs_dlnK"] / trained["close_pairs_mean_abs_dlnK"]
                                              if trained["close_pairs_mean_abs_dlnK"] else None),
        "trained_over_untrained_close_pairs": (untrained["close_pairs_mean_abs_dlnK"] / trained["close_pairs_mean_abs_dlnK"]
                                               if trained["close_pairs_mean_abs_dlnK"] else None),
        "head": {"c": c_head, "s": s_head},
        "train_pairs": int(Itr.size),
        "train_steps": rep.steps,
        "train_seconds": rep.seconds,
        "target_seconds": t_targets,
        "final_loss": rep.loss_history[-1][1] if rep.loss_history else None,
        "svm_subset": 4096,
        "svm_accuracy_exact": acc_exact,
        "svm_accuracy_surrogate": acc_sur,
        "model": f"z = [x, MLP(x)], MLP {n}->{cfg.d_h1}->{cfg.d_h2}->{cfg.d_out} GELU, bf16 weights, fp32 accumulate; "
                 "ln K_hat = -c (1 - exp(-s |z - z'|^2))",
    }
    log(f"surrogate: fallback {fb[0]} pairs one by one, {fb[1]} whole tiles")
    log(f"surrogate: {res['value']:.3e} entries/s ({sur_s*1e3:.1f} ms) vs exact {exact_s*1e3:.1f} ms; "
        f"held-out max|dK| {res['held_out_max_abs_dK']:.2e} ({int(big.sum())} pairs with K > 1e-3); "
        f"flagged {flagged} (untrained {untrained_flagged}, constant {constant_flagged}) of {len(upper)}; "
        f"|d ln K| trained {trained['mean_abs_dlnK']:.2f} untrained {untrained['mean_abs_dlnK']:.2f} "
        f"constant {constant['mean_abs_dlnK']:.2f}; SVM exact {acc_exact:.3f} surrogate {acc_sur:.3f}")
    del Kall, Kex, Lex
    torch.cuda.empty_cache()
    return res


def mlp_leg(args, rows: int = 32768, reps_timed: int = 5):
    """The surrogate's MLP kernels at the production widths 784 (padded to
    832) -> 512 -> 512 -> 256: the forward pass of 32768 rows (the whole
    surrogate workload's embedding) and one training step of 8192 pairs
    (16384 rows: gather, forward, log-domain head, backward with split-K
    weight gradients, AdamW), timed with HIP events; the GEMMs' BF16 flop rate
    against the 2.5 PFLOP/s dense BF16 peak."""
    import numpy as np
    import torch

    from paper_2405_02630_amd import qsvm, synth
    from paper_2405_02630_amd.surrogate import Surrogate, SurrogateConfig

    dev = torch.device("cuda:0")
    wl = synth.images784(seed=8, n_train=rows, n_test=0, reps=2)
    X = torch.as_tensor(wl.X, device=dev)
    sur = Surrogate(784, SurrogateConfig())
    sur.embed(X)  # warm-up, buffers
    torch.cuda.synchronize()
    ev = _events(2)
    ev[0].record()
    for _ in range(reps_timed):
        sur.embed(X)
    ev[1].record()
    torch.cuda.synchronize()
    fwd_s = ev[0].elapsed_time(ev[1]) / 1e3 / reps_timed
    dims = (sur.d_in, sur.cfg.d_h1, sur.cfg.d_h2, sur.cfg.d_out)
    fwd_flops = 2.0 * rows * (dims[0] * dims[1] + dims[1] * dims[2] + dims[2] * dims[3])
    rng = np.random.default_rng(3)
    P = sur.cfg.pairs_per_step
    ii, jj = rng.integers(0, rows, P), rng.integers(0, rows, P)
    tgt = np.full(P, -500.0)
    sur._pair_pass(X, ii, jj, tgt, train=True)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps_timed):
        sur._pair_pass(X, ii, jj, tgt, train=True)
    ev[1].record()
    torch.cuda.synchronize()
    step_s = ev[0].elapsed_time(ev[1]) / 1e3 / reps_timed
    # forward + backward GEMM flops of one step: forward 1x, activation and weight gradients 2x
    # (the first layer has no activation gradient)
    r2 = 2 * P
    step_flops = 2.0 * r2 * (3 * dims[0] * dims[1] - dims[0] * dims[1] + 3 * dims[1] * dims[2] + 3 * dims[2] * dims[3])
    res = {
        "widths": list(dims),
        "forward_rows": rows,
        "forward_ms": fwd_s * 1e3,
        "forward_gemm_tflops": fwd_flops / fwd_s / 1e12,
        "forward_frac_of_bf16_peak": fwd_flops / fwd_s / 1e12 / PEAK_BF16_MATRIX_TFLOPS,
        "train_step_pairs": P,
        "train_step_ms": step_s * 1e3,
        "train_step_gemm_tflops": step_flops / step_s / 1e12,
    }
    log(f"mlp: forward {rows} rows {fwd_s*1e3:.3f} ms ({res['forward_gemm_tflops']:.0f} TFLOP/s of GEMMs, "
        f"{res['forward_frac_of_bf16_peak']:.3f} of peak); train step {step_s*1e3:.3f} ms")
    return res


def surrogate_gram_only(N: int):
    """The prediction Gram alone: N synthetic embeddings z = [x (832 wide, uniform
    pixels in [0, 1]), e (256 wide, N(0, 0.01))] in BF16, head (c, s) = (30, 0.2);
    two warm-up and five timed calls of qsvm_surrogate_gram_log, then three
    timed plain fills of the same FP64 K (its write bound)."""
    import torch

    from paper_2405_02630_amd import qsvm

    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(0)
    Np = (N + 63) // 64 * 64
    X16 = torch.rand((Np, 832), device=dev, generator=g).to(torch.bfloat16)
    E16 = (torch.randn((Np, 256), device=dev, generator=g) * 0.1).to(torch.bfloat16)
    head = torch.tensor([math.log(30.0), math.log(0.2)], dtype=torch.float32, device=dev)
    K = torch.empty((N, N), dtype=torch.float64, device=dev)
    T = Np // 64
    tile_max = torch.empty(T * T, dtype=torch.float32, device=dev)
    for _ in range(2):
        qsvm.qsvm_surrogate_gram_log(X16, E16, N, head, K, tile_max)
    torch.cuda.synchronize()
    ev = _events(2)
    gram_ms = []
    for _ in range(5):
        ev[0].record()
        qsvm.qsvm_surrogate_gram_log(X16, E16, N, head, K, tile_max)
        ev[1].record()
        torch.cuda.synchronize()
        gram_ms.append(ev[0].elapsed_time(ev[1]))
    fill_ms = []
    for _ in range(3):
        ev[0].record()
        K.fill_(0.5)
        ev[1].record()
        torch.cuda.synchronize()
        fill_ms.append(ev[0].elapsed_time(ev[1]))
    return {"surrogate_gram_only": N, "K_bytes": N * N * 8, "gram_ms": [round(x, 4) for x in gram_ms],
            "fill_ms": [round(x, 4) for x in fill_ms]}


def svm_accuracies(K_exact, K_sur, labels, n_train_frac=0.75):
    """One-vs-rest SVM on a precomputed Gram: train on the first 75 %, test on the rest."""
    import numpy as np
    from sklearn.multiclass import OneVsRestClassifier
    from sklearn.svm import SVC

    M = K_exact.shape[0]
    tr = np.arange(int(M * n_train_frac))
    te = np.arange(int(M * n_train_frac), M)
    accs = []
    for K in (K_exact, K_sur):
        clf = OneVsRestClassifier(SVC(kernel="precomputed", C=1.0))
        clf.fit(K[np.ix_(tr, tr)], labels[tr])
        accs.append(float(np.mean(clf.predict(K[np.ix_(te, tr)]) == labels[te])))
    return accs[0], accs[1]


def batched_leg():
    """64 uneven jobs: one persistent hipGraph launch vs one launch per job,
    with the built-in work-item shape and after autotuning every (reps, n) of
    the mix (the tuned table also sets the variant of the one-launch-per-job
    calls)."""
    import numpy as np
    import torch

    from paper_2405_02630_amd import qsvm, synth

    dev = torch.device("cuda:0")
    wl = synth.uneven_jobs(seed=0)
    jobs = []
    for w in wl:
        m = qsvm.qsvm_encode_mps(torch.as_tensor(w.X, device=dev), w.reps)
        K = torch.empty((m.N, m.N), dtype=torch.float64, device=dev)
        jobs.append((m, K, None))
    pairs = [m.N * (m.N - 1) // 2 for m, _, _ in jobs]

    def time_plan(plan):
        plan.launch()
        torch.cuda.synchronize()
        ev = _events(2)
        ev[0].record()
        for _ in range(3):
            plan.launch()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / 3e3

    def time_per_job():
        for m, K, _ in jobs:
            qsvm.qsvm_gram_sym(m, K)
        torch.cuda.synchronize()
        per_job = []
        ev_all = _events(2)
        ev_all[0].record()
        for m, K, _ in jobs:
            e = _events(2)
            e[0].record()
            qsvm.qsvm_gram_sym(m, K)
            e[1].record()
            per_job.append(e)
        ev_all[1].record()
        torch.cuda.synchronize()
        return ev_all[0].elapsed_time(ev_all[1]) / 1e3, [p / (e[0].elapsed_time(e[1]) / 1e3) for p, e in zip(pairs, per_job)]

    # built-in defaults: variant 0 everywhere, 2 / 1 ket points per lane in the plan
    # one entry per (reps, n bucket, N bucket) of the mix, tuned at the bucket's
    # largest N that occurs (so the tuning problem is the size of a real job)
    shapes = {}
    for m, _, _ in jobs:
        key = (m.reps, m.n, m.N.bit_length() - 1)
        shapes[key] = max(shapes.get(key, 0), m.N)
    for (r, n, _), N in shapes.items():
        qsvm.qsvm_set_tuned_variant(r, n, N, 0)
    plan = qsvm.BatchPlan(jobs, use_graph=True, item_pi2=2, item_pi3=1)
    total_items, grid, _ = plan.info()
    default_s = time_plan(plan)
    plan.close()
    default_serial_s, _ = time_per_job()
    # autotune every (reps, n) of the mix on a 1024-point synthetic Gram
    tuned = {}
    t0 = time.perf_counter()
    for (r, n, _), N in sorted(shapes.items()):
        best, ms = qsvm.qsvm_autotune(r, n, N)
        tuned[f"r{r}_n{n}_N{N}"] = {"variant": best, "ms_per_variant": [round(x, 4) for x in ms]}
    tune_s = time.perf_counter() - t0
    plan = qsvm.BatchPlan(jobs, use_graph=True)
    shape = plan.shape()
    batched_s = time_plan(plan)
    plan.close()
    serial_s, job_rates = time_per_job()
    # executed sweep flops of all jobs (the same per-pair count as the roofline entry)
    flops = sum(p * sweep_flops_per_pair(m.n, m.reps, "butterfly") for p, (m, _, _) in zip(pairs, jobs))
    res = {
        "workload": "64 jobs, n in {16,64,196,400,784}, N in [64,2048], reps in {2,3}, uniform features",
        "jobs": len(jobs),
        "pairs": int(sum(pairs)),
        "work_items": total_items,
        "persistent_blocks": grid,
        "value": sum(pairs) / batched_s,
        "unit": "entries/s",
        "seconds": batched_s,
        "one_launch_per_job_value": sum(pairs) / serial_s,
        "one_launch_per_job_seconds": serial_s,
        "speedup": serial_s / batched_s,
        "sweep_flops": flops,
        "frac_of_fp32_peak": flops / batched_s / 1e12 / PEAK_FP32_VECTOR_TFLOPS,
        "one_launch_per_job_frac_of_fp32_peak": flops / serial_s / 1e12 / PEAK_FP32_VECTOR_TFLOPS,
        "per_job_entries_per_s": {"min": float(np.min(job_rates)), "median": float(np.median(job_rates)),
                                  "max": float(np.max(job_rates))},
        "tuned_item_shape": {"pi2": shape[0], "pi3": shape[1]},
        "default": {"seconds": default_s, "value": sum(pairs) / default_s,
                    "one_launch_per_job_seconds": default_serial_s, "item_shape": {"pi2": 2, "pi3": 1}},
        "tuned_over_default": default_s / batched_s,
        "autotune_seconds": tune_s,
        "autotune": tuned,
        "autotune_cache": qsvm.qsvm_autotune_cache_path(),
    }
    log(f"batched: {res['value']:.3e} entries/s ({batched_s*1e3:.1f} ms, {res['frac_of_fp32_peak']:.3f} of peak, "
        f"shape {shape}) vs default {default_s*1e3:.1f} ms vs one launch per job {serial_s*1e3:.1f} ms "
        f"(default variants {default_serial_s*1e3:.1f} ms)")
    return res


PEAK_FP64_MATRIX_TFLOPS = 78.6  # MI355X dense FP64 MFMA
PEAK_BF16_MATRIX_TFLOPS = 2500.0  # MI355X dense BF16 MFMA


def sv_leg(points: int = 512, qubits=(12, 16, 20), reps: int = 2):
    """State-vector engine vs MPS engine on the same points (uniform features):
    build + symmetric Gram time of each, their agreement, and the roofline of
    the state-vector Gram (FP64 MFMA, 6 executed flops per complex multiply-add)."""
    import numpy as np
    import torch

    from paper_2405_02630_amd import qsvm, synth

    dev = torch.device("cuda:0")
    rows = []
    for n in qubits:
        X = torch.as_tensor(synth.uniform_features(points, n, seed=6000 + n), device=dev)
        Ks = torch.empty((points, points), dtype=torch.float64, device=dev)
        Km = torch.empty_like(Ks)
        sv = qsvm.qsvm_encode_sv(X, reps)
        m = qsvm.qsvm_encode_mps(X, reps)
        qsvm.qsvm_sv_gram_sym(sv, Ks)
        qsvm.qsvm_gram_sym(m, Km)
        torch.cuda.synchronize()
        ev = _events(6)
        ev[0].record()
        qsvm.qsvm_encode_sv(X, reps, out=sv.buf)
        ev[1].record()
        qsvm.qsvm_sv_gram_sym(sv, Ks)
        ev[2].record()
        qsvm.qsvm_encode_mps(X, reps, out=m.buf)
        ev[3].record()
        qsvm.qsvm_gram_sym(m, Km)
        ev[4].record()
        torch.cuda.synchronize()
        enc_s = ev[0].elapsed_time(ev[1]) / 1e3
        gram_s = ev[1].elapsed_time(ev[2]) / 1e3
        mps_s = ev[2].elapsed_time(ev[4]) / 1e3
        pairs = points * (points - 1) // 2
        T = (points + 63) // 64
        # executed GEMM flops: the upper-triangular 64 x 64 tiles, 6 flops per complex
        # MAC (the 3M form: three real multiply-adds)
        flops = T * (T + 1) // 2 * 64 * 64 * (1 << n) * 6
        rows.append({
            "n_qubits": n,
            "sv_encode_ms": enc_s * 1e3,
            "sv_gram_ms": gram_s * 1e3,
            "sv_entries_per_s": pairs / (enc_s + gram_s),
            "mps_entries_per_s": pairs / mps_s,
            "mps_over_sv": (enc_s + gram_s) / mps_s,
            "max_abs_dK_sv_vs_mps": float((Ks - Km).abs().max().item()),
            "sv_gram_fp64_tflops": flops / gram_s / 1e12,
            "sv_gram_frac_of_fp64_matrix_peak": flops / gram_s / 1e12 / PEAK_FP64_MATRIX_TFLOPS,
        })
        log(f"sv n={n}: encode {enc_s*1e3:.2f} ms, gram {gram_s*1e3:.2f} ms "
            f"({rows[-1]['sv_gram_fp64_tflops']:.1f} FP64 TFLOP/s); mps {mps_s*1e3:.2f} ms; "
            f"max|dK| {rows[-1]['max_abs_dK_sv_vs_mps']:.1e}")
        del sv, Ks, Km
        torch.cuda.empty_cache()
    return {"workload": f"{points} points, uniform features, reps={reps}, symmetric Gram", "points": points,
            "unit": "entries/s", "peak_fp64_matrix_tflops": PEAK_FP64_MATRIX_TFLOPS, "by_qubits": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--n-train", type=int, default=4096)
    ap.add_argument("--sweep", choices=["butterfly", "dense"], default="butterfly")
    ap.add_argument("--renorm-every", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=720)
    ap.add_argument("--legs", default="exact,reps3,mixture64,deep,refine_worst,mlp,surrogate,batched,sv")  # "exact" adds the test x train Gram
    ap.add_argument("--sur-points", type=int, default=32768)
    ap.add_argument("--sur-steps", type=int, default=600)
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="run only a plain device copy of this many MiB (for HBM counter scaling)")
    ap.add_argument("--surrogate-gram-only", type=int, default=0, metavar="N",
                    help="run only the surrogate's prediction Gram (qsvm_surrogate_gram_log) on N synthetic "
                         "embeddings of the production widths, 5 timed calls, and a plain fill of the same K "
                         "(for its kernel's counters and write bound)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 "
                                   "(sharding across GPUs is not implemented)"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2405_02630_amd import qsvm, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).uniform_()
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 3}))
        return
    if args.surrogate_gram_only:
        print(json.dumps(surrogate_gram_only(args.surrogate_gram_only)))
        return

    reps = args.reps
    wl = synth.images784(seed=0, n_train=args.n_train, n_test=0, reps=reps)
    N, n = wl.X.shape
    X = torch.as_tensor(wl.X, dtype=torch.float64, device=dev)
    mps_bytes = qsvm.qsvm_mps_bytes(N, n, reps)
    mps_buf = torch.empty(mps_bytes, dtype=torch.uint8, device=dev)
    K = torch.empty((N, N), dtype=torch.float64, device=dev)
    sweep = qsvm.SWEEP_BUTTERFLY if args.sweep == "butterfly" else qsvm.SWEEP_DENSE
    stream = torch.cuda.current_stream()

    dense_buf = (torch.empty(qsvm.qsvm_dense_bytes(N, n, reps), dtype=torch.uint8, device=dev)
                 if sweep == qsvm.SWEEP_DENSE else None)

    def step(ev_mid=None):
        m = qsvm.qsvm_encode_mps(X, reps, out=mps_buf)
        if dense_buf is not None:  # the dense sweep reads the dense tensors
            m.dense = qsvm.qsvm_encode_dense(X, reps, out=dense_buf)
        if ev_mid is not None:
            ev_mid[0].record(stream)
        qsvm.qsvm_gram_sym(m, K, sweep=sweep, renorm_every=args.renorm_every)
        if ev_mid is not None:
            ev_mid[1].record(stream)

    log(f"workload images-n{n}-r{reps}-train{N}: warmup {args.warmup}, steps {args.steps}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(evs[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    sweep_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    pairs = N * (N - 1) // 2
    value = pairs / (ms_per_step / 1e3)
    log(f"{ms_per_step:.3f} ms/step, sweep {sweep_ms:.3f} ms, {value:.4e} entries/s")

    flops = sweep_flops_per_pair(n, reps, args.sweep) * pairs
    achieved = flops / (sweep_ms / 1e3) / 1e12
    # counters were taken for the default kernel variant and renormalisation
    traffic = (MEASURED_TRAFFIC.get((args.sweep, reps, N, n), (None, None)) if args.renorm_every == 0
               else (None, None))
    roofline = {
        "bound": "alu",
        "achieved": round(achieved, 3),
        "peak": PEAK_FP32_VECTOR_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
        "traffic": traffic[0],
        "traffic_source": traffic[1],
        "kernel": (f"sweep_split_kernel<{reps},*>" if args.sweep == "butterfly" and reps >= 4
                   else f"sweep_{args.sweep}_kernel<{reps},*>"),
        "flops_per_launch": flops,
        "avg_launch_ms": round(sweep_ms, 4),
    }

    out = {
        "metric": "Gram entries/sec at 784 qubits, reps=2 (exact vs surrogate) at max|dK|<=1e-5",
        "value": value,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"images-n{n}-r{reps}-train{N}-sym",
            "n_qubits": n,
            "reps": reps,
            "points": N,
            "pairs_per_step": pairs,
            "step": "encode MPS + symmetric Gram (pairs i<j), features resident in HBM",
            "sweep": args.sweep,
        },
        "roofline": roofline,
    }

    legs = set(args.legs.split(","))
    if "exact" in legs:
        out["test_by_train"] = test_by_train_leg(reps, N, mps_buf, X, sweep, args)
    if "reps3" in legs and reps == 2:
        out["reps3"] = exact_reps_leg(3, N, args)
    if "deep" in legs:
        # the split sweep at bond dimensions 16, 32 and 64 (symmetric Grams of
        # 2048, 1024 and 512 images; at most 3 timed steps each)
        out["deep_reps"] = {f"reps{r}": exact_reps_leg(r, pts, args, kinds=("sym",), steps=min(args.steps, 3))["sym"]
                            for r, pts in ((4, 2048), (5, 1024), (6, 512))}
    if "mixture64" in legs:
        out["mixture64"] = mixture64_leg(args)
    if "refine_worst" in legs:
        out["refine_worst"] = refine_worst_leg(args)
    if "mlp" in legs:
        out["mlp"] = mlp_leg(args)
    if "surrogate" in legs:
        del K  # release the exact leg's buffers first
        torch.cuda.empty_cache()
        out["surrogate"] = surrogate_leg(args, exact_rate=value)
        K = None
    if "batched" in legs:
        out["batched"] = batched_leg()
    if "sv" in legs:
        out["state_vector"] = sv_leg()

    if not args.no_cpu_baseline:
        dense_t = None if dense_buf is None else qsvm.qsvm_encode_dense(X, reps, out=dense_buf)
        if K is None:
            K = torch.empty((N, N), dtype=torch.float64, device=dev)
            m = qsvm.qsvm_encode_mps(X, reps, out=mps_buf)
            m.dense = dense_t
            qsvm.qsvm_gram_sym(m, K, sweep=sweep)
        Kh = K.cpu().numpy()
        cores = max(1, min(16, os.cpu_count() or 1))
        log(f"cpu baseline: oracle on {args.cpu_sample} points with {cores} processes")
        cb = cpu_baseline(wl.X, reps, Kh, args.cpu_sample, cores)
        # sampled parity of the timed GPU result against the oracle
        ia, jb = cb.pop("_pairs")
        lk = cb.pop("_lk")
        L = torch.empty_like(K)
        m = qsvm.qsvm_encode_mps(X, reps, out=mps_buf)
        m.dense = dense_t
        qsvm.qsvm_gram_sym(m, K, log_k=L, sweep=sweep, renorm_every=args.renorm_every)
        Lh = L.cpu().numpy()
        cb["sample_max_log_err_vs_gpu"] = float(np.max(np.abs(Lh[ia, jb] - lk)))
        cb["near_duplicates"] = near_duplicate_check(reps, cores)
        log(f"near duplicates: max|dK| {cb['near_duplicates']['max_abs_dK']:.2e} over "
            f"{cb['near_duplicates']['pairs']} pairs, K up to {cb['near_duplicates']['K_oracle_max']:.3f}")
        if "refine_worst" in out:
            acc = refine_worst_accuracy(out["refine_worst"]["_samples"], cores)
            out["refine_worst"].update(acc)
            log(f"refine worst case: sample max|dK| {acc['refined_sample_max_abs_dK']:.2e} refined, "
                f"{acc['fp32_only_sample_max_abs_dK']:.2e} FP32 only (K >= {acc['K_oracle_min_sample']:.3f})")
        out["cpu_baseline"] = cb
    if "refine_worst" in out:
        out["refine_worst"].pop("_samples", None)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
