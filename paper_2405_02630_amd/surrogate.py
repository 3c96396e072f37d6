"""Learned surrogate of the quantum kernel, trained on exact entries.

An MLP embedding f: R^n -> R^d_out (widths n -> 512 -> 512 -> 256 by default,
GELU after the hidden layers, BF16 weights and activations, FP32 master
weights and accumulation) predicts kernel entries as
    K_hat(x, y) = sigmoid(alpha <f(x), f(y)> + beta).
It is trained with AdamW on exact kernel entries computed by the MPS sweep.
At prediction time the whole N x N surrogate Gram is one BF16 matrix-core
GEMM with a sigmoid epilogue; every 64 x 64 tile whose largest off-diagonal
K_hat reaches the threshold tau is recomputed exactly (the exact sweep is
the fallback), and K_ii = 1.

This module only orchestrates: it allocates device buffers with PyTorch,
draws training pairs on the host (a seeded data loader) and calls the HIP
kernels of libqsvm.so through the binding for every arithmetic step.
"""

from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import qsvm


def _round_up(x: int, m: int) -> int:
    return (x + m - 1) // m * m


@dataclass
class SurrogateConfig:
    d_h1: int = 512
    d_h2: int = 512
    d_out: int = 256
    lr: float = 1e-3
    lr_head: float = 1e-2       # learning rate of alpha and beta
    weight_decay: float = 1e-4
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    pairs_per_step: int = 8192  # multiple of 32 (2 rows per pair, rows in multiples of 64)
    loss: int = qsvm.LOSS_BCE
    tau: float = 1e-6           # fallback threshold on the largest off-diagonal K_hat of a tile
    seed: int = 0


@dataclass
class FitReport:
    steps: int
    seconds: float
    loss_history: list = field(default_factory=list)


class _Param:
    """FP32 master tensor, its AdamW moments, gradient and BF16 copy."""

    def __init__(self, host: np.ndarray, dev, bf16: bool):
        import torch

        self.w = torch.as_tensor(np.ascontiguousarray(host, dtype=np.float32), device=dev)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.g = torch.zeros_like(self.w)
        self.w16 = torch.empty(self.w.shape, dtype=torch.bfloat16, device=dev) if bf16 else None


class Surrogate:
    def __init__(self, n_features: int, cfg: SurrogateConfig | None = None, device="cuda:0"):
        import torch

        self.cfg = cfg or SurrogateConfig()
        c = self.cfg
        self.n = n_features
        self.d_in = _round_up(n_features, 64)
        self.dev = torch.device(device)
        rng = np.random.default_rng(c.seed)

        def he(fan_in, fan_out, gain=2.0):
            return rng.normal(0.0, math.sqrt(gain / fan_in), (fan_in, fan_out))

        W1 = he(self.d_in, c.d_h1)
        W1[n_features:] = 0.0  # padded input columns carry no weight
        self.params = [
            _Param(W1, self.dev, True), _Param(np.zeros(c.d_h1), self.dev, False),
            _Param(he(c.d_h1, c.d_h2), self.dev, True), _Param(np.zeros(c.d_h2), self.dev, False),
            _Param(he(c.d_h2, c.d_out, gain=1.0), self.dev, True), _Param(np.zeros(c.d_out), self.dev, False),
        ]
        self.head = _Param(np.array([1.0 / c.d_out, 0.0]), self.dev, False)  # (alpha, beta)
        self.step = 0
        # BF16 copies of the initial weights: an AdamW step with lr = 0 and zero gradient
        for p in self.params:
            if p.w16 is not None:
                qsvm.qsvm_adamw(p.w, p.g, p.m, p.v, p.w16, 0.0, c.beta1, c.beta2, c.eps, 0.0, 1)
        self._bufs = {}

    # ------------------------------------------------------------------
    def net(self) -> qsvm.Mlp:
        W1, b1, W2, b2, W3, b3 = self.params
        return qsvm.Mlp(self.d_in, self.cfg.d_h1, self.cfg.d_h2, self.cfg.d_out,
                        W1.w16.data_ptr(), b1.w.data_ptr(), W2.w16.data_ptr(), b2.w.data_ptr(),
                        W3.w16.data_ptr(), b3.w.data_ptr())

    def _buffers(self, rows: int):
        import torch

        if rows in self._bufs:
            return self._bufs[rows]
        c = self.cfg
        f32, b16 = torch.float32, torch.bfloat16
        b = {
            "X16": torch.empty((rows, self.d_in), dtype=b16, device=self.dev),
            "H1": torch.empty((rows, c.d_h1), dtype=f32, device=self.dev),
            "A1": torch.empty((rows, c.d_h1), dtype=b16, device=self.dev),
            "H2": torch.empty((rows, c.d_h2), dtype=f32, device=self.dev),
            "A2": torch.empty((rows, c.d_h2), dtype=b16, device=self.dev),
            "E": torch.empty((rows, c.d_out), dtype=f32, device=self.dev),
            "E16": torch.empty((rows, c.d_out), dtype=b16, device=self.dev),
            "dE16": torch.empty((rows, c.d_out), dtype=b16, device=self.dev),
            "dH1": torch.empty((rows, c.d_h1), dtype=b16, device=self.dev),
            "dH2": torch.empty((rows, c.d_h2), dtype=b16, device=self.dev),
            "partial": torch.empty(3 * (rows // 2), dtype=f32, device=self.dev),
            "out3": torch.zeros(3, dtype=f32, device=self.dev),
            "idx": torch.empty(rows, dtype=torch.int32, device=self.dev),
            "target": torch.empty(rows // 2, dtype=f32, device=self.dev),
        }
        b["ws"] = torch.empty(max(1, qsvm.qsvm_mlp_workspace_floats(self.net(), rows)), dtype=f32, device=self.dev)
        self._bufs[rows] = b
        return b

    def _acts(self, b) -> qsvm.MlpActs:
        return qsvm.MlpActs(b["H1"].data_ptr(), b["A1"].data_ptr(), b["H2"].data_ptr(), b["A2"].data_ptr(),
                            b["E"].data_ptr(), b["E16"].data_ptr())

    def _grads(self, b) -> qsvm.MlpGrads:
        p = self.params
        return qsvm.MlpGrads(p[0].g.data_ptr(), p[1].g.data_ptr(), p[2].g.data_ptr(), p[3].g.data_ptr(),
                             p[4].g.data_ptr(), p[5].g.data_ptr(), b["dH1"].data_ptr(), b["dH2"].data_ptr(),
                             b["ws"].data_ptr(), b["ws"].numel())

    # ------------------------------------------------------------------
    def init_head_from_targets(self, mean_target: float) -> None:
        """beta := log-odds of the mean training target (clipped to [-20, 20])."""
        t = min(max(mean_target, 1e-300), 1.0 - 1e-12)
        beta = float(np.clip(math.log(t) - math.log1p(-t), -20.0, 20.0))
        self.head.w[1].fill_(beta)

    def train_step(self, X, idx_host: np.ndarray, target_host: np.ndarray) -> None:
        """One AdamW step on pairs (idx[p], idx[P + p]) with exact targets."""
        import torch

        c = self.cfg
        P = target_host.shape[0]
        rows = 2 * P
        b = self._buffers(rows)
        b["idx"].copy_(torch.from_numpy(idx_host.astype(np.int32)))
        b["target"].copy_(torch.from_numpy(target_host.astype(np.float32)))
        qsvm.qsvm_gather_features(X, b["idx"], self.d_in, b["X16"])
        net = self.net()
        acts = self._acts(b)
        qsvm.qsvm_mlp_forward(net, b["X16"], rows, acts)
        qsvm.qsvm_pair_head(b["E"], P, c.d_out, b["target"], self.head.w, b["dE16"], b["partial"], b["out3"],
                            loss_kind=c.loss)
        qsvm.qsvm_mlp_backward(net, b["X16"], acts, b["dE16"], rows, self._grads(b))
        self.step += 1
        for p in self.params:
            qsvm.qsvm_adamw(p.w, p.g, p.m, p.v, p.w16, c.lr, c.beta1, c.beta2, c.eps, c.weight_decay, self.step)
        # head gradient = out3[1:3]
        qsvm.qsvm_adamw(self.head.w, b["out3"][1:], self.head.m, self.head.v, None, c.lr_head, c.beta1, c.beta2,
                        c.eps, 0.0, self.step)

    def last_loss(self, pairs: int) -> float:
        return float(self._buffers(2 * pairs)["out3"][0].item())

    def fit(self, X, train_points: np.ndarray, K_train: np.ndarray, steps: int, log_every: int = 50) -> FitReport:
        """Train on the exact Gram K_train of the points train_points (host arrays)."""
        import torch

        c = self.cfg
        P = c.pairs_per_step
        if P % 32:
            raise ValueError("pairs_per_step must be a multiple of 32")
        S = train_points.shape[0]
        rng = np.random.default_rng(c.seed + 1)
        iu = np.triu_indices(S, 1)
        self.init_head_from_targets(float(np.mean(K_train[iu])))
        hist = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            i = rng.integers(0, S, P)
            j = rng.integers(0, S - 1, P)
            j = j + (j >= i)
            idx = np.concatenate([train_points[i], train_points[j]])
            self.train_step(X, idx, K_train[i, j])
            if log_every and (s % log_every == 0 or s == steps - 1):
                hist.append((s, self.last_loss(P)))
        torch.cuda.synchronize()
        return FitReport(steps, time.perf_counter() - t0, hist)

    # ------------------------------------------------------------------
    def embed(self, X, chunk: int = 32768):
        """BF16 embeddings of every row of X, padded to a multiple of 64 rows."""
        import torch

        N = X.shape[0]
        Np = _round_up(N, 64)
        E16 = torch.empty((Np, self.cfg.d_out), dtype=torch.bfloat16, device=self.dev)
        net = self.net()
        for r0 in range(0, Np, chunk):
            rows = min(chunk, Np - r0)
            b = self._buffers(rows)
            torch.arange(r0, r0 + rows, out=b["idx"])  # on the device; rows >= N are zero padding
            qsvm.qsvm_gather_features(X, b["idx"], self.d_in, b["X16"])
            qsvm.qsvm_mlp_forward(net, b["X16"], rows, self._acts(b))
            E16[r0:r0 + rows].copy_(b["E16"])
        return E16

    def gram(self, X, mps: "qsvm.MPS | None", K=None, tau: float | None = None):
        """Surrogate Gram of the rows of X with exact fallback on flagged tiles.

        Returns (K, flagged): flagged is a 1-element device int32 tensor, the
        number of flagged tiles.  mps (the exact MPS of the same points) feeds
        the fallback; pass None to skip it.  Nothing here waits for the GPU:
        the fallback reads the flagged count on the device."""
        import torch

        tau = self.cfg.tau if tau is None else tau
        N = X.shape[0]
        E16 = self.embed(X)
        Np = E16.shape[0]
        T = Np // 64
        if K is None:
            K = torch.empty((N, N), dtype=torch.float64, device=self.dev)
        tile_max = torch.empty(T * T, dtype=torch.float32, device=self.dev)
        qsvm.qsvm_surrogate_gram(E16, N, self.head.w, K, tile_max)
        tiles = torch.empty(T * (T + 1), dtype=torch.int32, device=self.dev)
        count = torch.empty(1, dtype=torch.int32, device=self.dev)
        qsvm.qsvm_flag_tiles(tile_max, T, tau, tiles, count)  # clears count first
        if mps is not None:
            qsvm.qsvm_gram_sym_tiles_dev(mps, tiles, count, T * (T + 1) // 2, K)
        return K, count
