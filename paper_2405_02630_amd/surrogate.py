"""Learned surrogate of the quantum kernel, trained on exact entries.

An MLP f: R^n -> R^d_out (widths n -> 512 -> 512 -> 256 by default, GELU
after the hidden layers, BF16 weights and activations, FP32 master weights
and accumulation) extends each point to the embedding z(x) = [x, f(x)], and
the kernel is predicted in the log domain from the embeddings' squared
distance d2 = ||z(x) - z(y)||^2 (their inner products and norms):

    ln K_hat(x, y) = -c (1 - exp(-s d2)),     c = exp(head[0]), s = exp(head[1]).

ln K_hat is 0 for identical points (K_ii = 1 needs no special case), -c s d2
for close ones, and saturates at -c for unrelated ones: at hundreds of qubits
kernel values of unrelated points concentrate at a tiny level (the vanishing
off-diagonal kernels of §4.2.1, ln K ~ -585 for 784-pixel images at two
repetitions), which no bounded K-domain predictor can represent, so both
training and judging are in the log domain.  The network is trained with
AdamW on the exact ln K that the MPS sweep exports (qsvm_gram_opts.log_k).

Prediction: one BF16 matrix-core Gram of the embeddings with the head in
its epilogue gives K_hat for all pairs and the largest off-diagonal ln K_hat
per 64 x 64 tile; every tile whose maximum reaches ln(tau) - margin is
recomputed by the exact sweep (the fallback), where margin bounds how far
the network under-predicts ln K (the largest ln K - ln K_hat over calibration
pairs with exact targets).  Entries left to the network are then below tau
both in K_hat and, up to the calibration, in K.

This module only orchestrates: it allocates device buffers with PyTorch,
draws training pairs on the host (a seeded data loader) and calls the HIP
kernels of libqsvm.so through the binding for every arithmetic step.
"""

from __future__ import annotations

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
    lr_head: float = 1e-2       # learning rate of (log c, log s)
    weight_decay: float = 1e-4
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    pairs_per_step: int = 8192  # multiple of 32 (2 rows per pair, rows in multiples of 64)
    out_init: float = 0.1       # output layer initialised at this fraction of its He scale (z starts near [x, 0])
    loss_scale: float = 0.0     # the loss divides ln K errors by this; 0 = the number of features
    high_log_k: float = -100.0  # training pairs above this ln K form the "close pairs" stratum ...
    high_fraction: float = 0.125  # ... from which this share of every minibatch is drawn
    tau: float = 1e-6           # fallback when a tile's largest K_hat may reach tau
    pair_cap: int = 256         # exact fallback per pair for tiles with at most this many flagged pairs
                                # (0: whole flagged tiles only)
    max_fallback_pairs: int = 1 << 20  # room of the pair list (tiles whose pairs do not fit fall back whole)
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


class _ParamSet:
    """Several parameters in one flat FP32 buffer (each a view), with flat
    AdamW moments, gradients and BF16 copies: one AdamW launch updates them
    all (the same hyper-parameters apply to every tensor)."""

    def __init__(self, hosts, dev):
        import torch

        sizes = [int(np.asarray(h).size) for h in hosts]
        total = sum(sizes)
        self.w = torch.empty(total, dtype=torch.float32, device=dev)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.g = torch.zeros_like(self.w)
        self.w16 = torch.empty(total, dtype=torch.bfloat16, device=dev)
        self.views = []
        off = 0
        for h, n in zip(hosts, sizes):  # offsets stay multiples of 8 (the widths are multiples of 64)
            h = np.asarray(h, dtype=np.float32)
            self.w[off:off + n].copy_(torch.from_numpy(np.ascontiguousarray(h).ravel()))
            view = _Param.__new__(_Param)
            view.w = self.w[off:off + n].view(h.shape)
            view.m = self.m[off:off + n].view(h.shape)
            view.v = self.v[off:off + n].view(h.shape)
            view.g = self.g[off:off + n].view(h.shape)
            view.w16 = self.w16[off:off + n].view(h.shape)
            self.views.append(view)
            off += n


class Surrogate:
    def __init__(self, n_features: int, cfg: SurrogateConfig | None = None, device="cuda:0"):
        import torch

        self.cfg = cfg or SurrogateConfig()
        c = self.cfg
        self.fallback = None  # device counts (pairs, whole tiles) of the last gram() fallback
        self.n = n_features
        self.d_in = _round_up(n_features, 64)
        self.dev = torch.device(device)
        self.scale = c.loss_scale if c.loss_scale > 0 else float(n_features)
        rng = np.random.default_rng(c.seed)

        def he(fan_in, fan_out, gain=2.0):
            return rng.normal(0.0, math.sqrt(gain / fan_in), (fan_in, fan_out))

        W1 = he(self.d_in, c.d_h1)
        W1[n_features:] = 0.0  # padded input columns carry no weight
        self.pset = _ParamSet([W1, np.zeros(c.d_h1), he(c.d_h1, c.d_h2), np.zeros(c.d_h2),
                               c.out_init * he(c.d_h2, c.d_out, gain=1.0), np.zeros(c.d_out)], self.dev)
        self.params = self.pset.views  # W1, b1, W2, b2, W3, b3
        self.head = _Param(np.array([0.0, 0.0]), self.dev, False)  # (log c, log s), set by init_head
        self.margin = 0.0
        self.step = 0
        # BF16 copies of the initial weights: an AdamW step with lr = 0 and zero gradient
        ps = self.pset
        qsvm.qsvm_adamw(ps.w, ps.g, ps.m, ps.v, ps.w16, 0.0, c.beta1, c.beta2, c.eps, 0.0, 1)
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
            "pred": torch.empty(rows, dtype=f32, device=self.dev),
            "idx": torch.empty(rows, dtype=torch.int32, device=self.dev),
            "target": torch.empty(rows // 2, dtype=f32, device=self.dev),
        }
        b["ws"] = torch.empty(max(1, qsvm.qsvm_mlp_workspace_floats(self.net(), rows)), dtype=f32, device=self.dev)
        self._bufs[rows] = b
        return b

    def _acts(self, b, E16=None, inference=False) -> qsvm.MlpActs:
        if inference:  # BF16 outputs only: no FP32 pre-activations for a backward pass
            return qsvm.MlpActs(None, b["A1"].data_ptr(), None, b["A2"].data_ptr(), None,
                                (b["E16"] if E16 is None else E16).data_ptr())
        return qsvm.MlpActs(b["H1"].data_ptr(), b["A1"].data_ptr(), b["H2"].data_ptr(), b["A2"].data_ptr(),
                            b["E"].data_ptr(), (b["E16"] if E16 is None else E16).data_ptr())

    def _grads(self, b) -> qsvm.MlpGrads:
        p = self.params
        return qsvm.MlpGrads(p[0].g.data_ptr(), p[1].g.data_ptr(), p[2].g.data_ptr(), p[3].g.data_ptr(),
                             p[4].g.data_ptr(), p[5].g.data_ptr(), b["dH1"].data_ptr(), b["dH2"].data_ptr(),
                             b["ws"].data_ptr(), b["ws"].numel())

    # ------------------------------------------------------------------
    def _pair_pass(self, X, ii: np.ndarray, jj: np.ndarray, target: np.ndarray | None, train: bool):
        """Forward (and with train=True backward + AdamW) of the pairs (ii[p], jj[p])."""
        import torch

        c = self.cfg
        P = ii.shape[0]
        rows = 2 * P
        b = self._buffers(rows)
        b["idx"].copy_(torch.from_numpy(np.concatenate([ii, jj]).astype(np.int32)))
        if target is None:
            b["target"].zero_()
        else:
            b["target"].copy_(torch.from_numpy(np.asarray(target, dtype=np.float32)))
        qsvm.qsvm_gather_features(X, b["idx"], self.d_in, b["X16"])
        net = self.net()
        acts = self._acts(b)
        qsvm.qsvm_mlp_forward(net, b["X16"], rows, acts)
        qsvm.qsvm_pair_head_log(b["X16"], b["E"], P, b["target"], self.head.w, self.scale, b["dE16"], b["partial"],
                                b["out3"], pred=b["pred"])
        if train:
            qsvm.qsvm_mlp_backward(net, b["X16"], acts, b["dE16"], rows, self._grads(b))
            self.step += 1
            ps = self.pset  # every weight and bias in one launch
            qsvm.qsvm_adamw(ps.w, ps.g, ps.m, ps.v, ps.w16, c.lr, c.beta1, c.beta2, c.eps, c.weight_decay, self.step)
            qsvm.qsvm_adamw(self.head.w, b["out3"][1:], self.head.m, self.head.v, None, c.lr_head, c.beta1,
                            c.beta2, c.eps, 0.0, self.step)
        return b

    def predict_pairs(self, X, ii: np.ndarray, jj: np.ndarray, chunk: int = 8192):
        """(ln K_hat, d2) of the pairs (ii[p], jj[p]) as host arrays."""
        out_l, out_d = [], []
        for p0 in range(0, ii.shape[0], chunk):
            i = ii[p0:p0 + chunk]
            j = jj[p0:p0 + chunk]
            P = i.shape[0]
            Pp = _round_up(P, 32)
            if Pp != P:  # pad to whole 64-row blocks with repeats of the first pair
                i = np.concatenate([i, np.full(Pp - P, i[0])])
                j = np.concatenate([j, np.full(Pp - P, j[0])])
            b = self._pair_pass(X, i, j, None, train=False)
            pr = b["pred"].view(-1, 2)[:P].cpu().numpy().astype(np.float64)
            out_l.append(pr[:, 0])
            out_d.append(pr[:, 1])
        return np.concatenate(out_l), np.concatenate(out_d)

    def init_head(self, X, ii, jj, log_k) -> None:
        """Set (c, s) to the least-squares fit of ln K = -c (1 - exp(-s d2)) on
        the given pairs at the current embedding (s on a log grid, c in closed
        form)."""
        _, d2 = self.predict_pairs(X, ii, jj)
        t = np.asarray(log_k, dtype=np.float64)
        best = None
        med = float(np.median(d2[d2 > 0])) if np.any(d2 > 0) else 1.0
        for s in np.geomspace(1e-3 / med, 1e3 / med, 241):
            u = -np.expm1(-s * d2)
            den = float(u @ u)
            if den <= 0:
                continue
            cval = max(1e-6, -float(t @ u) / den)
            err = float(np.mean((cval * u + t) ** 2))
            if best is None or err < best[0]:
                best = (err, cval, s)
        _, cval, s = best
        self.head.w.copy_(self._f32([math.log(cval), math.log(s)]))

    def _f32(self, v):
        import torch

        return torch.as_tensor(np.asarray(v, dtype=np.float32), device=self.dev)

    def head_values(self):
        h = self.head.w.cpu().numpy().astype(np.float64)
        return math.exp(h[0]), math.exp(h[1])

    def last_loss(self, pairs: int) -> float:
        return float(self._buffers(2 * pairs)["out3"][0].item())

    def fit(self, X, ii: np.ndarray, jj: np.ndarray, log_k: np.ndarray, steps: int, log_every: int = 50) -> FitReport:
        """Train on exact pairs (ii[p], jj[p]) with targets log_k[p] = ln K.

        Every minibatch draws high_fraction of its pairs from the pairs with
        ln K above high_log_k (when there are any) and the rest uniformly: a
        stratified loader, so that the rare close pairs, the ones the fallback
        must find, are seen in every step."""
        import torch

        c = self.cfg
        P = c.pairs_per_step
        if P % 32:
            raise ValueError("pairs_per_step must be a multiple of 32")
        rng = np.random.default_rng(c.seed + 1)
        high = np.flatnonzero(log_k > c.high_log_k)
        n_high = int(round(c.high_fraction * P)) if high.size else 0
        hist = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            sel = rng.integers(0, ii.shape[0], P - n_high)
            if n_high:
                sel = np.concatenate([sel, high[rng.integers(0, high.size, n_high)]])
            self._pair_pass(X, ii[sel], jj[sel], log_k[sel], train=True)
            if log_every and (s % log_every == 0 or s == steps - 1):
                hist.append((s, self.last_loss(P)))
        torch.cuda.synchronize()
        return FitReport(steps, time.perf_counter() - t0, hist)

    def calibrate(self, X, ii, jj, log_k, band: float = 20.0, safety: float = 1.0) -> float:
        """Set the margin gram() flags tiles with: the largest under-prediction
        ln K - ln K_hat over the given pairs whose exact ln K is at least
        ln(tau) - band, plus `safety` nats (>= 0).  A pair with K >= tau must
        be flagged, i.e. ln K_hat >= ln(tau) - margin, which the margin
        guarantees for every calibration pair of that kind; pairs far below tau
        need no flag.  Without such pairs, the largest under-prediction over
        all given pairs is used."""
        lh, _ = self.predict_pairs(X, ii, jj)
        lk = np.asarray(log_k, dtype=np.float64)
        under = lk - lh
        near = lk >= math.log(self.cfg.tau) - band
        worst = float(np.max(under[near])) if np.any(near) else float(np.max(under))
        self.margin = max(0.0, worst) + safety
        return self.margin

    # ------------------------------------------------------------------
    def embed(self, X, chunk: int = 32768):
        """BF16 inputs and MLP outputs of every row of X, padded to a multiple of 64 rows."""
        import torch

        N = X.shape[0]
        Np = _round_up(N, 64)
        X16 = torch.empty((Np, self.d_in), dtype=torch.bfloat16, device=self.dev)
        E16 = torch.empty((Np, self.cfg.d_out), dtype=torch.bfloat16, device=self.dev)
        net = self.net()
        for r0 in range(0, Np, chunk):
            rows = min(chunk, Np - r0)
            b = self._buffers(rows)
            torch.arange(r0, r0 + rows, out=b["idx"])  # on the device; rows >= N are zero padding
            qsvm.qsvm_gather_features(X, b["idx"], self.d_in, X16[r0:r0 + rows])
            qsvm.qsvm_mlp_forward(net, X16[r0:r0 + rows], rows, self._acts(b, E16[r0:r0 + rows], inference=True))
        return X16, E16

    def gram(self, X, mps: "qsvm.MPS | None", K=None, tau: float | None = None, margin: float | None = None):
        """Surrogate Gram of the rows of X with exact fallback.

        A tile is flagged when its largest off-diagonal ln K_hat reaches
        ln(tau) - margin (tau = 0 flags every tile, which are then recomputed
        whole); within a flagged tile the pairs with K_hat >= tau exp(-margin)
        are recomputed exactly, one by one when there are at most
        cfg.pair_cap of them (FP64), else the whole tile (the exact sweep with
        its refinement).  Returns (K, flagged):
        flagged is a 1-element device int32 tensor, the number of flagged
        tiles; self.fallback holds the device counts (pairs, whole tiles) of
        the last call with an MPS.  mps (the exact MPS of the same points)
        feeds the fallback; pass None to skip it.  Nothing here waits for the
        GPU: the fallback reads the counts on the device."""
        import torch

        tau = self.cfg.tau if tau is None else tau
        margin = self.margin if margin is None else margin
        thresh = -math.inf if tau <= 0.0 else math.log(tau) - margin
        N = X.shape[0]
        X16, E16 = self.embed(X)
        Np = E16.shape[0]
        T = Np // 64
        if K is None:
            K = torch.empty((N, N), dtype=torch.float64, device=self.dev)
        tile_max = torch.empty(T * T, dtype=torch.float32, device=self.dev)
        qsvm.qsvm_surrogate_gram_log(X16, E16, N, self.head.w, K, tile_max)
        n_tiles = T * (T + 1) // 2
        tiles = torch.empty(2 * n_tiles, dtype=torch.int32, device=self.dev)
        count = torch.empty(1, dtype=torch.int32, device=self.dev)
        qsvm.qsvm_flag_tiles(tile_max, T, max(thresh, -3.0e38), tiles, count)  # clears count first
        if mps is not None:
            if self.cfg.pair_cap > 0 and thresh > -math.inf:  # tau <= 0 (every tile) falls back whole
                cut = 0.0 if thresh == -math.inf else math.exp(thresh)
                maxp = self.cfg.max_fallback_pairs
                pairs = torch.empty(2 * maxp, dtype=torch.int32, device=self.dev)
                dense = torch.empty(2 * n_tiles, dtype=torch.int32, device=self.dev)
                counts = torch.empty(2, dtype=torch.int32, device=self.dev)  # pairs, dense tiles
                qsvm.qsvm_flag_pairs(K, N, tiles, count, n_tiles, cut, self.cfg.pair_cap, pairs, counts[0:1], maxp,
                                     dense, counts[1:2])
                qsvm.qsvm_gram_sym_tiles_dev(mps, dense, counts[1:2], n_tiles, K)
                qsvm.qsvm_gram_sym_pairs_dev(mps, pairs, counts[0:1], maxp, K)
                self.fallback = counts
            else:
                qsvm.qsvm_gram_sym_tiles_dev(mps, tiles, count, n_tiles, K)
                self.fallback = None
        return K, count
