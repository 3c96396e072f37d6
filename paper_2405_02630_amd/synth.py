"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws feature vectors; it holds none of the kernel's
arithmetic, so both the GPU path and the CPU oracle may use it.  The paper
measures on PCA-reduced and full 28x28 MNIST / Fashion-MNIST images (§4.2,
§5); those datasets are not available here, so these generators copy their
shapes instead: 10 classes, 64 features or 784 = 28x28 pixels, features
already scaled to angles in [0, pi].

All generators take an integer seed and use numpy's PCG64 through
``SeedSequence(seed).spawn``, so every stream is reproducible and the streams
of one configuration are independent.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

PI = math.pi


def _streams(seed: int, k: int):
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(k)]


def uniform_features(N: int, n: int, seed: int = 0) -> np.ndarray:
    """N x n float64 features, iid uniform on [0, pi]."""
    (g,) = _streams(seed, 1)
    return g.uniform(0.0, PI, size=(N, n))


def gaussian_mixture(N: int, n: int, n_classes: int = 10, seed: int = 0,
                     mean_lo: float = 0.5, mean_hi: float = 2.6, sigma: float = 0.3):
    """Class means uniform on [mean_lo, mean_hi]^n, x = clip(mu_c + sigma z, 0, pi).

    Labels are i mod n_classes.  Returns (X, labels).
    """
    gm, gx = _streams(seed, 2)
    means = gm.uniform(mean_lo, mean_hi, size=(n_classes, n))
    labels = np.arange(N) % n_classes
    X = means[labels] + sigma * gx.standard_normal((N, n))
    return np.clip(X, 0.0, PI), labels


def smooth_templates(n_classes: int = 10, side: int = 28, blur: float = 3.0,
                     border: int = 4, seed: int = 0) -> np.ndarray:
    """Smooth class templates in [0, 1]: blurred white noise, min-max scaled,
    with a zero border (most MNIST pixels near the frame are background)."""
    from scipy.ndimage import gaussian_filter

    (g,) = _streams(seed, 1)
    out = np.empty((n_classes, side, side))
    for c in range(n_classes):
        t = gaussian_filter(g.standard_normal((side, side)), sigma=blur, mode="wrap")
        t = (t - t.min()) / (t.max() - t.min())
        if border:
            t[:border, :] = 0.0
            t[-border:, :] = 0.0
            t[:, :border] = 0.0
            t[:, -border:] = 0.0
        out[c] = t
    return out


def template_images(N: int, templates: np.ndarray, noise: float = 0.1, seed: int = 0,
                    label_offset: int = 0):
    """Images = clip(template_c + N(0, noise^2), 0, 1) * pi, flattened row-major.

    Labels are (i + label_offset) mod n_classes (class balanced).  Returns (X, labels).
    """
    (g,) = _streams(seed, 1)
    n_classes = templates.shape[0]
    labels = (np.arange(N) + label_offset) % n_classes
    flat = templates.reshape(n_classes, -1)
    X = flat[labels] + noise * g.standard_normal((N, flat.shape[1]))
    return np.clip(X, 0.0, 1.0) * PI, labels


def pin_even_features(X: np.ndarray) -> np.ndarray:
    """Copy of X with every even-indexed feature set to pi (all entangling angles vanish)."""
    Y = np.array(X, dtype=np.float64, copy=True)
    Y[..., ::2] = PI
    return Y


def near_duplicates(base: np.ndarray, eps_list=(1e-3, 3e-3, 1e-2, 3e-2, 1e-1), seed: int = 0):
    """For every base row and eps, a copy x + eps z (z ~ N(0, I)) clipped to [0, pi].

    Returns (X, base_index, eps_of_row) with the perturbed rows stacked in the
    order (eps, base row).
    """
    (g,) = _streams(seed, 1)
    rows, idx, eps_col = [], [], []
    for eps in eps_list:
        z = g.standard_normal(base.shape)
        rows.append(np.clip(base + eps * z, 0.0, PI))
        idx.append(np.arange(base.shape[0]))
        eps_col.append(np.full(base.shape[0], eps))
    return np.concatenate(rows), np.concatenate(idx), np.concatenate(eps_col)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    n: int
    reps: int
    X: np.ndarray
    labels: np.ndarray | None = None
    X_test: np.ndarray | None = None
    labels_test: np.ndarray | None = None


def tiny_uniform(seed: int = 0) -> Workload:
    """n = 8 qubits, reps = 2, N = 32 points uniform on [0, pi]."""
    return Workload("tiny-n8-r2-N32", 8, 2, uniform_features(32, 8, seed))


def mixture64(seed: int = 0, N: int = 1024) -> Workload:
    """n = 64, reps = 2, N = 1024 points of a 10-class Gaussian mixture."""
    X, y = gaussian_mixture(N, 64, seed=seed)
    return Workload(f"mixture-n64-r2-N{N}", 64, 2, X, y)


def images784(seed: int = 0, n_train: int = 4096, n_test: int = 1024, reps: int = 2) -> Workload:
    """n = 784 (28x28), 10 smooth class templates + N(0, 0.1^2) pixel noise."""
    s_tpl, s_tr, s_te = (int(s.generate_state(1)[0]) for s in np.random.SeedSequence(seed).spawn(3))
    tpl = smooth_templates(seed=s_tpl)
    Xtr, ytr = template_images(n_train, tpl, seed=s_tr)
    Xte, yte = template_images(n_test, tpl, seed=s_te)
    return Workload(f"images-n784-r{reps}-train{n_train}-test{n_test}", 784, reps, Xtr, ytr, Xte, yte)


def image_near_duplicates(seed: int = 0, n_base: int = 256):
    """Near-duplicate validation set: base images plus eps-perturbed copies."""
    wl = images784(seed=seed, n_train=n_base, n_test=0)
    Xp, idx, eps = near_duplicates(wl.X, seed=seed + 1)
    return wl.X, Xp, idx, eps


def images784_with_near_duplicates(N: int = 32768, n_copies: int = 2048, seed: int = 0):
    """N 784-pixel images of which n_copies are near duplicates: copies
    x + eps z of distinct random base images (eps cycling through 1e-3, 3e-3,
    1e-2, 3e-2, 1e-1), rows shuffled.  Returns (X, labels, base_of_row) with
    base_of_row[r] = the row holding the original of a copy, -1 otherwise."""
    n_img = N - n_copies
    wl = images784(seed=seed, n_train=n_img, n_test=0)
    g_pick, g_eps, g_perm = _streams(seed + 23, 3)
    bases = g_pick.choice(n_img, size=n_copies, replace=False)
    eps = np.array([1e-3, 3e-3, 1e-2, 3e-2, 1e-1])[np.arange(n_copies) % 5]
    copies = np.clip(wl.X[bases] + eps[:, None] * g_eps.standard_normal((n_copies, wl.X.shape[1])), 0.0, PI)
    X = np.concatenate([wl.X, copies])
    labels = np.concatenate([wl.labels, wl.labels[bases]])
    src = np.concatenate([np.full(n_img, -1), bases])
    perm = g_perm.permutation(N)
    inv = np.empty(N, dtype=np.int64)
    inv[perm] = np.arange(N)
    base_of_row = np.where(src[perm] >= 0, inv[np.maximum(src[perm], 0)], -1)
    return X[perm], labels[perm], base_of_row


def near_identical_images(N: int = 4096, eps: float = 4e-4, seed: int = 0) -> np.ndarray:
    """N copies of one 784-pixel image, each x + eps z (z ~ N(0, I)) clipped to
    [0, pi]: every pair is a near duplicate (the worst case for work that only
    entries near 1 need)."""
    wl = images784(seed=seed, n_train=1, n_test=0)
    (g,) = _streams(seed + 11, 1)
    return np.clip(wl.X[0][None, :] + eps * g.standard_normal((N, wl.X.shape[1])), 0.0, PI)


def uneven_jobs(seed: int = 0, n_jobs: int = 64, n_choices=(16, 64, 196, 400, 784),
                N_lo: int = 64, N_hi: int = 2048, reps_choices=(2, 3)):
    """Independent Gram jobs with n, N and reps drawn per job; features uniform on [0, pi]."""
    g_meta, g_x = _streams(seed, 2)
    jobs = []
    for j in range(n_jobs):
        n = int(g_meta.choice(n_choices))
        N = int(g_meta.integers(N_lo, N_hi + 1))
        r = int(g_meta.choice(reps_choices))
        X = g_x.uniform(0.0, PI, size=(N, n))
        jobs.append(Workload(f"job{j}-n{n}-r{r}-N{N}", n, r, X))
    return jobs
