"""Pins of the surrogate's FP64 reference (oracle/mlp.py), no GPU.

The reference is checked against finite differences of its own loss (the
backward must be the derivative of the forward) and against PyTorch's CPU
float64 autograd, GELU and AdamW, and bfloat16 conversion -- library routines
that the reference does not use.
"""

import math

import numpy as np
import pytest
import torch

from oracle import mlp


def _params(rng, dims=(6, 5, 4, 3), scale=0.5):
    d0, d1, d2, d3 = dims
    return (
        rng.normal(0, scale, (d0, d1)), rng.normal(0, 0.1, d1),
        rng.normal(0, scale, (d1, d2)), rng.normal(0, 0.1, d2),
        rng.normal(0, scale, (d2, d3)), rng.normal(0, 0.1, d3),
    )


def _loss(params, X, target, alpha, beta, kind="mse"):
    acts = mlp.forward(params, X)
    return mlp.pair_loss(acts["E"], target, alpha, beta, kind)[0]


def test_gelu_matches_torch():
    x = np.linspace(-6, 6, 101)
    ref = torch.nn.functional.gelu(torch.tensor(x, dtype=torch.float64), approximate="none").numpy()
    assert np.max(np.abs(mlp.gelu(x) - ref)) < 1e-14


def test_gelu_grad_matches_finite_difference():
    x = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(mlp.gelu_grad(x) - fd)) < 1e-8


@pytest.mark.parametrize("kind", ["mse", "bce"])
def test_backward_matches_finite_differences(kind):
    rng = np.random.default_rng(0)
    params = list(_params(rng))
    X = rng.normal(0, 1, (8, 6))
    target = rng.uniform(0, 1, 4)
    alpha, beta = 0.7, -0.2
    acts = mlp.forward(params, X)
    _, dE, da, db = mlp.pair_loss(acts["E"], target, alpha, beta, kind)
    grads = mlp.backward(params, X, acts, dE)
    h = 1e-6
    for pi, (p, g) in enumerate(zip(params, grads)):
        flat = p.reshape(-1)
        for q in range(0, flat.size, max(1, flat.size // 7)):
            old = flat[q]
            flat[q] = old + h
            lp = _loss(params, X, target, alpha, beta, kind)
            flat[q] = old - h
            lm = _loss(params, X, target, alpha, beta, kind)
            flat[q] = old
            assert abs((lp - lm) / (2 * h) - g.reshape(-1)[q]) < 1e-7, (pi, q)
    fa = (_loss(params, X, target, alpha + h, beta, kind) - _loss(params, X, target, alpha - h, beta, kind)) / (2 * h)
    fb = (_loss(params, X, target, alpha, beta + h, kind) - _loss(params, X, target, alpha, beta - h, kind)) / (2 * h)
    assert abs(fa - da) < 1e-7 and abs(fb - db) < 1e-7


def test_bce_loss_matches_torch():
    rng = np.random.default_rng(5)
    E = rng.normal(0, 1, (8, 3))
    t = rng.uniform(0, 1, 4)
    loss, *_ = mlp.pair_loss(E, t, 0.9, -0.3, "bce")
    z = 0.9 * np.sum(E[:4] * E[4:], axis=1) - 0.3
    ref = torch.nn.functional.binary_cross_entropy_with_logits(torch.tensor(z), torch.tensor(t)).item()
    assert abs(loss - ref) < 1e-14


def test_forward_and_gradients_match_torch_autograd():
    rng = np.random.default_rng(1)
    params = _params(rng, dims=(10, 8, 7, 5))
    X = rng.normal(0, 1, (12, 10))
    target = rng.uniform(0, 1, 6)
    alpha, beta = 1.3, 0.4
    acts = mlp.forward(params, X)
    loss, dE, da, db = mlp.pair_loss(acts["E"], target, alpha, beta)
    grads = mlp.backward(params, X, acts, dE)

    tp = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in params]
    ta = torch.tensor(alpha, dtype=torch.float64, requires_grad=True)
    tb = torch.tensor(beta, dtype=torch.float64, requires_grad=True)
    tX = torch.tensor(X)
    g = torch.nn.functional.gelu
    E = g(g(tX @ tp[0] + tp[1]) @ tp[2] + tp[3]) @ tp[4] + tp[5]
    P = 6
    kh = torch.sigmoid(ta * (E[:P] * E[P:]).sum(1) + tb)
    tl = ((kh - torch.tensor(target)) ** 2).mean()
    tl.backward()
    assert abs(tl.item() - loss) < 1e-14
    assert np.max(np.abs(E.detach().numpy() - acts["E"])) < 1e-13
    for p, gr in zip(tp, grads):
        assert np.max(np.abs(p.grad.numpy() - gr)) < 1e-13
    assert abs(ta.grad.item() - da) < 1e-13 and abs(tb.grad.item() - db) < 1e-13


def test_adamw_matches_torch():
    rng = np.random.default_rng(2)
    w0 = rng.normal(0, 1, 17)
    grads = [rng.normal(0, 1, 17) for _ in range(3)]
    lr, b1, b2, eps, wd = 1e-2, 0.9, 0.99, 1e-8, 0.05
    tw = torch.tensor(w0, requires_grad=True)
    opt = torch.optim.AdamW([tw], lr=lr, betas=(b1, b2), eps=eps, weight_decay=wd)
    w, m, v = w0.copy(), np.zeros(17), np.zeros(17)
    for step, gr in enumerate(grads, start=1):
        tw.grad = torch.tensor(gr)
        opt.step()
        w, m, v = mlp.adamw_step(w, gr, m, v, step, lr, b1, b2, eps, wd)
    assert np.max(np.abs(tw.detach().numpy() - w)) < 1e-13


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 1, 1000), rng.normal(0, 1e-3, 100), [0.0, 1.0, -2.5, 1.00390625, 1.01171875]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)


def test_surrogate_gram_matches_torch_sigmoid():
    rng = np.random.default_rng(4)
    E = rng.normal(0, 1, (37, 9))
    K = mlp.surrogate_gram(E, 0.5, -1.0)
    tE = torch.tensor(E, dtype=torch.float64)
    ref = torch.sigmoid(0.5 * (tE @ tE.T) - 1.0).numpy()
    np.fill_diagonal(ref, 1.0)
    assert np.max(np.abs(K - ref)) < 1e-15
    assert np.array_equal(K, K.T)


def _sat_loss(params, Xr, X, target, lc, ls, scale):
    acts = mlp.forward(params, X)
    return mlp.sat_log_pair_loss(Xr, acts["E"], target, lc, ls, scale)[0]


def test_sat_log_head_matches_torch_autograd():
    # ln K_hat = -c (1 - exp(-s d2)), d2 the squared distance of [x, f(x)]
    # (torch.cdist, a library routine the reference does not use); loss and
    # every gradient against autograd
    rng = np.random.default_rng(6)
    params = _params(rng, dims=(10, 8, 7, 5))
    X = rng.normal(0, 1, (16, 10))
    Xr = rng.uniform(0, 3, (16, 4))  # the input part of the embedding
    target = rng.uniform(-40.0, 0.0, 8)
    lc, ls, scale = math.log(30.0), math.log(0.05), 7.0
    acts = mlp.forward(params, X)
    loss, dE, dlc, dls, lh, d2 = mlp.sat_log_pair_loss(Xr, acts["E"], target, lc, ls, scale)
    grads = mlp.backward(params, X, acts, dE)

    tp = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in params]
    tlc = torch.tensor(lc, dtype=torch.float64, requires_grad=True)
    tls = torch.tensor(ls, dtype=torch.float64, requires_grad=True)
    g = torch.nn.functional.gelu
    E = g(g(torch.tensor(X) @ tp[0] + tp[1]) @ tp[2] + tp[3]) @ tp[4] + tp[5]
    Z = torch.cat([torch.tensor(Xr), E], dim=1)
    P = 8
    td2 = torch.cdist(Z[:P].unsqueeze(0), Z[P:].unsqueeze(0)).squeeze(0).diagonal() ** 2
    tlh = -torch.exp(tlc) * (1 - torch.exp(-torch.exp(tls) * td2))
    tl = ((tlh - torch.tensor(target)) / scale).pow(2).mean()
    tl.backward()
    assert abs(tl.item() - loss) < 1e-13
    assert np.max(np.abs(td2.detach().numpy() - d2)) < 1e-11
    assert np.max(np.abs(tlh.detach().numpy() - lh)) < 1e-11
    for p, gr in zip(tp, grads):
        assert np.max(np.abs(p.grad.numpy() - gr)) < 1e-13
    assert abs(tlc.grad.item() - dlc) < 1e-12 and abs(tls.grad.item() - dls) < 1e-12


def test_sat_log_head_matches_finite_differences():
    rng = np.random.default_rng(7)
    params = list(_params(rng))
    X = rng.normal(0, 1, (8, 6))
    Xr = rng.uniform(0, 1, (8, 3))
    target = rng.uniform(-5, 0, 4)
    lc, ls, scale = math.log(6.0), math.log(0.3), 3.0
    acts = mlp.forward(params, X)
    _, dE, dlc, dls, _, _ = mlp.sat_log_pair_loss(Xr, acts["E"], target, lc, ls, scale)
    grads = mlp.backward(params, X, acts, dE)
    h = 1e-6
    for p, g in zip(params, grads):
        flat = p.reshape(-1)
        for q in range(0, flat.size, max(1, flat.size // 5)):
            old = flat[q]
            flat[q] = old + h
            lp = _sat_loss(params, Xr, X, target, lc, ls, scale)
            flat[q] = old - h
            lm = _sat_loss(params, Xr, X, target, lc, ls, scale)
            flat[q] = old
            assert abs((lp - lm) / (2 * h) - g.reshape(-1)[q]) < 1e-7
    fc = (_sat_loss(params, Xr, X, target, lc + h, ls, scale) - _sat_loss(params, Xr, X, target, lc - h, ls, scale)) / (2 * h)
    fs = (_sat_loss(params, Xr, X, target, lc, ls + h, scale) - _sat_loss(params, Xr, X, target, lc, ls - h, scale)) / (2 * h)
    assert abs(fc - dlc) < 1e-7 and abs(fs - dls) < 1e-7


def test_sat_log_head_special_cases():
    # identical embeddings predict ln K_hat = 0 (K_hat = 1) whatever c and s
    # are; small distances give -c s d2; large ones saturate at -c
    Xr = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 0.0], [1.0, 0.0]])  # pairs (0, 2) and (1, 3)
    E = np.zeros((4, 3))
    _, _, _, _, lh, d2 = mlp.sat_log_pair_loss(Xr, E, np.zeros(2), math.log(50.0), math.log(0.1), 1.0)
    assert lh[0] == 0.0 and d2[1] == 2.0
    assert lh[1] == pytest.approx(-50.0 * (1.0 - math.exp(-0.2)), rel=1e-15)
    assert mlp.sat_log_head(np.array([1e-9]), math.log(50.0), math.log(0.1))[0] == pytest.approx(-50.0 * 0.1 * 1e-9, rel=1e-8)
    assert mlp.sat_log_head(np.array([1e4]), math.log(50.0), math.log(0.1))[0] == pytest.approx(-50.0, rel=1e-15)
    L, K = mlp.sat_log_gram(Xr, E, math.log(50.0), math.log(0.1))
    assert np.array_equal(np.diag(L), np.zeros(4)) and np.array_equal(np.diag(K), np.ones(4))
    assert L[0, 2] == 0.0 and K[0, 2] == 1.0 and L[0, 1] == pytest.approx(lh[1], rel=1e-15)


def test_sat_log_gram_matches_torch_cdist():
    rng = np.random.default_rng(8)
    Xr = rng.uniform(0, 3, (70, 5))
    E = rng.normal(0, 0.3, (70, 12))
    L, K = mlp.sat_log_gram(Xr, E, math.log(20.0), math.log(0.25))
    Z = torch.tensor(np.concatenate([Xr, E], axis=1))
    ref = (-20.0 * (1 - torch.exp(-0.25 * torch.cdist(Z, Z).pow(2)))).numpy()
    np.fill_diagonal(ref, 0.0)
    assert np.max(np.abs(L - ref)) < 1e-12
    assert np.max(np.abs(K - np.exp(ref))) < 1e-12


def test_tile_max_offdiag():
    M = np.arange(130 * 130, dtype=np.float64).reshape(130, 130)
    tm = mlp.tile_max_offdiag(M)
    assert tm.shape == (3, 3)
    assert tm[0, 0] == M[63, 62]   # the diagonal entry M[63, 63] is excluded
    assert tm[0, 2] == M[63, 129]
    assert tm[2, 2] == M[129, 128]
    assert tm[2, 0] == M[129, 63]
