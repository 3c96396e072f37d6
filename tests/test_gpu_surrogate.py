"""GPU: the surrogate's kernels against the FP64 reference (oracle/mlp.py).

The kernels round to BF16 where the design says (inputs, weights, hidden
activations, back-propagated gradients) and accumulate in FP32.  Each check
compares with the FP64 reference evaluated on the same BF16-rounded operands,
with the kernels' intermediate BF16 roundings emulated (tight bar), and where
noted with the unrounded FP64 reference (loose bar, set by BF16's 2^-9 unit
roundoff compounded over three layers).
"""

import math

import numpy as np
import pytest

from oracle import mlp as ref
from oracle import statevector
from paper_2405_02630_amd import qsvm, synth

from gpu_helpers import K_ABS_TOL, encode, require_gpu

pytestmark = pytest.mark.gpu

DIMS = (128, 64, 128, 64)  # d_in, d_h1, d_h2, d_out (multiples of 64)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


def _bf16_dev(x):
    import torch

    return torch.as_tensor(np.asarray(x, np.float32)).to(torch.bfloat16).to("cuda:0")


def _f32_dev(x):
    import torch

    return torch.as_tensor(np.asarray(x, np.float32), device="cuda:0")


def _host(t):
    import torch

    return t.to(torch.float64).cpu().numpy()


# Element-wise bars.  A product of K-term dot products of BF16 values summed in
# FP32 is exact per term and rounds the running sum: its error is at most
# K u sum|a||b| (u = 2^-24) and typically sqrt(K) u sum|a||b|; the bar is
# GEMM_REL * (|A| |B|)_ij with GEMM_REL = 8 sqrt(K) u, per element.  A value
# the kernel rounds to BF16 may differ from the reference's rounding of the
# FP64 value by one BF16 spacing (at most 2^-7 of the value) where the two
# sit on either side of a rounding boundary: bar = 2^-7 |ref| plus the bar of
# the value before rounding.
U32 = 2.0**-24
U16 = 2.0**-8
GELU_ABS = 4e-7


def _gemm_bar(absA, absB):
    K = absA.shape[1]
    return 8.0 * math.sqrt(K) * U32 * (absA @ absB) + 1e-30


def _assert_elementwise(got, ref, bar, what):
    d = np.abs(np.asarray(got, np.float64) - ref)
    worst = np.unravel_index(np.argmax(d - bar), d.shape)
    assert np.all(d <= bar), (what, worst, float(d[worst]), float(np.asarray(bar)[worst] if np.ndim(bar) else bar))


def _setup(seed=0, rows=128, dims=DIMS):
    import torch

    rng = np.random.default_rng(seed)
    d0, d1, d2, d3 = dims
    W = [ref.bf16_round(rng.normal(0, math.sqrt(2 / d0), (d0, d1))), rng.normal(0, 0.1, d1),
         ref.bf16_round(rng.normal(0, math.sqrt(2 / d1), (d1, d2))), rng.normal(0, 0.1, d2),
         ref.bf16_round(rng.normal(0, math.sqrt(1 / d2), (d2, d3))), rng.normal(0, 0.1, d3)]
    W[1], W[3], W[5] = (np.float32(w).astype(np.float64) for w in (W[1], W[3], W[5]))
    X = ref.bf16_round(rng.normal(0, 1, (rows, d0)))
    dev = {k: v for k, v in zip(["W1", "b1", "W2", "b2", "W3", "b3"],
                                [_bf16_dev(W[0]), _f32_dev(W[1]), _bf16_dev(W[2]), _f32_dev(W[3]),
                                 _bf16_dev(W[4]), _f32_dev(W[5])])}
    net = qsvm.Mlp(d0, d1, d2, d3, dev["W1"].data_ptr(), dev["b1"].data_ptr(), dev["W2"].data_ptr(),
                   dev["b2"].data_ptr(), dev["W3"].data_ptr(), dev["b3"].data_ptr())
    f32, b16 = torch.float32, torch.bfloat16
    bufs = {
        "X16": _bf16_dev(X),
        "H1": torch.empty((rows, d1), dtype=f32, device="cuda:0"),
        "A1": torch.empty((rows, d1), dtype=b16, device="cuda:0"),
        "H2": torch.empty((rows, d2), dtype=f32, device="cuda:0"),
        "A2": torch.empty((rows, d2), dtype=b16, device="cuda:0"),
        "E": torch.empty((rows, d3), dtype=f32, device="cuda:0"),
        "E16": torch.empty((rows, d3), dtype=b16, device="cuda:0"),
    }
    acts = qsvm.MlpActs(*(bufs[k].data_ptr() for k in ("H1", "A1", "H2", "A2", "E", "E16")))
    return W, X, dev, net, bufs, acts


def _check_forward(W, X, bufs, idx=None):
    """Each layer against the FP64 reference evaluated on the kernel's own
    inputs to that layer (so rounding differences do not compound); on the
    rows `idx` only when given (every row's check stands on its own)."""
    H1, A1, H2, A2, E = (_host(bufs[k]) for k in ("H1", "A1", "H2", "A2", "E"))
    E16 = _host(bufs["E16"])
    if idx is not None:
        X, H1, A1, H2, A2, E, E16 = (a[idx] for a in (X, H1, A1, H2, A2, E, E16))
    _assert_elementwise(H1, X @ W[0] + W[1], _gemm_bar(np.abs(X), np.abs(W[0])) + 1e-7 * np.abs(W[1]), "H1")
    g1 = ref.gelu(H1)
    _assert_elementwise(A1, ref.bf16_round(g1), 2 * U16 * np.abs(g1) + 1e-6 * (1 + np.abs(H1)), "A1")
    _assert_elementwise(H2, A1 @ W[2] + W[3], _gemm_bar(np.abs(A1), np.abs(W[2])) + 1e-7 * np.abs(W[3]), "H2")
    g2 = ref.gelu(H2)
    _assert_elementwise(A2, ref.bf16_round(g2), 2 * U16 * np.abs(g2) + 1e-6 * (1 + np.abs(H2)), "A2")
    _assert_elementwise(E, A2 @ W[4] + W[5], _gemm_bar(np.abs(A2), np.abs(W[4])) + 1e-7 * np.abs(W[5]), "E")
    assert np.array_equal(E16, ref.bf16_round(E))
    return H1, A1, H2, A2, E


def _check_backward(W, X, acts_h, dEk, grads, dH1, dH2):
    """Backward against the FP64 reference on the kernel's own activations and
    incoming gradients, element by element."""
    H1, A1, H2, A2 = acts_h
    aX, aA1, aA2, adE = np.abs(X), np.abs(A1), np.abs(A2), np.abs(dEk)
    _assert_elementwise(_host(grads["dW3"]), A2.T @ dEk, _gemm_bar(aA2.T, adE), "dW3")
    _assert_elementwise(_host(grads["db3"]), dEk.sum(0), _gemm_bar(np.ones((1, dEk.shape[0])), adE)[0], "db3")
    acc2 = dEk @ W[4].T
    pre2 = acc2 * ref.gelu_grad(H2)
    # FP32 gelu'(h) = Phi(h) + h phi(h) carries an absolute error of a few
    # 1e-8 where 1 + erf cancels (h << 0): GELU_ABS |acc| on top
    bar2 = (_gemm_bar(adE, np.abs(W[4].T)) * np.abs(ref.gelu_grad(H2)) * 2 + GELU_ABS * np.abs(acc2)
            + 2 * U16 * np.abs(pre2) + 1e-30)
    dH2k = _host(dH2)
    _assert_elementwise(dH2k, ref.bf16_round(pre2), bar2, "dH2")
    _assert_elementwise(_host(grads["dW2"]), A1.T @ dH2k, _gemm_bar(aA1.T, np.abs(dH2k)), "dW2")
    _assert_elementwise(_host(grads["db2"]), dH2k.sum(0), _gemm_bar(np.ones((1, dH2k.shape[0])), np.abs(dH2k))[0], "db2")
    acc1 = dH2k @ W[2].T
    pre1 = acc1 * ref.gelu_grad(H1)
    bar1 = (_gemm_bar(np.abs(dH2k), np.abs(W[2].T)) * np.abs(ref.gelu_grad(H1)) * 2 + GELU_ABS * np.abs(acc1)
            + 2 * U16 * np.abs(pre1) + 1e-30)
    dH1k = _host(dH1)
    _assert_elementwise(dH1k, ref.bf16_round(pre1), bar1, "dH1")
    _assert_elementwise(_host(grads["dW1"]), X.T @ dH1k, _gemm_bar(aX.T, np.abs(dH1k)), "dW1")
    _assert_elementwise(_host(grads["db1"]), dH1k.sum(0), _gemm_bar(np.ones((1, dH1k.shape[0])), np.abs(dH1k))[0], "db1")


def _backward(net, bufs, acts, dev, dE16, rows, dims):
    import torch

    grads = {k: torch.empty_like(dev[w], dtype=torch.float32) for k, w in
             zip(["dW1", "db1", "dW2", "db2", "dW3", "db3"], ["W1", "b1", "W2", "b2", "W3", "b3"])}
    dH1 = torch.empty((rows, dims[1]), dtype=torch.bfloat16, device="cuda:0")
    dH2 = torch.empty((rows, dims[2]), dtype=torch.bfloat16, device="cuda:0")
    ws = torch.empty(qsvm.qsvm_mlp_workspace_floats(net, rows), dtype=torch.float32, device="cuda:0")
    g = qsvm.MlpGrads(*(grads[k].data_ptr() for k in ("dW1", "db1", "dW2", "db2", "dW3", "db3")),
                      dH1.data_ptr(), dH2.data_ptr(), ws.data_ptr(), ws.numel())
    qsvm.qsvm_mlp_backward(net, bufs["X16"], acts, dE16, rows, g)
    torch.cuda.synchronize()
    return grads, dH1, dH2


def test_mlp_forward_matches_reference():
    import torch

    W, X, dev, net, bufs, acts = _setup(0)
    qsvm.qsvm_mlp_forward(net, bufs["X16"], X.shape[0], acts)
    torch.cuda.synchronize()
    _check_forward(W, X, bufs)
    # the whole chain against the FP64 forward without intermediate rounding:
    # three layers of BF16 activations, each within 2^-8 relative
    full = ref.forward(W, X)["E"]
    E = _host(bufs["E"])
    assert np.max(np.abs(E - full)) <= 0.05 * np.max(np.abs(full))


PROD = (832, 512, 512, 256)  # 784 pixels padded to 832 -> 512 -> 512 -> 256


@pytest.mark.parametrize("rows,dims", [(32768, PROD), (16384, PROD), (128, DIMS)])
def test_mlp_forward_inference_mode_writes_the_same_bf16_outputs(rows, dims):
    """H1, H2 and E omitted (inference): the BF16 activations and embedding are
    bitwise those of the forward pass that keeps the FP32 values."""
    import torch

    W, X, dev, net, bufs, acts = _setup(13, rows=rows, dims=dims)
    qsvm.qsvm_mlp_forward(net, bufs["X16"], rows, acts)
    A1i, A2i, E16i = (torch.empty_like(bufs[k]) for k in ("A1", "A2", "E16"))
    qsvm.qsvm_mlp_forward(net, bufs["X16"], rows, qsvm.MlpActs(None, A1i.data_ptr(), None, A2i.data_ptr(), None,
                                                               E16i.data_ptr()))
    torch.cuda.synchronize()
    for a, b in ((A1i, bufs["A1"]), (A2i, bufs["A2"]), (E16i, bufs["E16"])):
        assert torch.equal(a.view(torch.int16), b.view(torch.int16))


def test_mlp_forward_backward_production_shape_elementwise():
    """The surrogate's production widths on 16384 rows: 13 K steps in layer 1,
    the XCD tile order, and each layer's weight and bias gradients as one
    product on k-contiguous copies (the activations with a row of ones),
    split 16 or 32 ways along the rows and summed in fixed order -- every
    element of every output against the FP64 reference on the kernel's own
    layer inputs."""
    import torch

    rows = 16384
    W, X, dev, net, bufs, acts = _setup(11, rows=rows, dims=PROD)
    qsvm.qsvm_mlp_forward(net, bufs["X16"], rows, acts)
    torch.cuda.synchronize()
    H1, A1, H2, A2, E = _check_forward(W, X, bufs)
    assert qsvm.qsvm_mlp_workspace_floats(net, rows) >= 16 * 896 * 512  # layer 1: 16 slabs of 896 x 512
    rng = np.random.default_rng(12)
    dEk = ref.bf16_round(rng.normal(0, 1e-3, (rows, PROD[3])))
    grads, dH1, dH2 = _backward(net, bufs, acts, dev, _bf16_dev(dEk), rows, PROD)
    _check_backward(W, X, (H1, A1, H2, A2), dEk, grads, dH1, dH2)


def test_mlp_forward_256x256_tiles_elementwise():
    """At 32768 rows layers 1 and 2 (512 outputs wide) fill every compute unit
    with 256 x 256 tiles: one 8-wave block each, 64-deep K steps (13 in layer
    1, K = 832), 128 KB of LDS.  Every element of every layer's output
    against the FP64 reference on the kernel's own layer inputs."""
    import torch

    rows = 32768
    W, X, dev, net, bufs, acts = _setup(21, rows=rows, dims=PROD)
    qsvm.qsvm_mlp_forward(net, bufs["X16"], rows, acts)
    torch.cuda.synchronize()
    _check_forward(W, X, bufs)


def test_mlp_forward_256x128_tiles_on_rows_sampled_from_every_tile():
    """Hidden widths of 384 (a multiple of 128, not of 256) on 44032 rows:
    layers 1 and 2 take 256 x 128 tiles of 4 waves (172 x 3 = 516 tiles, at
    least two per compute unit) and layer 3 128 x 128 tiles with 32-deep
    steps (688 blocks).  Every third row plus the last 256 against the FP64
    reference on the kernel's own layer inputs."""
    import torch

    rows, dims = 44032, (832, 384, 384, 256)
    W, X, dev, net, bufs, acts = _setup(23, rows=rows, dims=dims)
    qsvm.qsvm_mlp_forward(net, bufs["X16"], rows, acts)
    torch.cuda.synchronize()
    idx = np.union1d(np.arange(0, rows, 3), np.arange(rows - 256, rows))
    _check_forward(W, X, bufs, idx)


@pytest.mark.parametrize("kind", [qsvm.LOSS_MSE, qsvm.LOSS_BCE], ids=["mse", "bce"])
def test_pair_head_and_backward_match_reference(kind):
    import torch

    W, X, dev, net, bufs, acts = _setup(1)
    rows = X.shape[0]
    P = rows // 2
    rng = np.random.default_rng(7)
    target = rng.uniform(0, 1, P).astype(np.float32).astype(np.float64)
    ab = _f32_dev([0.05, -0.3])
    qsvm.qsvm_mlp_forward(net, bufs["X16"], rows, acts)
    dE16 = torch.empty((rows, DIMS[3]), dtype=torch.bfloat16, device="cuda:0")
    partial = torch.empty(3 * P, dtype=torch.float32, device="cuda:0")
    out3 = torch.empty(3, dtype=torch.float32, device="cuda:0")
    qsvm.qsvm_pair_head(bufs["E"], P, DIMS[3], _f32_dev(target), ab, dE16, partial, out3, loss_kind=kind)
    torch.cuda.synchronize()
    E = _host(bufs["E"])
    loss, dE, da, db = ref.pair_loss(E, target, float(np.float32(0.05)), float(np.float32(-0.3)),
                                     "bce" if kind == qsvm.LOSS_BCE else "mse")
    o = out3.cpu().numpy()
    assert abs(o[0] - loss) <= 1e-5 * max(1.0, abs(loss))
    assert abs(o[1] - da) <= 1e-4 * max(1e-3, abs(da)) + 1e-7
    assert abs(o[2] - db) <= 1e-4 * max(1e-3, abs(db)) + 1e-7
    _assert_elementwise(_host(dE16), dE, 2 * U16 * np.abs(dE) + 1e-6 * np.max(np.abs(dE)), "dE16")
    acts_h = tuple(_host(bufs[k]) for k in ("H1", "A1", "H2", "A2"))
    grads, dH1, dH2 = _backward(net, bufs, acts, dev, dE16, rows, DIMS)
    _check_backward(W, X, acts_h, _host(dE16), grads, dH1, dH2)


def test_pair_head_log_production_shape_elementwise():
    """The log-domain head on 8192 pairs of [784-pixel input padded to 832,
    256-wide MLP output]: loss, its head gradients, ln K_hat, d2 and the
    embedding gradient of every element against oracle/mlp.py."""
    import torch

    P, d_in, d = 8192, 832, 256
    rng = np.random.default_rng(21)
    Xr = ref.bf16_round(rng.uniform(0, math.pi, (2 * P, d_in)) * (rng.random((2 * P, d_in)) < 0.7))
    Xr[P:] = ref.bf16_round(np.clip(Xr[:P] + rng.normal(0, 0.05, (P, d_in)) * (rng.random((P, 1)) < 0.3), 0, math.pi))
    E = rng.normal(0, 0.2, (2 * P, d)).astype(np.float32).astype(np.float64)
    target = np.float32(rng.uniform(-600, 0, P)).astype(np.float64)
    lc, ls = float(np.float32(math.log(585.0))), float(np.float32(math.log(0.03)))
    scale = 784.0
    dE16 = torch.empty((2 * P, d), dtype=torch.bfloat16, device="cuda:0")
    partial = torch.empty(3 * P, dtype=torch.float32, device="cuda:0")
    out3 = torch.empty(3, dtype=torch.float32, device="cuda:0")
    pred = torch.empty(2 * P, dtype=torch.float32, device="cuda:0")
    qsvm.qsvm_pair_head_log(_bf16_dev(Xr), _f32_dev(E), P, _f32_dev(target), _f32_dev([lc, ls]), scale, dE16,
                            partial, out3, pred=pred)
    torch.cuda.synchronize()
    loss, dE, dlc, dls, lh, d2 = ref.sat_log_pair_loss(Xr, E, target, lc, ls, scale)
    pr = pred.view(-1, 2).cpu().numpy().astype(np.float64)
    # d2: FP32 sum of ~1100 squares (relative sqrt(K) u each way); ln K_hat from it
    _assert_elementwise(pr[:, 1], d2, 1e-5 * d2 + 1e-6, "d2")
    c, s = math.exp(lc), math.exp(ls)
    _assert_elementwise(pr[:, 0], lh, c * s * np.exp(-s * d2) * 1e-5 * d2 + 1e-5 * np.abs(lh) + 1e-6, "lnK_hat")
    o = out3.cpu().numpy()
    assert abs(o[0] - loss) <= 1e-4 * loss
    assert abs(o[1] - dlc) <= 1e-3 * abs(dlc) + 1e-6 and abs(o[2] - dls) <= 1e-3 * abs(dls) + 1e-6
    _assert_elementwise(_host(dE16), dE, 2 * U16 * np.abs(dE) + 1e-4 * np.max(np.abs(dE)), "dE16")


@pytest.mark.parametrize("N,d_in,d", [(150, 832, 256), (200, 64, 128), (130, 0, 64), (64, 832, 32), (300, 96, 256)])
def test_surrogate_gram_log_elementwise_and_tile_max(N, d_in, d):
    """Ragged N (odd tile counts: the last 128-row block half empty), an exact
    tile multiple, and input parts from none to the production 832."""
    import torch

    rng = np.random.default_rng(N + d_in)
    Np = (N + 63) // 64 * 64
    base = rng.uniform(0, 1, (8, d_in))
    Xr = ref.bf16_round(base[rng.integers(0, 8, Np)] + rng.normal(0, 0.02, (Np, d_in)))  # clusters: K spread out
    E = ref.bf16_round(rng.normal(0, 0.1, (Np, d)))
    lc, ls = float(np.float32(math.log(30.0))), float(np.float32(math.log(0.2)))
    K = torch.full((N, N), -1.0, dtype=torch.float64, device="cuda:0")
    T = Np // 64
    tmax = torch.empty(T * T, dtype=torch.float32, device="cuda:0")
    x16 = _bf16_dev(Xr) if d_in else None
    qsvm.qsvm_surrogate_gram_log(x16, _bf16_dev(E), N, _f32_dev([lc, ls]), K, tmax)
    torch.cuda.synchronize()
    Kh = K.cpu().numpy()
    L, Kr = ref.sat_log_gram(Xr[:N], E[:N], lc, ls)
    Z = np.concatenate([Xr[:N], E[:N]], axis=1)
    nrm = np.sum(Z * Z, axis=1)
    # d2 from norms and a BF16 inner product in FP32: error ~ 1e-6 (|z_i|^2 + |z_j|^2)
    err_d2 = 2e-6 * (nrm[:, None] + nrm[None, :]) + 1e-7
    err_l = 30.0 * 0.2 * err_d2 + 1e-6 * np.abs(L) + 1e-6  # |d ln K_hat / d d2| <= c s
    _assert_elementwise(Kh, Kr, Kr * np.expm1(err_l) + 1e-30, "K_hat")
    assert np.all(np.diag(Kh) == 1.0)
    assert np.array_equal(Kh, Kh.T)
    tm = tmax.cpu().numpy().reshape(T, T)
    tref = ref.tile_max_offdiag(L)
    valid = np.isfinite(tref)
    assert np.array_equal(np.isfinite(tm), valid)
    tbar = np.array([[err_l[a * 64:(a + 1) * 64, b * 64:(b + 1) * 64].max() for b in range(T)] for a in range(T)])
    assert np.all(np.abs(tm[valid] - tref[valid]) <= tbar[valid])
    # flags in the log domain: exactly the tiles at or above the threshold
    thr = float(np.median(tm[np.triu_indices(T)][np.isfinite(tm[np.triu_indices(T)])]))
    tiles = torch.empty(T * (T + 1), dtype=torch.int32, device="cuda:0")
    count = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    qsvm.qsvm_flag_tiles(tmax, T, thr, tiles, count)
    torch.cuda.synchronize()
    c = int(count.item())
    got = {tuple(x) for x in tiles.cpu().numpy()[: 2 * c].reshape(-1, 2)}
    want = {(ti, tj) for ti in range(T) for tj in range(ti, T) if tm[ti, tj] >= np.float32(thr)}
    assert got == want and c == len(want)


def test_surrogate_gram_log_many_super_tiles_every_entry_written():
    """N = 4160 at the production widths (832 + 256): 33 block rows of 128 in
    5 super-rows of 8 (the last partial, its last block half past N_pad).
    Every entry of K and every tile maximum is written (NaN before the call),
    K is exactly symmetric with a unit diagonal, and sampled rows around the
    block and super-tile boundaries, and whole tiles on and off the diagonal,
    match the FP64 reference."""
    import torch

    N, d_in, d = 4160, 832, 256
    rng = np.random.default_rng(4160)
    base = rng.uniform(0, 1, (16, d_in))
    Xr = ref.bf16_round(base[rng.integers(0, 16, N)] + rng.normal(0, 0.02, (N, d_in)))
    E = ref.bf16_round(rng.normal(0, 0.1, (N, d)))
    lc, ls = float(np.float32(math.log(30.0))), float(np.float32(math.log(0.2)))
    T = N // 64
    K = torch.full((N, N), float("nan"), dtype=torch.float64, device="cuda:0")
    tmax = torch.full((T * T,), float("nan"), dtype=torch.float32, device="cuda:0")
    qsvm.qsvm_surrogate_gram_log(_bf16_dev(Xr), _bf16_dev(E), N, _f32_dev([lc, ls]), K, tmax)
    torch.cuda.synchronize()
    assert not torch.isnan(K).any().item()
    assert torch.equal(K, K.T)
    assert torch.all(torch.diagonal(K) == 1.0).item()
    tm = tmax.cpu().numpy().reshape(T, T)
    assert not np.isnan(tm).any() and np.array_equal(tm, tm.T)

    def bars(rows):
        Z = np.concatenate([Xr[rows], E[rows]], axis=1)
        nrm = np.sum(Z * Z, axis=1)
        err_d2 = 2e-6 * (nrm[:, None] + nrm[None, :]) + 1e-7
        return err_d2

    idx = np.unique(np.concatenate([[0, 1, 127, 128, 129, 1023, 1024, 1025, 2047, 2048, 4095, 4096, 4159],
                                    rng.integers(0, N, 150)]))
    L, Kr = ref.sat_log_gram(Xr[idx], E[idx], lc, ls)
    err_l = 30.0 * 0.2 * bars(idx) + 1e-6 * np.abs(L) + 1e-6
    Kh = K.cpu().numpy()
    _assert_elementwise(Kh[np.ix_(idx, idx)], Kr, Kr * np.expm1(err_l) + 1e-30, "K_hat sampled")
    for ta, tb in [(0, 0), (0, 1), (15, 16), (16, 16), (31, 64), (64, 64), (2, 60)]:
        rows = np.concatenate([np.arange(ta * 64, ta * 64 + 64), np.arange(tb * 64, tb * 64 + 64)])
        L, Kr = ref.sat_log_gram(Xr[rows], E[rows], lc, ls)
        err_l = 30.0 * 0.2 * bars(rows) + 1e-6 * np.abs(L) + 1e-6
        blk = (slice(0, 64), slice(64, 128)) if ta != tb else (slice(0, 64), slice(0, 64))
        got = Kh[ta * 64:ta * 64 + 64, tb * 64:tb * 64 + 64]
        _assert_elementwise(got, Kr[blk], Kr[blk] * np.expm1(err_l[blk]) + 1e-30, f"tile ({ta},{tb})")
        lref = L[blk].copy()
        if ta == tb:
            np.fill_diagonal(lref, -np.inf)
        assert abs(tm[ta, tb] - lref.max()) <= err_l[blk].max(), (ta, tb, tm[ta, tb], lref.max())


def test_adamw_matches_reference():
    import torch

    rng = np.random.default_rng(3)
    w0 = rng.normal(0, 1, 1000).astype(np.float32)
    w = _f32_dev(w0)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    w16 = torch.empty(1000, dtype=torch.bfloat16, device="cuda:0")
    rw, rm, rv = w0.astype(np.float64), np.zeros(1000), np.zeros(1000)
    for step in range(1, 4):
        gr = rng.normal(0, 1, 1000).astype(np.float32)
        qsvm.qsvm_adamw(w, _f32_dev(gr), m, v, w16, 1e-2, 0.9, 0.999, 1e-8, 0.01, step)
        rw, rm, rv = ref.adamw_step(rw, gr.astype(np.float64), rm, rv, step, 1e-2, 0.9, 0.999, 1e-8, 0.01)
    torch.cuda.synchronize()
    assert np.max(np.abs(w.cpu().numpy() - rw)) < 1e-5
    assert np.array_equal(_host(w16), ref.bf16_round(w.cpu().numpy()))


# Ragged N with an odd tile count (the last 128-row block half empty), an
# exact tile multiple, and several embedding widths.
@pytest.mark.parametrize("N,d", [(150, 64), (200, 128), (130, 256), (64, 256), (150, 96), (300, 32)])
def test_surrogate_gram_tile_max_and_flags(N, d):
    import torch

    rng = np.random.default_rng(4 + d)
    Np = (N + 63) // 64 * 64
    E = ref.bf16_round(rng.normal(0, 0.3, (Np, d)))
    E16 = _bf16_dev(E)
    ab = _f32_dev([0.5, -3.0])
    K = torch.full((N, N), -1.0, dtype=torch.float64, device="cuda:0")
    T = Np // 64
    tmax = torch.empty(T * T, dtype=torch.float32, device="cuda:0")
    qsvm.qsvm_surrogate_gram(E16, N, ab, K, tmax)
    torch.cuda.synchronize()
    Kh = K.cpu().numpy()
    Kr = ref.surrogate_gram(E[:N], 0.5, -3.0)
    assert np.max(np.abs(Kh - Kr)) < 1e-6
    assert np.array_equal(Kh, Kh.T)
    tm = tmax.cpu().numpy().reshape(T, T)
    for ti in range(T):
        for tj in range(T):
            blk = Kh[ti * 64:min(N, ti * 64 + 64), tj * 64:min(N, tj * 64 + 64)].copy()
            if ti == tj:
                np.fill_diagonal(blk, -np.inf)
            assert tm[ti, tj] == np.float32(blk.max())
    tau = float(np.median(tm[np.triu_indices(T)]))
    tiles = torch.empty(T * (T + 1), dtype=torch.int32, device="cuda:0")
    count = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    qsvm.qsvm_flag_tiles(tmax, T, tau, tiles, count)
    torch.cuda.synchronize()
    c = int(count.item())
    got = {tuple(x) for x in tiles.cpu().numpy()[: 2 * c].reshape(-1, 2)}
    want = {(ti, tj) for ti in range(T) for tj in range(ti, T) if tm[ti, tj] >= np.float32(tau)}
    assert got == want and c == len(want)


def test_gram_sym_tiles_equals_full_gram_on_those_tiles():
    import torch

    X = synth.uniform_features(200, 20, seed=5)
    m = encode(X, 2)
    full = qsvm.qsvm_gram_sym(m)
    K = torch.full((200, 200), -2.0, dtype=torch.float64, device="cuda:0")
    lst = [(0, 0), (0, 2), (1, 3), (2, 2), (3, 1), (5, 5), (-1, 0)]  # last three are invalid, skipped
    tiles = torch.tensor(lst, dtype=torch.int32, device="cuda:0").reshape(-1)
    qsvm.qsvm_gram_sym_tiles(m, tiles, len(lst), K)
    torch.cuda.synchronize()
    Kh, F = K.cpu().numpy(), full.cpu().numpy()
    mask = np.zeros((200, 200), dtype=bool)
    for ti, tj in lst[:4]:
        mask[ti * 64:(ti + 1) * 64, tj * 64:(tj + 1) * 64] = True
        mask[tj * 64:(tj + 1) * 64, ti * 64:(ti + 1) * 64] = True
    assert np.array_equal(Kh[mask], F[mask])
    assert np.all(Kh[~mask] == -2.0)


def _near_duplicate_rich(seed, n_img, n_base):
    """784-pixel images plus eps-perturbed copies of the first n_base of them,
    rows shuffled: ln K spans [-660, 0] (copies of one image down to ~-0.01)."""
    wl = synth.images784(seed=seed, n_train=n_img, n_test=0, reps=2)
    Xp, _, _ = synth.near_duplicates(wl.X[:n_base], seed=seed + 1)
    X = np.concatenate([wl.X, Xp])
    return X[np.random.default_rng(seed).permutation(X.shape[0])]


def test_surrogate_learns_the_log_kernel_and_meets_the_bar():
    """What the trained network gains, on 784-pixel images (reps = 2) with
    near duplicates: trained on half of the exact pairs (ln K from the MPS
    sweep), judged on a quarter held out.  Its held-out log-domain error is
    below the best constant predictor's (on all pairs, and by a wide margin on
    the close pairs) and below the untrained network's on the close pairs;
    calibrated on the last quarter, the Gram with exact fallback stays within
    1e-5 of the exact Gram on every pair while recomputing only a part of the
    tiles."""
    import torch

    from paper_2405_02630_amd.surrogate import Surrogate, SurrogateConfig

    Xh = _near_duplicate_rich(31, 1024, 64)  # 1344 points, 21 tiles a side
    N = Xh.shape[0]
    X = torch.as_tensor(Xh, device="cuda:0")
    m = encode(Xh, 2)
    L = torch.empty((N, N), dtype=torch.float64, device="cuda:0")
    exact = qsvm.qsvm_gram_sym(m, log_k=L)
    Lh, Kx = L.cpu().numpy(), exact.cpu().numpy()
    ii, jj = np.triu_indices(N, 1)
    lk = Lh[ii, jj]
    part = np.random.default_rng(2).random(ii.size)
    tr, cal, ho = part < 0.5, (part >= 0.5) & (part < 0.75), part >= 0.75
    sur = Surrogate(784, SurrogateConfig(pairs_per_step=4096, seed=3))
    pick = np.random.default_rng(4).choice(np.flatnonzero(tr), 65536, replace=False)
    sur.init_head(X, ii[pick], jj[pick], lk[pick])
    lh0, _ = sur.predict_pairs(X, ii[ho], jj[ho])
    rep = sur.fit(X, ii[tr], jj[tr], lk[tr], steps=400, log_every=100)
    assert rep.loss_history[-1][1] < rep.loss_history[0][1]
    lh1, _ = sur.predict_pairs(X, ii[ho], jj[ho])
    close = lk[ho] > -100.0
    assert close.sum() >= 50
    e0, e1 = np.abs(lh0 - lk[ho]), np.abs(lh1 - lk[ho])
    ec = np.abs(np.median(lk[tr]) - lk[ho])  # best constant (median of the training targets)
    print(f"held-out mean |d ln K|: trained {e1.mean():.2f}, untrained {e0.mean():.2f}, constant {ec.mean():.2f}; "
          f"close pairs: {e1[close].mean():.2f} / {e0[close].mean():.2f} / {ec[close].mean():.2f}", flush=True)
    assert e1.mean() < ec.mean()
    assert e1[close].mean() < 0.1 * ec[close].mean()
    assert e1[close].mean() < e0[close].mean()
    margin = sur.calibrate(X, ii[cal], jj[cal], lk[cal])
    Ks, flagged = sur.gram(X, m)
    torch.cuda.synchronize()
    T = (N + 63) // 64
    flagged = int(flagged.item())
    print(f"margin {margin:.1f} nats, flagged {flagged} of {T * (T + 1) // 2} tiles", flush=True)
    assert 0 < flagged < T * (T + 1) // 2
    assert float(np.max(np.abs(Ks.cpu().numpy() - Kx))) <= K_ABS_TOL


def test_surrogate_gram_with_full_fallback_is_exact():
    """tau = 0 flags every tile: the result must equal the exact Gram bit for bit."""
    import torch

    from paper_2405_02630_amd.surrogate import Surrogate, SurrogateConfig

    Xh = synth.uniform_features(150, 12, seed=12)
    X = torch.as_tensor(Xh, device="cuda:0")
    m = encode(Xh, 2)
    exact = qsvm.qsvm_gram_sym(m)
    sur = Surrogate(12, SurrogateConfig(d_h1=64, d_h2=64, d_out=64))
    K, flagged = sur.gram(X, m, tau=0.0)
    torch.cuda.synchronize()
    assert int(flagged.item()) == 3 * 4 // 2
    assert torch.equal(K, exact)


@pytest.mark.parametrize("N,n,d_pad", [(37, 13, 16), (37, 13, 18), (50, 784, 832), (5, 7, 7), (3, 1, 4)])
def test_gather_features_matches_torch_conversion(N, n, d_pad):
    """Rows idx[r] of X converted to bf16 (through float32, round to nearest
    even) and zero-padded; rows with idx outside [0, N) are all zero."""
    import torch

    rng = np.random.default_rng(N * 1000 + d_pad)
    Xh = rng.uniform(-4.0, 4.0, (N, n))
    idx = np.concatenate([rng.integers(0, N, 60), [-1, N, N + 5, 0, N - 1]]).astype(np.int32)
    X = torch.as_tensor(Xh, device="cuda:0")
    out = torch.full((len(idx), d_pad), 7.0, dtype=torch.bfloat16, device="cuda:0")
    qsvm.qsvm_gather_features(X, torch.as_tensor(idx, device="cuda:0"), d_pad, out)
    torch.cuda.synchronize()
    ref = torch.zeros((len(idx), d_pad), dtype=torch.bfloat16)
    ok = (idx >= 0) & (idx < N)
    ref[torch.as_tensor(ok), :n] = torch.as_tensor(Xh[idx[ok]]).to(torch.float32).to(torch.bfloat16)
    assert torch.equal(out.cpu().view(torch.int16), ref.view(torch.int16))


@pytest.mark.parametrize("reps", [1, 2, 3, 4, 5, 6])
def test_gram_sym_pairs_dev_writes_the_fp64_entries(reps):
    """Listed pairs (either order, duplicates, the diagonal, invalid indices
    and entries past the count among them) get exactly the FP64 value the
    refinement writes for that entry; nothing else is touched."""
    import torch

    N = 150
    Xh = synth.uniform_features(N, 64, seed=70 + reps)
    m = encode(Xh, reps)
    Lref = torch.empty((N, N), dtype=torch.float64, device="cuda:0")
    Kref = qsvm.qsvm_gram_sym(m, log_k=Lref, refine_above=1e-300)  # every entry refined in FP64
    rng = np.random.default_rng(5)
    P = 600
    pr = rng.integers(0, N, size=(P, 2))
    pr[:5] = [[3, 3], [7, 2], [2, 7], [149, 0], [0, 149]]  # diagonal, both orders
    pr[5:8] = [[-1, -1], [4, 150], [-3, 9]]               # skipped on the device
    pairs = torch.as_tensor(pr.astype(np.int32).ravel(), device="cuda:0")
    count = torch.tensor([P - 50], dtype=torch.int32, device="cuda:0")  # the last 50 are past the count
    K = torch.full((N, N), -1.0, dtype=torch.float64, device="cuda:0")
    L = torch.full((N, N), -1.0, dtype=torch.float64, device="cuda:0")
    qsvm.qsvm_gram_sym_pairs_dev(m, pairs, count, P, K, log_k=L)
    torch.cuda.synchronize()
    Kh, Lh, Kr, Lr = K.cpu().numpy(), L.cpu().numpy(), Kref.cpu().numpy(), Lref.cpu().numpy()
    want = np.zeros((N, N), dtype=bool)
    for i, j in pr[:P - 50]:
        if 0 <= i < N and 0 <= j < N and i != j:
            want[i, j] = want[j, i] = True
    assert want.sum() > 900
    assert np.array_equal(Kh[want], Kr[want]) and np.array_equal(Lh[want], Lr[want])
    assert np.all(Kh[~want] == -1.0) and np.all(Lh[~want] == -1.0)  # incl. the diagonal (diag_mode 0)


def test_flag_pairs_matches_a_host_listing():
    import torch

    N, T = 200, 4
    rng = np.random.default_rng(9)
    Kh = np.exp(-rng.exponential(30.0, size=(N, N)))  # most entries tiny, a few near 1
    K = torch.as_tensor(Kh, device="cuda:0")
    cut = 1e-6
    tl = [(0, 0), (0, 2), (1, 3), (3, 3), (2, 2), (0, 1)]
    tiles = torch.as_tensor(np.array(tl, dtype=np.int32).ravel(), device="cuda:0")
    tcount = torch.tensor([len(tl) - 1], dtype=torch.int32, device="cuda:0")  # (0, 1) is past the count

    def host(tmax):
        pairs, dense = set(), set()
        for ti, tj in tl[:tmax]:
            hits = [(i, j) for i in range(64 * ti, min(N, 64 * ti + 64)) for j in range(64 * tj, min(N, 64 * tj + 64))
                    if j > i and Kh[i, j] >= cut]
            if len(hits) > cap:
                dense.add((ti, tj))
            elif hits:
                pairs.update(hits)
        return pairs, dense

    for cap, maxp in [(64, 4096), (4096, 4096), (64, 30)]:
        pairs = torch.full((2 * maxp,), -7, dtype=torch.int32, device="cuda:0")
        dense = torch.full((2 * len(tl),), -7, dtype=torch.int32, device="cuda:0")
        counts = torch.full((2,), 99, dtype=torch.int32, device="cuda:0")
        qsvm.qsvm_flag_pairs(K, N, tiles, tcount, len(tl), cut, cap, pairs, counts[0:1], maxp, dense, counts[1:2])
        torch.cuda.synchronize()
        npair, ndense = (int(v) for v in counts.cpu())
        P = pairs.cpu().numpy().reshape(-1, 2)[:min(npair, maxp)]
        D = dense.cpu().numpy().reshape(-1, 2)[:ndense]
        got_pairs = {(int(i), int(j)) for i, j in P if i >= 0}
        got_dense = {(int(a), int(b)) for a, b in D}
        want_pairs, want_dense = host(len(tl) - 1)
        if maxp >= 4096:
            assert got_pairs == want_pairs and got_dense == want_dense
            assert npair == len(want_pairs) and all(i >= 0 for i, _ in P)
        else:
            # the pair list overflows: tiles that did not fit fall back whole,
            # their reserved slots hold (-1, -1); every flagged pair is covered
            assert got_pairs <= want_pairs and want_dense <= got_dense
            covered = got_pairs | {(i, j) for (ti, tj) in got_dense for (i, j) in want_pairs
                                   if i // 64 == ti and j // 64 == tj}
            assert covered == want_pairs
            assert all((i >= 0) == (j >= 0) for i, j in P)
