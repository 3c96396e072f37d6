"""Constants written into the HIP kernels, checked on the CPU (no GPU).

The MLP's GELU in csrc/mlp.hip evaluates max(x, 0) - |x| Q(|x|) with the
normal tail Q(u) = exp2(R(min(u, U)) - k u), R a polynomial.  Its
coefficients, U and k are read from the source text and the kernel's FP32
steps are replayed here (each fmaf as one rounding of the exact value), then
compared with the reference GELU x Phi(x) of oracle/mlp.py, which is itself
pinned to PyTorch's exact GELU.  A typo in any coefficient fails the bar.
"""

import os
import re

import numpy as np

from oracle import mlp as ref

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2405_02630_amd", "csrc", "mlp.hip")
F32 = np.float32


def _gelu_source():
    text = open(SRC).read()
    m = re.search(r"__device__ __forceinline__ float gelu\(float x\) \{(.*?)\n\}", text, re.S)
    assert m, "gelu() not found in mlp.hip"
    return m.group(1)


def _num(s):
    return float(s.rstrip("f"))


def _parse(body):
    num = r"(-?[0-9.]+(?:e-?[0-9]+)?f)"
    clamp = _num(re.search(r"fminf\(u, " + num + r"\)", body).group(1))
    lead = _num(re.search(r"float p = " + num + ";", body).group(1))
    coefs = [_num(c) for c in re.findall(r"p = fmaf\(p, v, " + num + r"\);", body)]
    k = -_num(re.search(r"exp2f\(fmaf\(u, " + num + r", p\)\)", body).group(1))
    return clamp, [lead] + coefs, k


def _fma32(a, b, c):
    # the product of two FP32 values is exact in FP64; one rounding to FP32 after the add
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(F32)


def _kernel_gelu(x, clamp, coefs, k):
    x = x.astype(F32)
    u = np.abs(x)
    v = np.minimum(u, F32(clamp))
    p = np.full_like(x, F32(coefs[0]))
    for c in coefs[1:]:
        p = _fma32(p, v, np.full_like(x, F32(c)))
    q = np.exp2(_fma32(u, np.full_like(x, F32(-k)), p).astype(np.float64)).astype(F32)
    return _fma32(-u, q, np.maximum(x, F32(0)))


def test_gelu_constants_are_parsed():
    clamp, coefs, k = _parse(_gelu_source())
    assert clamp == 6.0 and len(coefs) == 9 and 8.0 < k < 10.0


def test_gelu_constants_meet_the_accuracy_bar():
    """Relative error below 5e-6 wherever |GELU| is above 1e-8, absolute
    below 1e-10 further out in the negative tail (the MLP's BF16 outputs
    round at a relative 2^-9)."""
    clamp, coefs, k = _parse(_gelu_source())
    x = np.linspace(-14.0, 14.0, 400001)
    got = _kernel_gelu(x, clamp, coefs, k).astype(np.float64)
    want = ref.gelu(x.astype(F32).astype(np.float64))
    err = np.abs(got - want)
    big = np.abs(want) > 1e-8
    assert np.max(err[big] / np.abs(want[big])) < 5e-6
    assert np.max(err[~big]) < 1e-10


def test_gelu_tail_continues_the_fit_at_the_clamp():
    """k is the slope of -log2 Q at the clamp point, so the tail continues
    the fit smoothly: just inside and just outside it the kernel's GELU is
    within 5e-6 (relative) of the reference."""
    clamp, coefs, k = _parse(_gelu_source())
    x = np.array([-clamp + 1e-3, -clamp - 1e-3, clamp - 1e-3, clamp + 1e-3])
    got = _kernel_gelu(x, clamp, coefs, k).astype(np.float64)
    want = ref.gelu(x.astype(F32).astype(np.float64))
    assert np.all(np.abs(got - want) <= 5e-6 * np.abs(want))
