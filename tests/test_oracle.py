"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

The oracle is trusted only because it reproduces, independently of itself:
  * hand-derived exact kernel values (tests/golden/closed_form_cases.json);
  * a textbook construction of U(x) from 2^n x 2^n Kronecker products;
  * the one-rep kernel as an explicit 2^n-term sum (paper §2, Eq. 4 with
    U = D H^n) and as a transfer-matrix product;
  * the entanglement-free product formula (prod_k cos^2(x_k - y_k) for one rep);
  * the structural properties of a Gram matrix (diag 1, symmetric, range, PSD).
Planted-mistake tests at the end show that a plausible bug in the oracle
(wrong entangling angle, wrong phase sign, wrong Hadamard, a dropped ZZ block,
an over-truncating SVD, a missing conjugate) fails at least one pin.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import closed_forms, feature_map, mps, statevector
from oracle.mps import mps_to_statevector
from paper_2405_02630_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_form_cases.json")


def _golden_cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


# --------------------------------------------------------------------------
# Textbook construction: every gate as a full 2^n x 2^n matrix (n <= 5)
# --------------------------------------------------------------------------

def _op_on(n, k, g):
    # qubit k is bit k of the basis index (least significant = qubit 0)
    return np.kron(np.kron(np.eye(1 << (n - k - 1)), g), np.eye(1 << k))


def _cnot_matrix(n, c, t):
    dim = 1 << n
    m = np.zeros((dim, dim))
    for i in range(dim):
        j = i ^ (1 << t) if (i >> c) & 1 else i
        m[j, i] = 1.0
    return m


def kron_state(x, reps):
    """|psi(x)> from the written-out circuit: H, P(2x_k), CNOT P(theta_k) CNOT."""
    n = len(x)
    h = np.array([[1, 1], [1, -1]]) / math.sqrt(2)
    u = np.eye(1 << n, dtype=complex)
    for _ in range(reps):
        for k in range(n):
            u = _op_on(n, k, h) @ u
        for k in range(n):
            u = _op_on(n, k, np.diag([1, np.exp(2j * x[k])])) @ u
        for k in range(n - 1):
            th = 2 * (math.pi - x[k]) * (math.pi - x[k + 1])
            cx = _cnot_matrix(n, k, k + 1)
            u = cx @ _op_on(n, k + 1, np.diag([1, np.exp(1j * th)])) @ cx @ u
    e0 = np.zeros(1 << n, dtype=complex)
    e0[0] = 1
    return u @ e0


# --------------------------------------------------------------------------
# Golden closed forms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: f"n{c['n']}r{c['reps']}-{c['expr']}")
def test_golden_state_vector(case):
    x = np.array(case["x_over_pi"]) * math.pi
    y = np.array(case["y_over_pi"]) * math.pi
    K = statevector.sv_gram_rect(x[None], y[None], case["reps"])[0, 0]
    assert abs(K - case["value"]) < 1e-12


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: f"n{c['n']}r{c['reps']}-{c['expr']}")
def test_golden_mps(case):
    x = np.array(case["x_over_pi"]) * math.pi
    y = np.array(case["y_over_pi"]) * math.pi
    la, _ = mps.mps_overlap_log(mps.mps_state(x, case["reps"]), mps.mps_state(y, case["reps"]))
    K = math.exp(2 * la) if la > -700 else 0.0
    assert abs(K - case["value"]) < 1e-12


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: f"n{c['n']}r{c['reps']}-{c['expr']}")
def test_golden_closed_forms(case):
    x = np.array(case["x_over_pi"]) * math.pi
    y = np.array(case["y_over_pi"]) * math.pi
    if case["n"] == 1:
        assert abs(closed_forms.k_one_qubit(x[0], y[0], case["reps"]) - case["value"]) < 1e-12
    if case["reps"] == 1:
        assert abs(closed_forms.k_reps1_bruteforce(x, y) - case["value"]) < 1e-12
        _, k = closed_forms.k_reps1_transfer(x, y)
        assert abs(k - case["value"]) < 1e-12


# --------------------------------------------------------------------------
# O1 against the textbook construction; O2 against O1
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("reps", [1, 2, 3, 4])
def test_state_vector_matches_kron(n, reps):
    rng = np.random.default_rng(100 * n + reps)
    x = rng.uniform(0, math.pi, n)
    assert np.max(np.abs(statevector.sv_state(x, reps) - kron_state(x, reps))) < 1e-12


@pytest.mark.parametrize("n", [2, 3, 6, 9, 12])
@pytest.mark.parametrize("reps", [1, 2, 3, 4])
def test_mps_state_matches_state_vector(n, reps):
    rng = np.random.default_rng(7 * n + reps)
    x = rng.uniform(0, math.pi, n)
    v = mps_to_statevector(mps.mps_state(x, reps))
    assert np.max(np.abs(v - statevector.sv_state(x, reps))) < 1e-12


@pytest.mark.parametrize("reps", [1, 2, 3, 4])
def test_mps_gram_matches_state_vector(reps):
    X = synth.uniform_features(10, 10, seed=reps)
    K1 = statevector.sv_gram(X, reps)
    S = mps.mps_states(X, reps)
    ii, jj = np.meshgrid(np.arange(10), np.arange(10), indexing="ij")
    _, K2 = mps.mps_gram_pairs(S, S, ii.ravel(), jj.ravel())
    assert np.max(np.abs(K1 - K2.reshape(10, 10))) < 1e-12


def test_mps_rect_gram_matches_state_vector():
    Xa = synth.uniform_features(5, 8, seed=11)
    Xb = synth.uniform_features(7, 8, seed=12)
    K1 = statevector.sv_gram_rect(Xa, Xb, 2)
    Sa, Sb = mps.mps_states(Xa, 2), mps.mps_states(Xb, 2)
    ii, jj = np.meshgrid(np.arange(5), np.arange(7), indexing="ij")
    _, K2 = mps.mps_gram_pairs(Sa, Sb, ii.ravel(), jj.ravel())
    assert np.max(np.abs(K1 - K2.reshape(5, 7))) < 1e-12


@pytest.mark.parametrize("reps", [1, 2, 3, 4])
def test_mps_bond_dimension_is_two_to_the_reps(reps):
    x = synth.uniform_features(1, 14, seed=3)[0]
    bonds = [t.shape[2] for t in mps.mps_state(x, reps)[:-1]]
    # the cut after site k separates k+1 qubits: rank <= min(2^reps, 2^(k+1), 2^(n-k-1))
    n = len(x)
    for k, d in enumerate(bonds):
        assert d <= min(2**reps, 2 ** (k + 1), 2 ** (n - k - 1))
    assert max(bonds) == 2**reps  # generic inputs saturate the bound


# --------------------------------------------------------------------------
# One-rep sum and transfer matrix
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 5, 8, 11])
def test_reps1_bruteforce_matches_state_vector(n):
    rng = np.random.default_rng(n)
    x, y = rng.uniform(0, math.pi, (2, n))
    K = statevector.sv_gram_rect(x[None], y[None], 1)[0, 0]
    assert abs(closed_forms.k_reps1_bruteforce(x, y) - K) < 1e-12


@pytest.mark.parametrize("n", [1, 3, 7, 12])
def test_reps1_transfer_matches_bruteforce(n):
    rng = np.random.default_rng(50 + n)
    x, y = rng.uniform(0, math.pi, (2, n))
    _, k = closed_forms.k_reps1_transfer(x, y)
    assert abs(k - closed_forms.k_reps1_bruteforce(x, y)) < 1e-13


def test_reps1_transfer_matches_mps_at_784():
    X = synth.uniform_features(2, 784, seed=21)
    la, _ = mps.mps_overlap_log(mps.mps_state(X[0], 1), mps.mps_state(X[1], 1))
    lk, _ = closed_forms.k_reps1_transfer(X[0], X[1])
    assert lk < -300  # far below the FP64 range of K itself
    assert abs(2 * la - lk) < 1e-9 * abs(lk)


# --------------------------------------------------------------------------
# Entanglement-free inputs
# --------------------------------------------------------------------------

@pytest.mark.parametrize("reps", [1, 2, 3, 4])
def test_product_form_matches_state_vector(reps):
    X = synth.pin_even_features(synth.uniform_features(2, 8, seed=30 + reps))
    K = statevector.sv_gram_rect(X[:1], X[1:], reps)[0, 0]
    assert abs(closed_forms.k_product(X[0], X[1], reps) - K) < 1e-13
    if reps == 1:
        assert abs(np.prod(np.cos(X[0] - X[1]) ** 2) - K) < 1e-13


@pytest.mark.parametrize("reps", [1, 2, 3, 4])
def test_product_form_matches_mps_at_784(reps):
    X = synth.pin_even_features(synth.images784(seed=1, n_train=2, n_test=0).X)
    la, _ = mps.mps_overlap_log(mps.mps_state(X[0], reps), mps.mps_state(X[1], reps))
    lk = closed_forms.k_product_log(X[0], X[1], reps)
    assert abs(2 * la - lk) < 1e-9 * max(1.0, abs(lk))


def test_product_form_rejects_entangled_inputs():
    X = synth.uniform_features(2, 6, seed=2)
    with pytest.raises(ValueError):
        closed_forms.k_product(X[0], X[1], 2)


# --------------------------------------------------------------------------
# Gram-matrix properties
# --------------------------------------------------------------------------

def test_tiny_gram_properties():
    wl = synth.tiny_uniform(seed=0)
    K = statevector.sv_gram(wl.X, wl.reps)
    assert oracle.check_gram(K) == {}


def test_check_gram_detects_violations():
    K = np.eye(3)
    K[0, 1] = 0.5
    assert "symmetry" in oracle.check_gram(K)
    K2 = np.array([[1.0, 0.9, -0.9], [0.9, 1.0, 0.9], [-0.9, 0.9, 1.0]])
    bad = oracle.check_gram(K2)
    assert "psd" in bad and "range" in bad


def test_self_overlap_is_one_at_784():
    x = synth.images784(seed=2, n_train=1, n_test=0).X[0]
    s = mps.mps_state(x, 2)
    la, ph = mps.mps_overlap_log(s, s)
    assert abs(la) < 1e-11 and abs(ph - 1) < 1e-11


# --------------------------------------------------------------------------
# Planted mistakes must fail a pin
# --------------------------------------------------------------------------

def _pins_hold():
    """A fast subset of the pins above; False as soon as one fails."""
    for case in _golden_cases():
        x = np.array(case["x_over_pi"]) * math.pi
        y = np.array(case["y_over_pi"]) * math.pi
        if abs(statevector.sv_gram_rect(x[None], y[None], case["reps"])[0, 0] - case["value"]) > 1e-12:
            return False
        la, _ = mps.mps_overlap_log(mps.mps_state(x, case["reps"]), mps.mps_state(y, case["reps"]))
        if abs((math.exp(2 * la) if la > -700 else 0.0) - case["value"]) > 1e-12:
            return False
    rng = np.random.default_rng(0)
    for n in (3, 6):
        for reps in (1, 2, 3):
            x, y = rng.uniform(0, math.pi, (2, n))
            K1 = statevector.sv_gram_rect(x[None], y[None], reps)[0, 0]
            if reps == 1 and abs(closed_forms.k_reps1_bruteforce(x, y) - K1) > 1e-12:
                return False
            if np.max(np.abs(statevector.sv_state(x, reps) - kron_state(x, reps))) > 1e-12:
                return False
            la, _ = mps.mps_overlap_log(mps.mps_state(x, reps), mps.mps_state(y, reps))
            if abs(math.exp(2 * la) - K1) > 1e-12:
                return False
    return True


def test_pins_hold_for_the_oracle_as_written():
    assert _pins_hold()


def test_planted_wrong_entangling_angle(monkeypatch):
    monkeypatch.setattr(feature_map, "zz_angle", lambda a, b: 2.0 * float(a) * float(b))
    assert not _pins_hold()


def test_planted_phase_sign(monkeypatch):
    orig = feature_map.feature_map_gates

    def flipped(x, reps):
        return [(g, q, (-p if g == "P" and i % 7 == 0 else p)) for i, (g, q, p) in enumerate(orig(x, reps))]

    monkeypatch.setattr(statevector, "feature_map_gates", flipped)
    assert not _pins_hold()


def test_planted_wrong_hadamard(monkeypatch):
    monkeypatch.setattr(statevector, "H_GATE", np.array([[1, 1], [1, -1]], dtype=complex) / 2.0)
    assert not _pins_hold()


def test_planted_dropped_zz_block(monkeypatch):
    orig = feature_map.feature_map_gates

    def dropped(x, reps):
        g = orig(x, reps)
        n = len(x)
        if n < 2:
            return g
        # remove the three gates of the last ZZ block of the first repetition
        start = 2 * n + 3 * (n - 2)
        return g[:start] + g[start + 3:]

    monkeypatch.setattr(statevector, "feature_map_gates", dropped)
    assert not _pins_hold()


def test_planted_truncating_svd(monkeypatch):
    monkeypatch.setattr(mps, "SVD_ZERO_REL", 0.3)
    assert not _pins_hold()


def test_planted_missing_conjugate(monkeypatch):
    def overlap_no_conj(sa, sb):
        e = np.ones((1, 1), dtype=complex)
        acc = 0.0
        for a, b in zip(sa, sb):
            e = np.einsum("ysv,ysu->vu", b, np.einsum("yx,xsu->ysu", e, a))
            m = np.max(np.abs(e))
            e = e / m
            acc += math.log(m)
        return acc + math.log(abs(e[0, 0])), 1.0

    monkeypatch.setattr(mps, "mps_overlap_log", overlap_no_conj)
    assert not _pins_hold()
