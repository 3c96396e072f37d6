"""Host-side parts of the end-to-end QSVC path (no GPU): the macro metrics of
Table macro_metrics against scikit-learn's, and the PCA-to-angles map."""

import math

import numpy as np
import pytest
from sklearn.decomposition import PCA
from sklearn.metrics import accuracy_score, confusion_matrix, f1_score, recall_score

from paper_2405_02630_amd.qsvc import PCAAngles, macro_metrics


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_macro_metrics_match_sklearn(seed):
    rng = np.random.default_rng(seed)
    y = rng.integers(0, 10, 500)
    p = np.where(rng.random(500) < 0.6, y, rng.integers(0, 10, 500))
    p[p == 7] = 3  # class 7 never predicted: precision and F1 of that class are 0
    m = macro_metrics(y, p)
    assert m["accuracy"] == pytest.approx(accuracy_score(y, p), abs=1e-15)
    assert m["sensitivity"] == pytest.approx(recall_score(y, p, average="macro", zero_division=0), abs=1e-15)
    assert m["f1"] == pytest.approx(f1_score(y, p, average="macro", zero_division=0), abs=1e-15)
    cm = confusion_matrix(y, p)
    assert np.array_equal(m["confusion"], cm)
    fp = cm.sum(0) - np.diag(cm)
    tn = cm.sum() - cm.sum(1) - fp
    assert m["specificity"] == pytest.approx(np.mean(tn / (tn + fp)), abs=1e-15)


def test_macro_metrics_perfect_and_binary():
    y = np.array([0, 1, 1, 0, 2])
    m = macro_metrics(y, y)
    assert m["accuracy"] == m["sensitivity"] == m["specificity"] == m["f1"] == 1.0
    # binary by hand: TP=1 FN=1 FP=1 TN=1 for class 1, and the mirror for class 0
    m = macro_metrics(np.array([1, 1, 0, 0]), np.array([1, 0, 1, 0]))
    assert m["accuracy"] == 0.5 and m["sensitivity"] == 0.5 and m["specificity"] == 0.5 and m["f1"] == 0.5


def test_pca_angles_span_and_subspace():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(300, 20)) @ rng.normal(size=(20, 20))
    p = PCAAngles.fit(X, 6)
    A = p.transform(X)
    assert A.shape == (300, 6)
    assert np.allclose(A.min(0), 0.0) and np.allclose(A.max(0), math.pi)
    ref = PCA(n_components=6).fit(X)
    # same components up to sign
    assert np.allclose(np.abs(np.sum(p.components * ref.components_, axis=1)), 1.0, atol=1e-10)
    # values outside the training range are clipped to [0, pi]
    B = p.transform(X * 3.0)
    assert B.min() >= 0.0 and B.max() <= math.pi


def test_pca_angles_rejects_bad_width():
    with pytest.raises(ValueError):
        PCAAngles.fit(np.zeros((5, 3)), 4)
