"""End-to-end quantum-kernel SVM: features -> angles -> exact MPS -> Gram -> SVC.

The paper's pipeline (§3.2, the pipeline figure) reduces images with PCA to
as many features as qubits, encodes each data point with the feature-map
circuit, computes the kernel matrix of the training set and the kernel
between test and training points (§3.4, Alg. 2), and trains a support vector
classifier on the precomputed kernel; it reports accuracy and the macro
averages of sensitivity, specificity and F1 (§4.2.2, Table macro_metrics).

Here the two Gram matrices come from the HIP library (qsvm_encode_mps,
qsvm_gram_sym, qsvm_gram through the binding), the classifier is
scikit-learn's SVC on the precomputed kernel (the learner the paper's QSVC
wraps), and PCA and the metrics are small host-side NumPy steps.

Readings where the paper is silent:
  * PCA is fitted on the training set (centred, top n_qubits right singular
    vectors); each component is then mapped linearly to [0, pi] with the
    training set's minimum and maximum, and test values are clipped to that
    range (the paper does not say how components become angles).
  * Without PCA the features must already be angles in [0, pi].
  * Multi-class SVC is one-vs-one (scikit-learn's default).
  * Specificity of class c is TN / (TN + FP) with class c as the positive
    class; every macro average weighs the classes equally.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import qsvm


@dataclass
class PCAAngles:
    """PCA to n components followed by a per-component map onto [0, pi]."""

    mean: np.ndarray
    components: np.ndarray  # n x d
    lo: np.ndarray
    hi: np.ndarray

    @classmethod
    def fit(cls, X: np.ndarray, n_components: int) -> "PCAAngles":
        X = np.asarray(X, dtype=np.float64)
        if not 1 <= n_components <= min(X.shape):
            raise ValueError(f"n_components = {n_components} outside [1, {min(X.shape)}]")
        mean = X.mean(axis=0)
        _, _, vt = np.linalg.svd(X - mean, full_matrices=False)
        comp = vt[:n_components]
        Z = (X - mean) @ comp.T
        return cls(mean, comp, Z.min(axis=0), Z.max(axis=0))

    def transform(self, X: np.ndarray) -> np.ndarray:
        Z = (np.asarray(X, dtype=np.float64) - self.mean) @ self.components.T
        span = np.where(self.hi > self.lo, self.hi - self.lo, 1.0)
        return np.clip((Z - self.lo) / span, 0.0, 1.0) * math.pi


def macro_metrics(y_true, y_pred, labels=None) -> dict:
    """Accuracy and macro-averaged sensitivity, specificity and F1 from the
    confusion matrix (the measures of Table macro_metrics)."""
    y_true = np.asarray(y_true)
    y_pred = np.asarray(y_pred)
    labels = np.unique(np.concatenate([y_true, y_pred])) if labels is None else np.asarray(labels)
    idx = {c: k for k, c in enumerate(labels.tolist())}
    L = labels.shape[0]
    cm = np.zeros((L, L), dtype=np.int64)  # rows: true class, columns: predicted class
    for t, p in zip(y_true.tolist(), y_pred.tolist()):
        cm[idx[t], idx[p]] += 1
    tp = np.diag(cm).astype(np.float64)
    fn = cm.sum(axis=1) - tp
    fp = cm.sum(axis=0) - tp
    tn = cm.sum() - tp - fn - fp

    def ratio(a, b):
        return np.divide(a, b, out=np.zeros_like(a), where=b > 0)

    sens = ratio(tp, tp + fn)
    spec = ratio(tn, tn + fp)
    prec = ratio(tp, tp + fp)
    f1 = ratio(2.0 * prec * sens, prec + sens)
    return {
        "accuracy": float(tp.sum() / max(1, cm.sum())),
        "sensitivity": float(sens.mean()),
        "specificity": float(spec.mean()),
        "f1": float(f1.mean()),
        "confusion": cm,
        "labels": labels,
    }


class QSVC:
    """Support vector classifier on the exact quantum kernel of the ZZ feature
    map (K computed by the library's MPS contraction on the GPU)."""

    def __init__(self, reps: int = 2, C: float = 1.0, n_qubits: int | None = None, device="cuda:0"):
        self.reps = reps
        self.C = C
        self.n_qubits = n_qubits
        self.device = device
        self.pca: PCAAngles | None = None
        self._train_mps = None
        self.svc = None
        self.K_train = None

    def _angles(self, X: np.ndarray) -> np.ndarray:
        if self.pca is not None:
            return self.pca.transform(X)
        A = np.asarray(X, dtype=np.float64)
        if A.min() < 0.0 or A.max() > math.pi:
            raise ValueError("without PCA the features must be angles in [0, pi]")
        return A

    def _encode(self, A: np.ndarray):
        import torch

        return qsvm.qsvm_encode_mps(torch.as_tensor(np.ascontiguousarray(A), device=self.device), self.reps)

    def fit(self, X, y) -> "QSVC":
        from sklearn.svm import SVC

        X = np.asarray(X, dtype=np.float64)
        if self.n_qubits is not None and self.n_qubits != X.shape[1]:
            self.pca = PCAAngles.fit(X, self.n_qubits)
        A = self._angles(X)
        self._train_mps = self._encode(A)
        self.K_train = qsvm.qsvm_gram_sym(self._train_mps).cpu().numpy()
        self.svc = SVC(kernel="precomputed", C=self.C)
        self.svc.fit(self.K_train, np.asarray(y))
        return self

    def kernel(self, X) -> np.ndarray:
        """K[i][j] = |<psi(x_train_j)|psi(x_i)>|^2 for the rows of X."""
        if self._train_mps is None:
            raise RuntimeError("fit() first")
        m = self._encode(self._angles(np.asarray(X, dtype=np.float64)))
        return qsvm.qsvm_gram(m, self._train_mps).cpu().numpy()

    def predict(self, X, K=None) -> np.ndarray:
        K = self.kernel(X) if K is None else K
        return self.svc.predict(K)

    def evaluate(self, X, y) -> dict:
        K = self.kernel(X)
        pred = self.predict(X, K)
        m = macro_metrics(np.asarray(y), pred, labels=np.unique(np.concatenate([np.asarray(y), self.svc.classes_])))
        m["predictions"] = pred
        m["K_test"] = K
        return m
