"""Oracle: SVD basis of training frequency tracks (test infrastructure only).

Sec. II C factorises the matrix of training tracks f_{i,alpha} with the SVD
(Eq. (9)) and searches over coefficients of the leading right singular vectors
(Eq. (10)); the coefficient prior is uniform inside symmetric 3-sigma quantiles
of the training projections.

Readings:
* the basis is centred: f0[alpha] is the mean training track and the SVD is
  taken of the centred matrix, so a track is f0 + sum_k c_k U[:, k] (an
  uncentred basis is the special case f0 = 0);
* sign rule: each column is flipped so that its largest-magnitude entry is
  positive (the lowest index wins a magnitude tie);
* "symmetric 3 sigma quantiles" = the 0.135 % and 99.865 % quantiles of each
  projection column, with linear interpolation between order statistics.
"""
from __future__ import annotations

import numpy as np

BOX_Q_LO = 0.00135
BOX_Q_HI = 0.99865


def centre_tracks(F: np.ndarray):
    """Mean track f0[alpha] and the centred matrix F - f0."""
    f0 = F.mean(axis=0)
    return f0, F - f0[None, :]


def leading_right_vectors(X: np.ndarray, K: int):
    """Thin SVD X = A diag(s) V^T (Eq. (9)); the first K columns of V and all s."""
    _, s, vt = np.linalg.svd(X, full_matrices=False)
    return vt[:K].T.copy(), s


def apply_sign_rule(U: np.ndarray) -> np.ndarray:
    """Flip each column so that its largest-magnitude entry (first on ties) is positive."""
    U = U.copy()
    for k in range(U.shape[1]):
        pivot = int(np.argmax(np.abs(U[:, k])))
        if U[pivot, k] < 0:
            U[:, k] = -U[:, k]
    return U


def coefficient_box(C: np.ndarray):
    """Per-column 0.135 % / 99.865 % quantiles (linear interpolation)."""
    if C.shape[1] == 0:
        return np.zeros(0), np.zeros(0)
    lo = np.quantile(C, BOX_Q_LO, axis=0, method="linear")
    hi = np.quantile(C, BOX_Q_HI, axis=0, method="linear")
    return np.asarray(lo), np.asarray(hi)


def build_basis(tracks, K: int):
    """Return (f0[n_seg], U[n_seg, K], sv[K], box_lo[K], box_hi[K]), all FP64."""
    F = np.asarray(tracks, dtype=np.float64)
    n_train, n_seg = F.shape
    K = int(K)
    if K < 0 or K > min(n_train, n_seg):
        raise ValueError("K out of range")
    f0, X = centre_tracks(F)
    U, s = leading_right_vectors(X, K)
    U = apply_sign_rule(U)
    box_lo, box_hi = coefficient_box(X @ U)
    return f0, U, s[:K].copy(), box_lo, box_hi
