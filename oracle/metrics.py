"""Sign- and rotation-invariant comparison metrics (test infrastructure).

Singular vectors are fixed only up to sign, and only up to a rotation inside
a cluster of equal singular values, so results are compared through
quantities that do not depend on those choices.
"""

import numpy as np


def sigma_rel_err(s_test, s_ref):
    """max_k |s_test_k - s_ref_k| / s_ref_k."""
    s_test = np.asarray(s_test, dtype=np.float64)
    s_ref = np.asarray(s_ref, dtype=np.float64)
    return float(np.max(np.abs(s_test - s_ref) / np.abs(s_ref)))


def sin_theta_max(Phi_test, Phi_ref):
    """Sine of the largest principal angle between range(Phi_test) and range(Phi_ref).

    Phi_test is re-orthonormalised in FP64 first; Phi_ref must be orthonormal.
    Computed as || Q_t - Phi_ref (Phi_ref^T Q_t) ||_2 (the sine form, which
    stays accurate at small angles).
    """
    Qt, _ = np.linalg.qr(np.asarray(Phi_test, dtype=np.float64))
    Pr = np.asarray(Phi_ref, dtype=np.float64)
    D = Qt - Pr @ (Pr.T @ Qt)
    return float(np.linalg.norm(D, 2))


def per_mode_sin(Phi_test, Phi_ref):
    """Per-column sine of the angle between matching columns (sign-invariant)."""
    Pt = np.asarray(Phi_test, dtype=np.float64)
    Pr = np.asarray(Phi_ref, dtype=np.float64)
    Pt = Pt / np.linalg.norm(Pt, axis=0, keepdims=True)
    Pr = Pr / np.linalg.norm(Pr, axis=0, keepdims=True)
    c = np.sum(Pt * Pr, axis=0)
    return np.linalg.norm(Pt - Pr * c[None, :], axis=0)


def orth_err(Phi):
    """max |Phi^T Phi - I|."""
    Phi = np.asarray(Phi, dtype=np.float64)
    return float(np.max(np.abs(Phi.T @ Phi - np.eye(Phi.shape[1]))))


def lowrank_rel_diff(Phi_t, A_t, Phi_r, A_r):
    """|| Phi_t A_t - Phi_r A_r ||_F / || A_r ||_F without forming m x n products.

    With W = [Phi_t, Phi_r] = Q_W R_W and H = [A_t; -A_r], the difference is
    Q_W (R_W H), whose Frobenius norm equals || R_W H ||_F. Invariant to the
    sign and rotation freedom of the modes. Phi_r must be orthonormal.
    """
    W = np.hstack([np.asarray(Phi_t, np.float64), np.asarray(Phi_r, np.float64)])
    H = np.vstack([np.asarray(A_t, np.float64), -np.asarray(A_r, np.float64)])
    _, Rw = np.linalg.qr(W, mode="reduced")
    return float(np.linalg.norm(Rw @ H) / np.linalg.norm(A_r))


def gap_ok(s, k, rel=1e-3):
    """True when the cut after mode k (1-based count) has relative gap >= rel."""
    s = np.asarray(s, dtype=np.float64)
    if k >= len(s):
        return True
    return (s[k - 1] - s[k]) / s[k - 1] >= rel
