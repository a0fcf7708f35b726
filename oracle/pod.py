"""O1: deterministic POD, CPU FP64 (test infrastructure only).

POD as defined in Sec. 4.1: the thin SVD S = U Sigma V^T of the m x n
snapshot matrix (the SVD equation of Sec. 4.1), K = min(m, n), singular values
in descending order; the basis is the first r left singular vectors and the
modal coefficients are C = U_r^T S (Sec. 4.3, the coefficient matrix whose
entry (i, (k-1) N^t + p) is alpha_i(t_p, mu_k)).

Three routes, each a plain definition written out:
  pod_svd        LAPACK thin SVD (numpy.linalg.svd, gesdd).
  pod_snapshots  method of snapshots: eigen-decomposition of S^T S (n <= m) or
                 S S^T (m < n); sigma = sqrt(eigenvalue).
  pod_tsqr       streaming tall-skinny QR over row blocks (only R is kept),
                 then svd(R) = U_R Sigma V^T and Phi = S V_r Sigma_r^-1 on a
                 second pass; for matrices too large to factor whole.

Sign convention (the paper leaves it open): every mode is flipped so that
its entry of largest magnitude is positive, the lowest row index winning
ties; the coefficient row flips with it.
"""

import numpy as np


def sign_fix(Phi, A=None):
    """Flip columns of Phi (and rows of A) so each column's largest-|.| entry is > 0."""
    idx = np.argmax(np.abs(Phi), axis=0)  # first occurrence on ties
    s = np.sign(Phi[idx, np.arange(Phi.shape[1])])
    s[s == 0] = 1.0
    Phi = Phi * s[None, :]
    if A is not None:
        A = A * s[:, None]
    return Phi, A, s


def pod_svd(S, r):
    """Thin SVD of S (m x n, FP64). Returns (Phi m x r, sigma r, A r x n, sigma_all)."""
    S = np.asarray(S, dtype=np.float64)
    U, s, Vt = np.linalg.svd(S, full_matrices=False)
    Phi = U[:, :r].copy()
    A = Phi.T @ S
    Phi, A, _ = sign_fix(Phi, A)
    return Phi, s[:r].copy(), A, s


def pod_snapshots(S, r):
    """Method of snapshots: eigenvectors of the smaller Gram matrix."""
    S = np.asarray(S, dtype=np.float64)
    m, n = S.shape
    if n <= m:
        lam, W = np.linalg.eigh(S.T @ S)          # right singular vectors
        order = np.argsort(lam)[::-1]
        lam, W = lam[order], W[:, order]
        s = np.sqrt(np.clip(lam, 0.0, None))
        Phi = (S @ W[:, :r]) / s[:r][None, :]
    else:
        lam, U = np.linalg.eigh(S @ S.T)          # left singular vectors
        order = np.argsort(lam)[::-1]
        lam, U = lam[order], U[:, order]
        s = np.sqrt(np.clip(lam, 0.0, None))
        Phi = U[:, :r].copy()
    A = Phi.T @ S
    Phi, A, _ = sign_fix(Phi, A)
    return Phi, s[:r].copy(), A, s


class SnapshotMajor:
    """S (m x n) as the oracle reads it -- by row blocks -- when the caller
    holds it snapshot-major as St (n x m, one snapshot per row): a row block
    of S is the transposed view St[:, rows].T, so the blocked products run on
    that array in place (no second copy of a matrix of tens of GB)."""

    def __init__(self, St):
        self.St = St
        self.shape = (St.shape[1], St.shape[0])

    def __getitem__(self, rows):
        return self.St[:, rows].T


def row_blocks(S, block_rows):
    """Yield (row offset, FP64 copy of a row block) of a 2-D array-like S."""
    m = S.shape[0]
    for i0 in range(0, m, block_rows):
        yield i0, np.asarray(S[i0:i0 + block_rows], dtype=np.float64)


def pod_tsqr(S, r, block_rows=65536):
    """Streaming TSQR route for tall S (m >= n), FP64 arithmetic on row blocks.

    R is accumulated as R <- qr([R; S_block]).R, so only an n x n factor is
    kept; then svd(R) gives Sigma and V, and Phi = S V_r Sigma_r^-1.
    """
    m, n = S.shape
    assert m >= n, "pod_tsqr expects a tall matrix"
    R = np.zeros((0, n))
    for _, blk in row_blocks(S, block_rows):
        R = np.linalg.qr(np.vstack([R, blk]), mode="r")
    _, s, Vt = np.linalg.svd(R, full_matrices=False)
    Vr = Vt[:r].T
    Phi = np.empty((m, r))
    for i0, blk in row_blocks(S, block_rows):
        Phi[i0:i0 + blk.shape[0]] = (blk @ Vr) / s[:r][None, :]
    A = np.zeros((r, n))
    for i0, blk in row_blocks(S, block_rows):
        A += Phi[i0:i0 + blk.shape[0]].T @ blk
    Phi, A, _ = sign_fix(Phi, A)
    return Phi, s[:r].copy(), A, s


def pod_sigma_sine_field(amp, T, nx, ny):
    """Singular values of the noise-free synthetic field S0 = F diag(amp) T^T in
    closed form (the POD of Sec. 4.1 without a decomposition of S0): the
    columns of F are the sampled sine modes sin(pi a x) sin(pi b y / 2) on the
    cell centres of an nx x ny grid, mutually orthogonal with squared norm
    nx ny / 4, so S0 = (sqrt(nx ny) / 2) F_hat diag(amp) T^T with F_hat
    orthonormal and sigma(S0) = (sqrt(nx ny) / 2) sigma(diag(amp) T^T), an SVD
    of a (modes x n) matrix."""
    M = np.asarray(amp, dtype=np.float64)[:, None] * np.asarray(T, dtype=np.float64).T
    return 0.5 * np.sqrt(float(nx) * float(ny)) * np.linalg.svd(M, compute_uv=False)
