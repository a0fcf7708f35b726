"""O2: randomized POD, CPU FP64 (test infrastructure only).

Alg. 1 of Sec. 4.2 ("randomized POD with subspace iterations"), taken step by
step in the paper's order:
  1. Gaussian sketch Lambda (n x l, l = r + p), passed in as data here;
  2. sampled matrix P = S Lambda;
  3. q subspace iterations P <- (S S^T)^q P;
  4. P = Q R (QR decomposition);
  5. T = Q^T S;
  6. SVD T = U_hat Sigma V^T;
  7. U = Q U_hat, whose first r columns are the basis (Sec. 4.2, text after
     the lift), and C = U_r^T S are the coefficients (Sec. 4.3).

rpod_stable() re-orthonormalises after every product with S or S^T (step 3
written as alternating QR factorisations). In exact arithmetic this spans
the same space as step 3 and so returns the same modes, values and
coefficients; it avoids the loss of the trailing directions that the
unnormalised powers suffer in floating point. rpod_literal() performs step 3
exactly as printed and exists to check that equivalence.

S may be any 2-D array-like (numpy array, memmap, FP32 or FP64); products
with S run over row blocks, upcast to FP64.
"""

import numpy as np

from .pod import sign_fix, row_blocks

_BLOCK = 65536


def s_times(S, X, block_rows=_BLOCK):
    """S @ X in FP64, streaming S by row blocks."""
    m = S.shape[0]
    out = np.empty((m, X.shape[1]))
    for i0, blk in row_blocks(S, block_rows):
        out[i0:i0 + blk.shape[0]] = blk @ X
    return out


def st_times(S, Q, block_rows=_BLOCK):
    """S^T @ Q in FP64, streaming S by row blocks."""
    out = np.zeros((S.shape[1], Q.shape[1]))
    for i0, blk in row_blocks(S, block_rows):
        out += blk.T @ Q[i0:i0 + blk.shape[0]]
    return out


def _orth(Y):
    """Orthonormal basis of range(Y) by Householder QR (LAPACK geqrf/orgqr)."""
    Q, _ = np.linalg.qr(Y, mode="reduced")
    return Q


def _finish(S, Q, r, block_rows, literal_A=True):
    """Steps 5-7 plus the coefficients: T = Q^T S, SVD, lift, C = U_r^T S.

    literal_A=False takes C = Sigma_r V_r^T from the SVD of T instead of a
    further pass over S (equal in exact arithmetic, since T = Q^T S and
    Phi = Q U_hat_r give U_r^T S = U_hat_r^T T); for matrices so large that
    one more pass matters."""
    T = st_times(S, Q, block_rows).T             # step 5: l x n
    Uh, s, Vt = np.linalg.svd(T, full_matrices=False)   # step 6
    Phi = Q @ Uh[:, :r]                          # step 7, first r columns
    if literal_A:
        A = st_times(S, Phi, block_rows).T       # C = U_r^T S, computed literally
    else:
        A = s[:r, None] * Vt[:r]
    Phi, A, signs = sign_fix(Phi, A)
    Vt_r = Vt[:r] * signs[:, None]
    return Phi, s[:r].copy(), A, dict(ritz=s, Vt_r=Vt_r, T=T, Q=Q, U_hat=Uh)


def rpod_stable(S, r, omega, q, block_rows=_BLOCK, literal_A=True):
    """Alg. 1 with re-orthonormalisation after every product.

    omega: n x l FP64 sketch (step 1 drawn by the caller). Returns
    (Phi m x r, sigma r, A r x n, extras).
    """
    omega = np.asarray(omega, dtype=np.float64)
    Q = _orth(s_times(S, omega, block_rows))              # steps 2 and 4
    for _ in range(q):                                    # step 3, stable form
        Z = _orth(st_times(S, Q, block_rows))
        Q = _orth(s_times(S, Z, block_rows))
    return _finish(S, Q, r, block_rows, literal_A)


def rpod_literal(S, r, omega, q, block_rows=_BLOCK):
    """Alg. 1 exactly as printed: powers of S S^T without intermediate QR."""
    omega = np.asarray(omega, dtype=np.float64)
    P = s_times(S, omega, block_rows)                     # step 2
    for _ in range(q):                                    # step 3
        P = s_times(S, st_times(S, P, block_rows), block_rows)
    Q = _orth(P)                                          # step 4
    return _finish(S, Q, r, block_rows)
