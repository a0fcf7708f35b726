"""Adaptive-rank randomized POD, CPU FP64 (test infrastructure only).

Sec. 4.1 picks the number of modes by an energy threshold, while Alg. 1 of
Sec. 4.2 needs the sketch width l = r + p before it starts. This module grows
l block by block until the threshold is met, with the blocked
fixed-accuracy range finder of Yu, Gu and Li (SIAM J. Matrix Anal. Appl. 39,
2018, algorithm randQB_EI), written out in its published order:

  E = ||S||_F^2, Q = [], B = []
  for block i = 1, 2, ...  (b columns each, until l_max):
      Q_i = orth(S Omega_i - Q (B Omega_i))
      q times:  Z_i = orth(S^T Q_i - B^T (Q^T Q_i))
                Q_i = orth(S Z_i - Q (B Z_i))
      Q_i = orth(Q_i - Q (Q^T Q_i))            (re-orthogonalisation)
      B_i = Q_i^T S;  Q = [Q, Q_i];  B = [B; B_i]
      E = E - ||B_i||_F^2
      stop when E <= (1 - delta) ||S||_F^2

E is the exact squared Frobenius error ||S - Q B||_F^2 (Q orthonormal, so
||S - Q Q^T S||_F^2 = ||S||_F^2 - ||Q^T S||_F^2). Omega_i are columns
(i-1) b .. i b - 1 of one Gaussian sketch, passed in as data. Steps 6-7 of
Alg. 1 then run on B: B = U_hat Sigma V^T, Phi = Q U_hat, A = Sigma V^T. The
rank is the energy rule of Sec. 4.1 in its squared form (the denominator is
||S||_F^2): the smallest r with sigma_1^2 + .. + sigma_r^2 >= delta ||S||_F^2,
which the stopping rule guarantees to exist among the l computed values.

With q = 0 the union of the blocks spans S Omega[:, :l], so the result equals
the non-adaptive O2 with the same l columns of the sketch.
"""

import numpy as np

from .energy import frobenius2
from .pod import sign_fix
from .rpod import _BLOCK, _orth, s_times, st_times


def rand_qb_ei(S, omega, b, q, delta, l_max, block_rows=_BLOCK):
    """Blocked adaptive range finder; returns (Q m x l, B l x n, info) with
    info = dict(l, blocks, fro2, E (the residual indicator after each block))."""
    omega = np.asarray(omega, dtype=np.float64)
    m, n = S.shape
    if l_max % b != 0 or omega.shape[1] < l_max:
        raise ValueError("l_max must be a multiple of b and omega must hold l_max columns")
    fro2 = frobenius2(S, block_rows)
    E = fro2
    Q = np.zeros((m, 0))
    B = np.zeros((0, n))
    trace = []
    for i in range(l_max // b):
        Om = omega[:, i * b:(i + 1) * b]
        Qi = _orth(s_times(S, Om, block_rows) - Q @ (B @ Om))
        for _ in range(q):
            Zi = _orth(st_times(S, Qi, block_rows) - B.T @ (Q.T @ Qi))
            Qi = _orth(s_times(S, Zi, block_rows) - Q @ (B @ Zi))
        Qi = _orth(Qi - Q @ (Q.T @ Qi))
        Bi = st_times(S, Qi, block_rows).T
        Q = np.hstack([Q, Qi])
        B = np.vstack([B, Bi])
        E = E - float(np.sum(Bi * Bi))
        trace.append(E)
        if E <= (1.0 - delta) * fro2:
            break
    return Q, B, dict(l=Q.shape[1], blocks=len(trace), fro2=fro2, E=trace)


def rpod_adaptive(S, omega, b, q, delta, l_max, block_rows=_BLOCK):
    """Adaptive rPOD: the range finder above, then steps 6-7 of Alg. 1 on B.
    Returns (Phi m x l, sigma l, A l x n, info); info adds r (the energy rank,
    or -1 when the l_max columns fall short of delta) and the energies e_k."""
    Q, B, info = rand_qb_ei(S, omega, b, q, delta, l_max, block_rows)
    Uh, s, Vt = np.linalg.svd(B, full_matrices=False)
    Phi = Q @ Uh
    A = s[:, None] * Vt
    Phi, A, _ = sign_fix(Phi, A)
    e = np.cumsum(s * s) / info["fro2"]
    hit = np.nonzero(e >= delta)[0]
    info.update(r=int(hit[0]) + 1 if hit.size else -1, energy=e)
    return Phi, s, A, info
