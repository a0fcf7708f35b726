"""Fluctuation snapshots, CPU FP64 (test infrastructure only).

Sec. 4.1: before POD, every snapshot is replaced by its fluctuation about the
time average of its own parameter. The snapshot matrix holds, for parameter
k = 1..M, the N^t time instants of that parameter as consecutive columns
(columns (k-1) N^t .. k N^t - 1, zero-based), so the time average of
parameter k is the mean of that block of columns and the fluctuation matrix
is S' = S - [mean_1 1^T, ..., mean_M 1^T].

fluctuations() is that definition written out (an explicit FP64 subtraction,
block by block). The GPU library never forms S'; it centres the products with
S algebraically. The oracle's randomized POD of the fluctuations is rpod_stable
applied to the array this function returns.
"""

import numpy as np


def block_means(S, block_cols):
    """The M = n / block_cols time averages (m x M, FP64), one per block."""
    S = np.asarray(S, dtype=np.float64)
    m, n = S.shape
    if block_cols < 1 or n % block_cols != 0:
        raise ValueError("n must be a positive multiple of block_cols")
    M = n // block_cols
    out = np.empty((m, M))
    for k in range(M):
        out[:, k] = S[:, k * block_cols:(k + 1) * block_cols].mean(axis=1)
    return out


def fluctuations(S, block_cols):
    """S' = S minus the time average of each column's block (FP64 copy)."""
    S = np.asarray(S, dtype=np.float64)
    means = block_means(S, block_cols)
    out = S.copy()
    for k in range(means.shape[1]):
        out[:, k * block_cols:(k + 1) * block_cols] -= means[:, k:k + 1]
    return out
