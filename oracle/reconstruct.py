"""Reduced-order reconstruction and its error, CPU FP64 (test infrastructure only).

Sec. 4: the reduced-order field at time t is the zeroth-order time average
plus the modes weighted by the time-dependent coefficients,
q^r(t) = q0 + sum_i alpha_i(t) phi_i. Sec. 5 scores a reduced-order model by
the relative L2 error of time-averaged fields, ||avg FOM - avg ROM|| / ||avg
FOM||; on a uniform grid the L2 norm is the Euclidean norm over the cells
times the cell area, which cancels in the ratio.
"""

import numpy as np


def reconstruct(Phi, alpha, mean=None):
    """Fields (m x T): mean + Phi alpha (Phi m x r, alpha r x T)."""
    F = np.asarray(Phi, dtype=np.float64) @ np.asarray(alpha, dtype=np.float64)
    if mean is not None:
        F = F + np.asarray(mean, dtype=np.float64)[:, None]
    return F


def time_average(F):
    """The mean over the time columns of an m x T array."""
    return np.asarray(F, dtype=np.float64).mean(axis=1)


def rel_l2_error_of_time_averages(ref, rom):
    """||avg ref - avg rom|| / ||avg ref|| for m x T arrays."""
    f = time_average(ref)
    g = time_average(rom)
    return float(np.linalg.norm(f - g) / np.linalg.norm(f))
