"""Energy of the leading modes, CPU FP64 (test infrastructure only).

Sec. 4.1 picks the number of POD modes as the smallest N^r whose share of the
singular-value total reaches a threshold delta. The paper's tables report the
share as an eigenvalue energy, so it is read here with squared singular
values: e_k = (sigma_1^2 + .. + sigma_k^2) / (sum over all i of sigma_i^2),
and the denominator is ||S||_F^2 (the sum of all squared singular values).
The form the energy criterion prints, with singular values themselves
(sum of the first k over the sum of all), is `energy_sigma`: it needs every
singular value of S, so only the exact POD can give it.
"""

import numpy as np

from .pod import row_blocks


def frobenius2(S, block_rows=65536):
    """||S||_F^2 in FP64, as the plain sum of the squared entries."""
    tot = 0.0
    for _, blk in row_blocks(S, block_rows):
        b = np.asarray(blk, dtype=np.float64)
        tot += float(np.sum(b * b))
    return tot


def energy(sigma_lead, fro2):
    """e_k for k = 1..len(sigma_lead) from the leading singular values."""
    s = np.asarray(sigma_lead, dtype=np.float64)
    return np.cumsum(s * s) / fro2


def rank_for(e, delta):
    """The smallest k (1-based) with e_k >= delta, or -1 when none reaches it."""
    hit = np.nonzero(np.asarray(e) >= delta)[0]
    return int(hit[0]) + 1 if hit.size else -1


def energy_sigma(sigma_all):
    """The criterion as printed in Sec. 4.1: (sigma_1 + .. + sigma_k) / (sum of
    all singular values), k = 1..len(sigma_all); sigma_all must hold every
    singular value of S (the thin SVD's full list)."""
    s = np.asarray(sigma_all, dtype=np.float64)
    return np.cumsum(s) / np.sum(s)
