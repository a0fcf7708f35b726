"""Pins of the reconstruction oracle (Secs. 4 and 5): the hand-worked
two-cell example, zero error for an exact reconstruction, and the time
average of the fields equal to the reconstruction from the time-averaged
coefficients (linearity)."""
import os

import numpy as np

from oracle.reconstruct import reconstruct, rel_l2_error_of_time_averages, time_average

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "reconstruct_2cells.txt")


def test_hand_worked_example():
    rows = {ln.split()[0]: [float(x) for x in ln.split()[1:]]
            for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")}
    F = reconstruct(np.array([[1.0], [0.0]]), np.array([[1.0, 3.0]]), np.array([0.0, 1.0]))
    np.testing.assert_array_equal(F.ravel(), rows["fields"])
    eps = rel_l2_error_of_time_averages(np.full((2, 2), 2.0), F)
    assert abs(eps - rows["eps"][0]) < 1e-15


def test_exact_reconstruction_and_linearity():
    rng = np.random.default_rng(1)
    Phi = np.linalg.qr(rng.standard_normal((50, 4)))[0]
    alpha = rng.standard_normal((4, 9))
    mean = rng.standard_normal(50)
    F = reconstruct(Phi, alpha, mean)
    assert rel_l2_error_of_time_averages(F, F) == 0.0
    np.testing.assert_allclose(time_average(F), mean + Phi @ alpha.mean(axis=1), atol=1e-14)
