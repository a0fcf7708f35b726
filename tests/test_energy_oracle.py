"""Pins of the energy oracle (Sec. 4.1, the energy criterion read with squared
singular values): the hand-worked three-mode example, the identity
||S||_F^2 = sum sigma_i^2 on matrices built from chosen singular values, and
the rank rule's edge cases."""
import os

import numpy as np
import pytest

import synth
from oracle.energy import energy, energy_sigma, frobenius2, rank_for

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "energy_3modes.txt")


def test_hand_worked_example():
    lines = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    sigma = [float(x) for x in lines[0][1:]]
    e = energy(sigma, sum(x * x for x in sigma))
    np.testing.assert_allclose(e, [9 / 14, 13 / 14, 1.0], rtol=0, atol=1e-15)
    es = energy_sigma(sigma)
    np.testing.assert_allclose(es, [3 / 6, 5 / 6, 1.0], rtol=0, atol=1e-15)
    for tag, delta, rank in lines[1:]:
        assert tag in ("delta", "sumdelta")
        assert rank_for(e if tag == "delta" else es, float(delta)) == int(rank)


@pytest.mark.parametrize("m,n,k", [(300, 40, 40), (64, 200, 64), (500, 30, 7)])
def test_frobenius_equals_sum_of_squared_singular_values(m, n, k):
    U = synth._orthonormal(m, k, 3, 1)
    V = synth._orthonormal(n, k, 3, 2)
    s = np.exp(-0.3 * np.arange(k)) * 5.0
    S = (U * s) @ V.T
    assert frobenius2(S) == pytest.approx(float(np.sum(s * s)), rel=1e-13)
    e = energy(s, frobenius2(S))
    assert e[-1] == pytest.approx(1.0, rel=1e-13)
    assert np.all(np.diff(e) >= 0)


def test_rank_rule_edges():
    e = np.array([0.5, 0.8, 0.95])
    assert rank_for(e, 0.5) == 1       # reached exactly
    assert rank_for(e, 0.96) == -1     # not reached within the sketch
    assert rank_for(e, 1e-9) == 1


def test_sum_form_against_squared_form_on_4096x200():
    """Both readings of the energy criterion on the 4096 x 200 workload
    (sigma_k = exp(-0.1 k) plus noise of std 1e-4): the sum form weighs the
    noise floor's 180-odd singular values far more than the squared form, so
    it needs more modes for the same delta. Values printed for the record."""
    g = synth.lowrank_exp(4096, 200, decay=0.1, noise_std=1e-4, seed=1)
    s = np.linalg.svd(g["St"].T.astype(np.float64), compute_uv=False)
    e2 = energy(s, frobenius2(g["St"]))
    e1 = energy_sigma(s)
    assert e2[-1] == pytest.approx(1.0, rel=1e-12) and e1[-1] == pytest.approx(1.0, rel=1e-12)
    assert np.all(e1 <= e2 + 1e-15)   # sqrt-weights spread the total: the sum form never leads
    r1, r2 = rank_for(e1, 0.9), rank_for(e2, 0.9)
    print(f"4096x200: rank for delta = 0.9: sum form {r1}, squared form {r2}; "
          f"e_20 = {e1[19]:.4f} (sum) / {e2[19]:.4f} (squared)")
    assert r1 > r2
