"""GPU parity of the energy report (Sec. 4.1, the energy criterion read with
squared singular values) through the C ABI: rpod_energy after a compute call
against the oracle's energy from O2's singular values on the same sketch and
its own ||S||_F^2; the rank rule; the bound by the exact POD energy (the
sketched singular values never exceed the true ones); error handling."""

import numpy as np
import pytest
import torch

import paper_2504_15350_amd as rp
import synth
from oracle import pod
from oracle import rpod as orpod
from oracle.energy import energy, frobenius2, rank_for

from test_gpu_parity import sketch_for, upload

pytestmark = pytest.mark.gpu
DEV = "cuda"
RTOL = {torch.float64: 3e-12, torch.float32: 3e-5, torch.bfloat16: 3e-3}  # twice the sigma tolerances, plus margin


@pytest.mark.parametrize("nx,ny,n,r,p,q,dtype", [
    (32, 32, 200, 10, 6, 1, torch.float64),
    (64, 64, 500, 20, 10, 2, torch.float32),
    (64, 64, 400, 20, 10, 2, torch.bfloat16),
])
def test_energy_matches_oracle(nx, ny, n, r, p, q, dtype):
    g = synth.fourier_field(nx, ny, n, n_modes=100, noise_std=1e-4, seed=n + r)
    m = nx * ny
    Sd, S64 = upload(g["St"], dtype)
    plan = rp.Plan(m, n, r, p, q, dtype=dtype, device=DEV, energy=True)
    plan.compute(Sd, 7)
    delta = 0.9
    e, rank = plan.energy(delta)
    plan.close()
    om = sketch_for(7, n, r + p, dtype)
    _, _, _, ex = orpod.rpod_stable(S64, r, om, q)
    fro = frobenius2(S64)
    e_ref = energy(ex["ritz"][:r + p], fro)
    print(f"[energy] e[:5]={e[:5]} rank={rank} ref rank={rank_for(e_ref, delta)}", flush=True)
    np.testing.assert_allclose(e, e_ref, rtol=RTOL[dtype], atol=0)
    if np.all(np.abs(e_ref - delta) > 10 * RTOL[dtype]):
        assert rank == rank_for(e_ref, delta)
    # sketched singular values never exceed the true ones: e_k <= the exact energy
    _, s1, _, _ = pod.pod_svd(S64, r + p)
    assert np.all(e <= energy(s1, fro) * (1 + RTOL[dtype]))


def test_energy_rank_not_reached_and_errors():
    g = synth.lowrank_exp(3000, 200, decay=0.01, noise_std=1e-3, seed=5)  # slow decay
    Sd, _ = upload(g["St"], torch.float32)
    plan = rp.Plan(3000, 200, 5, 3, 1, dtype=torch.float32, device=DEV, energy=True)
    plan.compute(Sd, 3)
    e, rank = plan.energy(0.999)
    assert rank == -1 and e[-1] < 0.999
    with pytest.raises(rp.RpodError) as err:
        plan.energy(1.5)
    assert err.value.status == 1
    plan.close()
    plain = rp.Plan(3000, 200, 5, 3, 1, dtype=torch.float32, device=DEV)
    plain.compute(Sd, 3)
    with pytest.raises(rp.RpodError) as err:
        plain.energy(0.5)
    assert err.value.status == 1
    plain.close()
