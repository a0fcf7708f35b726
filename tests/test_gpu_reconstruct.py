"""GPU parity of the reduced-order reconstruction (Sec. 4) and the relative L2
error of time-averaged fields (Sec. 5) through the C ABI, against the oracle;
and the ROM loop closed on synthetic data: rPOD of the fluctuations, then the
fields rebuilt from the time average plus the modes and their coefficients."""

import numpy as np
import pytest
import torch

import paper_2504_15350_amd as rp
import synth
from oracle.center import block_means
from oracle.reconstruct import reconstruct, rel_l2_error_of_time_averages

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.mark.parametrize("m,r,T,dtype,with_mean", [
    (1000, 7, 33, torch.float64, True),
    (70000, 50, 300, torch.float32, True),
    (4099, 128, 17, torch.float32, False),   # ragged rows, r = 128, T below one tile
])
def test_reconstruct_matches_oracle(m, r, T, dtype, with_mean):
    rng = np.random.default_rng(m + r)
    Phi = np.linalg.qr(rng.standard_normal((m, r)))[0]
    alpha = rng.standard_normal((r, T)) * 10.0
    mean = rng.standard_normal(m) if with_mean else None
    ref = reconstruct(Phi, alpha, mean) + 1e-2 * rng.standard_normal((m, T))
    npd = np.float64 if dtype == torch.float64 else np.float32
    Phi_r, alpha_r = Phi.astype(npd), alpha.astype(npd)
    mean_r = mean.astype(npd) if with_mean else None
    ref_r = ref.astype(npd)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    F_t, eps = rp.reconstruct(t(Phi_r.T), t(alpha_r.T), t(mean_r) if with_mean else None, t(ref_r.T))
    F_ref = reconstruct(Phi_r, alpha_r, mean_r)
    tol = 1e-12 if dtype == torch.float64 else 2e-6
    F = F_t.double().cpu().numpy().T
    assert np.max(np.abs(F - F_ref)) <= tol * np.max(np.abs(F_ref))
    e_ref = rel_l2_error_of_time_averages(ref_r, F_ref)
    assert abs(eps - e_ref) <= (1e-10 if dtype == torch.float64 else 1e-5) * e_ref
    # exact reconstruction: zero error up to rounding
    _, eps0 = rp.reconstruct(t(Phi_r.T), t(alpha_r.T), t(mean_r) if with_mean else None,
                             t(reconstruct(Phi_r, alpha_r, mean_r).astype(npd).T), want_fields=False)
    assert eps0 < (1e-13 if dtype == torch.float64 else 1e-6)


def test_rom_loop_on_fluctuations():
    # rPOD of the fluctuations of one parameter block, then q = time average + Phi A
    nx, ny, n, r = 64, 64, 400, 40
    g = synth.fourier_field(nx, ny, n, n_modes=60, noise_std=1e-4, seed=8)
    St = g["St"]
    synth.add_block_means(St, nx, ny, n, float(np.sqrt(np.mean(St * St))), 8)
    m = nx * ny
    Sd = torch.from_numpy(St.astype(np.float32)).to(DEV)
    plan = rp.Plan(m, n, r, 10, 2, dtype=torch.float32, device=DEV, block_cols=n)
    Phi_t, sig, A_t = plan.compute(Sd, 3)
    plan.close()
    S64 = St.astype(np.float32).astype(np.float64).T
    q0 = block_means(S64, n)[:, 0]
    F_t, eps = rp.reconstruct(Phi_t, A_t.contiguous(), torch.from_numpy(q0.astype(np.float32)).to(DEV), Sd)
    F = F_t.double().cpu().numpy().T
    # the coefficients of the fluctuations sum to zero over time, so the time
    # average of the reduced-order fields is q0 itself and eps is tiny
    assert eps < 1e-5
    # the fields themselves: the error is the discarded modes' share
    rel = np.linalg.norm(F - S64) / np.linalg.norm(S64 - q0[:, None])
    sv = np.linalg.svd(S64 - q0[:, None], compute_uv=False)
    assert rel <= 1.01 * np.sqrt(np.sum(sv[r:] ** 2) / np.sum(sv ** 2)) + 1e-4
