"""Seeded synthetic snapshot matrices (inputs only; no rPOD arithmetic here).

The paper's quasi-geostrophic snapshots are not public, so tests and the
benchmark use synthetic matrices with the same layout: an m x n snapshot
matrix S (m grid cells, n snapshots), stored column-major, i.e. as a row-major
array St of shape (n, m) whose row t is snapshot t (Sec. 4.1, the snapshot
matrix collects one field per column).

Both the GPU path and the CPU oracle draw their inputs from this module.
Every generator is keyed by (seed, stream, column) through numpy's
SeedSequence, so the matrix does not depend on how it is chunked.

Generators
----------
lowrank_exp     S = U diag(sigma) V^T + noise, U and V orthonormal from the
                Householder QR of seeded Gaussian matrices (diag(R) > 0),
                sigma_k = exp(-decay k), k = 1..K.
fourier_field   a QG-like field on a cell-centred nx x ny grid of
                [0,1] x [0,2]: each snapshot is a sum of the n_modes
                lowest Dirichlet modes sin(kx x) sin(ky y),
                kx = pi a, ky = pi b / 2, with amplitude |k|^-beta times a
                stationary unit-variance AR(1) series, plus white noise.
add_block_means adds a time average per parameter block (Sec. 4.1: the
                columns form blocks of N^t consecutive snapshots, one block
                per parameter): a random combination of the 12 lowest
                Fourier modes per block, scaled to a given RMS, added to
                every column of that block.
batch_shapes    the shapes of an uneven batch: m in {2^16, 2^17, 2^18},
                n in [500, 4000], r in {10, 25, 50, 100}, decay in
                [0.05, 0.2], all drawn per matrix from the seed.
"""

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

# stream ids: 1 = U, 2 = V, 3 = noise, 4 = AR(1) series, 5 = shape draws
_S_U, _S_V, _S_NOISE, _S_AR, _S_SHAPE = 1, 2, 3, 4, 5


def rng(seed, stream, *extra):
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(stream), *map(int, extra)]))


def _orthonormal(rows, cols, seed, stream):
    """Q of the Householder QR of a seeded rows x cols Gaussian matrix, diag(R) > 0."""
    G = rng(seed, stream).standard_normal((rows, cols))
    Q, R = np.linalg.qr(G, mode="reduced")
    return Q * np.sign(np.diag(R))[None, :]


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


def _add_noise(St, noise_std, seed, col0=0):
    """Add i.i.d. N(0, noise_std^2) noise; column t uses its own stream (seed, 3, t)."""
    if noise_std == 0.0:
        return St
    m = St.shape[1]

    def one(t):
        St[t] += noise_std * rng(seed, _S_NOISE, col0 + t).standard_normal(m).astype(St.dtype)

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(one, range(St.shape[0])))
    return St


def lowrank_exp(m, n, decay=0.1, noise_std=1e-4, seed=1, K=None, dtype=np.float64):
    """S = U diag(exp(-decay k)) V^T + noise, returned as St (n, m) plus factors.

    K defaults to min(m, n). noise_std is the standard deviation of the
    Gaussian noise (variance noise_std**2).
    """
    K = min(m, n) if K is None else K
    U = _orthonormal(m, K, seed, _S_U)
    V = _orthonormal(n, K, seed, _S_V)
    sigma = np.exp(-decay * np.arange(1, K + 1))
    St = (V * sigma[None, :]) @ U.T          # (n, m) = (U diag(s) V^T)^T
    St = np.ascontiguousarray(St)
    _add_noise(St, noise_std, seed)
    return dict(St=St.astype(dtype, copy=False), U=U, V=V, sigma=sigma)


def fourier_modes(nx, ny, n_modes):
    """The n_modes lowest modes (a, b), a, b >= 1, ordered by |k| then a then b.

    |k|^2 = pi^2 (a^2 + b^2 / 4); the integer key 4 a^2 + b^2 orders it exactly.
    Only a < nx and b < ny are used, where the sampled sines are orthogonal.
    """
    amax = min(nx - 1, 4 * int(np.sqrt(n_modes)) + 8)
    bmax = min(ny - 1, 8 * int(np.sqrt(n_modes)) + 16)
    cand = [(4 * a * a + b * b, a, b) for a in range(1, amax + 1) for b in range(1, bmax + 1)]
    cand.sort()
    if len(cand) < n_modes:
        raise ValueError("grid too small for the requested number of modes")
    modes = np.array([(a, b) for _, a, b in cand[:n_modes]], dtype=np.int64)
    kmag = np.pi * np.sqrt(modes[:, 0] ** 2 + modes[:, 1] ** 2 / 4.0)
    return modes, kmag


def fourier_basis(nx, ny, modes):
    """F (m x n_modes): column = sin(kx x_i) sin(ky y_j) at cell centres, row = i + nx j.

    x_i = (i + 1/2)/nx on [0,1], y_j = 2 (j + 1/2)/ny on [0,2], so
    kx x_i = pi a (i + 1/2)/nx and ky y_j = pi b (j + 1/2)/ny.
    Columns are exactly orthogonal with squared norm nx ny / 4.
    """
    ix = np.arange(nx) + 0.5
    iy = np.arange(ny) + 0.5
    sx = np.sin(np.pi * np.outer(modes[:, 0], ix) / nx)   # (K, nx)
    sy = np.sin(np.pi * np.outer(modes[:, 1], iy) / ny)   # (K, ny)
    F = (sy[:, :, None] * sx[:, None, :]).reshape(len(modes), nx * ny)
    return F.T


def ar1_series(n, k, phi, seed, stream=_S_AR):
    """k independent stationary unit-variance AR(1) series of length n: (n, k)."""
    eps = rng(seed, stream).standard_normal((n, k))
    T = np.empty((n, k))
    T[0] = eps[0]
    c = np.sqrt(1.0 - phi * phi)
    for t in range(1, n):
        T[t] = phi * T[t - 1] + c * eps[t]
    return T


def fourier_field(nx, ny, n, n_modes=200, beta=1.5, phi=0.95, noise_std=1e-4, seed=2,
                  dtype=np.float64, col_block=512, amp_scale=None):
    """QG-like snapshot field; returns dict(St=(n, m) array, modes, kmag, amp, T, ...).

    Snapshot t = sum_k amp_k T[t, k] F[:, k] + noise, amp_k = |k|^-beta
    (times amp_scale[k] when given).
    """
    m = nx * ny
    modes, kmag = fourier_modes(nx, ny, n_modes)
    amp = kmag ** (-beta)
    if amp_scale is not None:
        amp = amp * np.asarray(amp_scale)
    T = ar1_series(n, n_modes, phi, seed)
    F = fourier_basis(nx, ny, modes)                       # (m, K)
    St = np.empty((n, m), dtype=dtype)
    C = T * amp[None, :]                                   # (n, K)
    for t0 in range(0, n, col_block):
        t1 = min(n, t0 + col_block)
        blk = C[t0:t1] @ F.T
        _add_noise(blk, noise_std, seed, col0=t0)
        St[t0:t1] = blk
    return dict(St=St, modes=modes, kmag=kmag, amp=amp, T=T, nx=nx, ny=ny)



def fourier_field_device(nx, ny, n, n_modes=200, beta=1.5, phi=0.95, noise_std=1e-4, seed=3,
                         dtype=None, device="cuda", col_block=512):
    """fourier_field() built on the GPU with torch (FP32 arithmetic), for sizes
    too large to generate on the host. Same modes, amplitudes and AR(1) series
    (drawn on the host from the same streams); the white noise comes from a
    seeded torch generator on the device, so the matrix equals the host
    generator's only up to the noise draw. Returns St (n, nx*ny) on device.
    """
    import torch

    dtype = torch.float32 if dtype is None else dtype
    m = nx * ny
    modes, kmag = fourier_modes(nx, ny, n_modes)
    amp = kmag ** (-beta)
    T = ar1_series(n, n_modes, phi, seed)
    dev = torch.device(device)
    ix = torch.arange(nx, dtype=torch.float64, device=dev) + 0.5
    iy = torch.arange(ny, dtype=torch.float64, device=dev) + 0.5
    ma = torch.as_tensor(modes[:, 0], dtype=torch.float64, device=dev)
    mb = torch.as_tensor(modes[:, 1], dtype=torch.float64, device=dev)
    sx = torch.sin(torch.pi * ma[:, None] * ix[None, :] / nx)
    sy = torch.sin(torch.pi * mb[:, None] * iy[None, :] / ny)
    F = (sy[:, :, None] * sx[:, None, :]).reshape(n_modes, m).to(torch.float32)     # (K, m)
    C = torch.as_tensor(T * amp[None, :], dtype=torch.float32, device=dev)          # (n, K)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed) * 1000003 + _S_NOISE)
    St = torch.empty((n, m), dtype=dtype, device=dev)
    for t0 in range(0, n, col_block):
        t1 = min(n, t0 + col_block)
        blk = C[t0:t1] @ F
        if noise_std:
            blk += noise_std * torch.randn((t1 - t0, m), generator=gen, device=dev, dtype=torch.float32)
        St[t0:t1] = blk.to(dtype)
    return dict(St=St, modes=modes, kmag=kmag, amp=amp, T=T, nx=nx, ny=ny)


# ---------------------------------------------------------------------------
# uneven batches
# ---------------------------------------------------------------------------

BATCH_RANKS = (10, 25, 50, 100)


def batch_shapes(count=64, seed=4):
    """Shapes of an uneven batch of snapshot matrices, drawn from stream 5.

    Per matrix (m, n, r, alpha): m = 2^k with k uniform in {16, 17, 18},
    n a uniform integer in [500, 4000], r uniform in {10, 25, 50, 100} and
    the spectral decay alpha uniform in [0.05, 0.2]. r + 10 <= n always.
    """
    g = rng(seed, _S_SHAPE)
    out = []
    for _ in range(count):
        m = 1 << int(g.integers(16, 19))
        n = int(g.integers(500, 4001))
        r = int(BATCH_RANKS[int(g.integers(0, len(BATCH_RANKS)))])
        alpha = float(g.uniform(0.05, 0.2))
        out.append((m, n, r, alpha))
    return out


def lowrank_exp_device(m, n, decay, noise_std=1e-4, seed=1, K=256, dtype=None, device="cuda"):
    """S = U diag(exp(-decay k)) V^T + noise built on the GPU with torch, as
    St (n, m): U (m x K) and V (n x K) orthonormalised from seeded Gaussian
    matrices by CholeskyQR twice (FP32 products on the device, the K x K
    Cholesky factor and its inverse in FP64 on the host), noise
    N(0, noise_std^2) from a seeded torch generator. Only plain FP32 matrix
    products run on the device. For sizes too large for the host; not
    bitwise equal to lowrank_exp()."""
    import torch

    dtype = torch.float32 if dtype is None else dtype
    dev = torch.device(device)
    K = min(K, n, m)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed) * 1000003 + _S_U)

    def orth(rows):
        X = torch.randn((rows, K), generator=gen, device=dev, dtype=torch.float32)
        for _ in range(2):
            G = (X.T.contiguous() @ X).to("cpu", torch.float64)
            Rinv = np.linalg.inv(np.linalg.cholesky(G.numpy()).T)
            X = X @ torch.from_numpy(Rinv.astype(np.float32)).to(dev)
        return X

    U = orth(m)
    V = orth(n)
    sig = torch.from_numpy(np.exp(-decay * np.arange(1, K + 1)).astype(np.float32)).to(dev)
    C = V * sig[None, :]                              # (n, K)
    U32 = U.T.contiguous()                            # (K, m)
    del U, V
    St = torch.empty((n, m), dtype=dtype, device=dev)
    gen.manual_seed(int(seed) * 1000003 + _S_NOISE)
    for t0 in range(0, n, 512):
        t1 = min(n, t0 + 512)
        blk = C[t0:t1] @ U32
        if noise_std:
            blk += noise_std * torch.randn((t1 - t0, m), generator=gen, device=dev, dtype=torch.float32)
        St[t0:t1] = blk.to(dtype)
    return St


# ---------------------------------------------------------------------------
# parametric family for the learned warm start
# ---------------------------------------------------------------------------
# stream ids: 6 = skew generators, 7 = parameter draws, 8 = train/test split
_S_SKEW, _S_MU, _S_SPLIT, _S_MEAN = 6, 7, 8, 9

# physical box of the parameter vector (delta, sigma, Fr, alpha), mapped to [-1, 1]^4
PARAM_BOX = np.array([[0.2, 0.6], [0.006, 0.01], [0.07, 0.11], [0.05, 0.2]])


def normalise_mu(mu):
    mu = np.asarray(mu, dtype=np.float64)
    return 2.0 * (mu - PARAM_BOX[:, 0]) / (PARAM_BOX[:, 1] - PARAM_BOX[:, 0]) - 1.0


def draw_params(count=128, seed=5):
    """count parameter vectors uniform in PARAM_BOX: (physical (count, 4), normalised (count, 4))."""
    g = rng(seed, _S_MU)
    u = g.uniform(size=(count, 4))
    mu = PARAM_BOX[:, 0] + u * (PARAM_BOX[:, 1] - PARAM_BOX[:, 0])
    return mu, normalise_mu(mu)


def train_test_split(count=128, n_train=96, seed=5):
    perm = rng(seed, _S_SPLIT).permutation(count)
    return np.sort(perm[:n_train]), np.sort(perm[n_train:])


def farthest_points(X, k):
    """k row indices of X by farthest-point sampling, starting nearest the origin."""
    X = np.asarray(X, dtype=np.float64)
    idx = [int(np.argmin(np.sum(X * X, axis=1)))]
    d = np.sum((X - X[idx[0]]) ** 2, axis=1)
    while len(idx) < k:
        j = int(np.argmax(d))
        idx.append(j)
        d = np.minimum(d, np.sum((X - X[j]) ** 2, axis=1))
    return idx


class ParamFamily:
    """S(mu) = U(mu) diag(exp(-alpha k)) V^T + noise on an nx x ny grid.

    U(mu) = F expm(sum_j mu_j G_j)[:, :K]: F holds the n_cand lowest
    orthonormal Dirichlet sine modes of the grid (fourier_basis scaled to unit
    norm), G_j are seeded skew-symmetric n_cand x n_cand matrices (stream 6)
    scaled by `angle`/||G_j||_2 (so that the leading 50-dimensional subspaces
    at opposite corners of the box are about 30 degrees apart), mu is the
    normalised parameter vector in [-1, 1]^4 and alpha its physical fourth
    component. U(mu) is orthonormal
    and smooth in mu. V (n x K) is the Q factor of a seeded Gaussian matrix
    per matrix seed; the noise is N(0, noise_std^2) per column stream.
    """

    def __init__(self, nx, ny, n_cand=400, K=100, angle=0.205, family_seed=5):
        self.nx, self.ny, self.K = nx, ny, K
        modes, _ = fourier_modes(nx, ny, n_cand)
        self.F = fourier_basis(nx, ny, modes) / np.sqrt(nx * ny / 4.0)    # (m, n_cand), orthonormal
        g = rng(family_seed, _S_SKEW)
        self.G = []
        for _ in range(4):
            A = g.standard_normal((n_cand, n_cand))
            Sk = 0.5 * (A - A.T)
            self.G.append(Sk * (angle / np.linalg.norm(Sk, 2)))

    @property
    def m(self):
        return self.nx * self.ny

    def rotation(self, mu_hat):
        from scipy.linalg import expm
        M = sum(float(a) * Gj for a, Gj in zip(mu_hat, self.G))
        return expm(M)

    def U(self, mu_hat):
        return self.F @ self.rotation(mu_hat)[:, :self.K]

    @staticmethod
    def spectrum(alpha, K):
        return np.exp(-alpha * np.arange(1, K + 1))

    def matrix(self, mu, n, noise_std=1e-7, seed=0, dtype=np.float64):
        """Host St (n, m) for the physical parameter vector mu; also U, V, sigma."""
        mu = np.asarray(mu, dtype=np.float64)
        U = self.U(normalise_mu(mu))
        V = _orthonormal(n, self.K, seed, _S_V)
        s = self.spectrum(mu[3], self.K)
        St = np.ascontiguousarray((V * s[None, :]) @ U.T)
        _add_noise(St, noise_std, seed)
        return dict(St=St.astype(dtype, copy=False), U=U, V=V, sigma=s)

    def matrix_device(self, mu, n, noise_std=1e-7, seed=0, dtype=None, device="cuda", F_dev=None):
        """matrix() built on the GPU with FP32 products (U from the host
        rotation); the noise comes from a seeded torch generator."""
        import torch
        dtype = torch.float32 if dtype is None else dtype
        dev = torch.device(device)
        mu = np.asarray(mu, dtype=np.float64)
        if F_dev is None:
            F_dev = torch.from_numpy(self.F.astype(np.float32)).to(dev)
        R = self.rotation(normalise_mu(mu))[:, :self.K]
        s = self.spectrum(mu[3], self.K)
        V = _orthonormal(n, self.K, seed, _S_V)
        U32t = (F_dev @ torch.from_numpy(R.astype(np.float32)).to(dev)).T.contiguous()   # (K, m)
        C = torch.from_numpy((V * s[None, :]).astype(np.float32)).to(dev)                 # (n, K)
        gen = torch.Generator(device=dev)
        gen.manual_seed(int(seed) * 1000003 + _S_NOISE)
        St = torch.empty((n, self.m), dtype=dtype, device=dev)
        for t0 in range(0, n, 512):
            t1 = min(n, t0 + 512)
            blk = C[t0:t1] @ U32t
            if noise_std:
                blk += noise_std * torch.randn((t1 - t0, self.m), generator=gen, device=dev, dtype=torch.float32)
            St[t0:t1] = blk.to(dtype)
        return St


def add_block_means(St, nx, ny, block_cols, rms, seed):
    """St (n, m) plus a smooth field per block of block_cols rows of St (in place).

    Block k's field is sum_i c_ki F_i over the 12 lowest Fourier modes F_i,
    c_ki ~ N(0, 1) from (seed, stream _S_MEAN), scaled to element RMS `rms`.
    Returns the (m, K) fields that were added, in FP64.
    """
    n, m = St.shape
    K = n // block_cols
    modes, _ = fourier_modes(nx, ny, 12)
    F = fourier_basis(nx, ny, modes)                        # (m, 12)
    c = rng(seed, _S_MEAN).standard_normal((12, K))
    means = F @ c
    means *= rms / np.sqrt(np.mean(means * means))
    for k in range(K):
        St[k * block_cols:(k + 1) * block_cols] += means[:, k].astype(St.dtype)[None, :]
    return means
