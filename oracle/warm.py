"""Learned warm start for randomized POD, CPU FP64 oracle (test infrastructure only).

The paper has no warm start; this is an extension of its Alg. 1 (Sec. 4.2):
a small network maps a parameter vector to a predicted subspace of the
snapshot matrix, which takes the place of most Gaussian sketch columns.
Everything here follows the plain definitions below; it shares no code with
the GPU library.

Definitions
-----------
Bank: K orthonormal bases Phi_1..Phi_K (m x r each), [Phi] = [Phi_1 .. Phi_K].
  G_W = [Phi]^T [Phi] (Kr x Kr), G8[k, l] = ||Phi_k^T Phi_l||_F^2.
Network (4 -> 256 -> 256 -> K, tanh, softmax):
  h1 = tanh(W1 mu + b1), h2 = tanh(W2 h1 + b2), z = W3 h2 + b3, c = softmax(z).
Loss of a training pair (mu_i, Phi_i), with P(c) = sum_k c_k Phi_k Phi_k^T:
  L_i = ||Phi_i Phi_i^T - P(c)||_F^2 = r - 2 b_i^T c + c^T G8 c,
  b_ik = ||Phi_k^T Phi_i||_F^2; the training loss is the mean over pairs.
Optimiser: Adam with L2 weight decay added to the gradient (the convention
  of torch.optim.Adam), bias-corrected moments.
Predicted subspace: W = P(c)^j Phi_k*, k* = argmax c (lowest index on ties):
  j steps of subspace iteration on P(c) started from the bank basis of
  largest weight. In the bank's coordinates W = [Phi] Z with
  Z_0 = E_k* (the columns of block k*) and Z <- C (G_W Z), C = diag(c (x) 1_r).
  A one-hot c gives W = Phi_k exactly.
Warm rPOD: Y = [W, S Omega_p] (Omega_p the first p columns of the Gaussian
  sketch), Q = orth(Y), q subspace iterations as in Alg. 1 (stable form),
  then steps 5-7 of Alg. 1 and the coefficients.
Per-mode residual of the returned modes (the acceptance rule of warm plans):
  with v_k = A_k^T / sigma_k (A = Phi^T S = Sigma V^T), the singular triplet
  (phi_k, sigma_k, v_k) of S has residual r_k = S v_k - sigma_k phi_k (its
  other half S^T phi_k - sigma_k v_k vanishes by construction), and
  rho = max_{k <= r} ||r_k|| / sigma_k. For the exact SVD rho = 0, and by
  the residual bound for the symmetric matrix [[0, S], [S^T, 0]] some
  singular value of S lies within ||r_k|| of sigma_k, so rho <= tol bounds
  every sigma_k's relative error by tol to first order.
Fallback by continuation: when rho > tol, q_fb further subspace iterations
  run from the warm range basis Q (Z = orth(S^T Q), Q = orth(S Z)), then
  steps 5-7 of Alg. 1 again; the warm work is kept, not repeated.
"""

import numpy as np

from .rpod import _finish, _orth, s_times, st_times

IN, HIDDEN = 4, 256
PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def param_shapes(K=8):
    return {"W1": (HIDDEN, IN), "b1": (HIDDEN,), "W2": (HIDDEN, HIDDEN), "b2": (HIDDEN,),
            "W3": (K, HIDDEN), "b3": (K,)}


def softmax(z):
    z = z - np.max(z, axis=-1, keepdims=True)
    e = np.exp(z)
    return e / np.sum(e, axis=-1, keepdims=True)


def mlp_forward(P, X):
    """X (N x 4) -> dict(h1, h2, z, c), all FP64."""
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ P["W1"].T + P["b1"])
    h2 = np.tanh(h1 @ P["W2"].T + P["b2"])
    z = h2 @ P["W3"].T + P["b3"]
    return dict(h1=h1, h2=h2, z=z, c=softmax(z))


def bank_gram(bases):
    Phi = np.hstack([np.asarray(b, dtype=np.float64) for b in bases])
    return Phi.T @ Phi


def block_gram(GW, K, r):
    """G8[k, l] = ||Phi_k^T Phi_l||_F^2 from the blocks of G_W."""
    G8 = np.empty((K, K))
    for k in range(K):
        for l in range(K):
            G8[k, l] = np.sum(GW[k * r:(k + 1) * r, l * r:(l + 1) * r] ** 2)
    return G8


def targets(bases, Phi_i):
    Phi_i = np.asarray(Phi_i, dtype=np.float64)
    return np.array([np.sum((np.asarray(b, dtype=np.float64).T @ Phi_i) ** 2) for b in bases])


def loss(P, X, B, G8, r):
    """Mean loss and per-pair losses."""
    c = mlp_forward(P, X)["c"]
    B = np.asarray(B, dtype=np.float64)
    per = r - 2.0 * np.sum(B * c, axis=1) + np.einsum("ik,kl,il->i", c, G8, c)
    return float(np.mean(per)), per


def backward(P, X, B, G8):
    """Analytic gradient of the mean loss with respect to every parameter."""
    X = np.asarray(X, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    N = X.shape[0]
    f = mlp_forward(P, X)
    c, h1, h2 = f["c"], f["h1"], f["h2"]
    dc = (2.0 / N) * (c @ G8.T - B)                      # dL/dc (G8 is symmetric)
    dz = c * (dc - np.sum(c * dc, axis=1, keepdims=True))  # softmax Jacobian
    g = {"W3": dz.T @ h2, "b3": dz.sum(axis=0)}
    da2 = (dz @ P["W3"]) * (1.0 - h2 * h2)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ P["W2"]) * (1.0 - h1 * h1)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(axis=0)
    return g


def adam_step(P, g, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=1e-5):
    """One Adam step in place on P; state holds t and the moments m, v."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in PARAM_ORDER:
        gk = g[k] + weight_decay * P[k]
        m = state.setdefault("m", {}).setdefault(k, np.zeros_like(P[k]))
        v = state.setdefault("v", {}).setdefault(k, np.zeros_like(P[k]))
        m *= beta1
        m += (1.0 - beta1) * gk
        v *= beta2
        v += (1.0 - beta2) * gk * gk
        mh = m / (1.0 - beta1 ** t)
        vh = v / (1.0 - beta2 ** t)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
    return P


def argmax_first(c):
    c = np.asarray(c)
    return int(np.flatnonzero(c == np.max(c))[0])


def assemble(GW, c, kstar, r, j=2):
    """Z (Kr x r) with W = [Phi] Z = P(c)^j Phi_k*."""
    Kr = GW.shape[0]
    Z = np.zeros((Kr, r))
    Z[kstar * r:(kstar + 1) * r, :] = np.eye(r)
    w = np.repeat(np.asarray(c, dtype=np.float64), r)
    for _ in range(j):
        Z = w[:, None] * (GW @ Z)
    return Z


def warm_rpod(S, bases, c, kstar, r, omega_p, q, j=2):
    """Warm-started rPOD; returns (Phi, sigma, A, extras) with extras['rho'],
    extras['rho_modes'] the per-mode residual of the result."""
    Phi_b = np.hstack([np.asarray(b, dtype=np.float64) for b in bases])
    Z = assemble(Phi_b.T @ Phi_b, c, kstar, r, j)
    W = Phi_b @ Z
    Y = np.hstack([W, s_times(S, np.asarray(omega_p, dtype=np.float64))])
    Q = _orth(Y)
    for _ in range(q):
        Zs = _orth(st_times(S, Q))
        Q = _orth(s_times(S, Zs))
    Phi, s, A, ex = _finish(S, Q, r, 65536)
    ex["rho"], ex["rho_modes"] = mode_residual(S, Phi, s, A)
    ex["W"] = W
    return Phi, s, A, ex


def mode_residual(S, Phi, sigma, A):
    """rho = max_k ||S v_k - sigma_k phi_k|| / sigma_k with v_k = A_k^T / sigma_k,
    and the per-mode values (S m x n, Phi m x r, sigma r, A r x n)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    V = np.asarray(A, dtype=np.float64).T / sigma[None, :]
    R = s_times(S, V) - np.asarray(Phi, dtype=np.float64) * sigma[None, :]
    per = np.linalg.norm(R, axis=0) / sigma
    return float(np.max(per)), per


def warm_rpod_continued(S, bases, c, kstar, r, omega_p, q, tol, q_fb, j=2):
    """Warm-started rPOD with the per-mode acceptance rule: the warm result if
    rho <= tol, else q_fb further subspace iterations from the warm range basis
    and steps 5-7 again. Returns (Phi, sigma, A, extras) with extras['rho'] the
    warm result's residual and extras['fell_back']."""
    Phi_b = np.hstack([np.asarray(b, dtype=np.float64) for b in bases])
    Z = assemble(Phi_b.T @ Phi_b, c, kstar, r, j)
    Y = np.hstack([Phi_b @ Z, s_times(S, np.asarray(omega_p, dtype=np.float64))])
    Q = _orth(Y)
    for _ in range(q):
        Q = _orth(s_times(S, _orth(st_times(S, Q))))
    Phi, s, A, ex = _finish(S, Q, r, 65536)
    rho, per = mode_residual(S, Phi, s, A)
    ex.update(rho=rho, rho_modes=per, fell_back=bool(rho > tol))
    if rho > tol:
        for _ in range(q_fb):
            Q = _orth(s_times(S, _orth(st_times(S, Q))))
        Phi, s, A, ex2 = _finish(S, Q, r, 65536)
        ex2.update(rho=rho, rho_modes=per, fell_back=True)
        ex = ex2
    return Phi, s, A, ex
