"""Rounding the SDP solution to scaled rotations (test infrastructure: oracle only).

Prop. "SDP Relaxation" and the paragraph after it: take the top three
eigenvectors of X = U^T U, project each 3x3 block to a scaled rotation, and
anchor with the first block (U* = Rbar_1^T Ubar).  The paper does not say how
the sign/reflection ambiguity of the eigenvectors is settled; reading used
(listed in the design notes): if most blocks have negative determinant, the
third row of Ubar is negated (X is unchanged), then each block M = A S B^T
(SVD) becomes R = A diag(1, 1, det(A B^T)) B^T with scale tr(R^T M) / 3.
"""
from __future__ import annotations

import numpy as np


def top3_factor(U, method="auto"):
    """Ubar (3 x 3N) with Ubar^T Ubar the best rank-3 approximation of X = U^T U.

    method "dense": eigendecomposition of X itself (3N x 3N); "gram": the same
    eigenpairs from the r x r Gram U U^T (identical nonzero spectrum: if
    U U^T v = mu v then X (U^T v) = mu U^T v, and |U^T v|^2 = mu for unit v);
    "auto": dense for 3N <= 6000, gram above."""
    n = U.shape[1]
    if method == "dense" or (method == "auto" and n <= 6000):
        mu, E = np.linalg.eigh(U.T @ U)
        idx = np.argsort(mu)[::-1][:3]
        return np.sqrt(np.maximum(mu[idx], 0.0))[:, None] * E[:, idx].T
    mu, V = np.linalg.eigh(U @ U.T)
    idx = np.argsort(mu)[::-1][:3]
    return V[:, idx].T @ U


def project_scaled_rotation(M):
    """Nearest s R (R in SO(3), s > 0) to a 3x3 block M in Frobenius norm."""
    A, S, Bt = np.linalg.svd(M)
    d = np.sign(np.linalg.det(A @ Bt))
    D = np.diag([1.0, 1.0, d if d != 0 else 1.0])
    R = A @ D @ Bt
    s = float(np.trace(R.T @ M)) / 3.0
    return R, s


def round_solution(U, method="auto"):
    """Rounded, anchored rotations R_hat [N,3,3] and scales s_hat [N]."""
    N = U.shape[1] // 3
    Ub = top3_factor(U, method)
    dets = np.array([np.linalg.det(Ub[:, 3 * k:3 * k + 3]) for k in range(N)])
    if np.sum(dets < 0) > N / 2:
        Ub[2, :] = -Ub[2, :]
    Rs = np.empty((N, 3, 3))
    ss = np.empty(N)
    for k in range(N):
        Rs[k], ss[k] = project_scaled_rotation(Ub[:, 3 * k:3 * k + 3])
    R_hat = np.einsum("ji,njk->nik", Rs[0], Rs)      # R_0^T R_k
    s_hat = ss / ss[0]
    return R_hat, s_hat


def rounded_U(R_hat, s_hat):
    """U_hat = [s_0 R_0, ..., s_{N-1} R_{N-1}] (3 x 3N), feasible for the
    scaled-rotation-only problem."""
    N = R_hat.shape[0]
    return (s_hat[:, None, None] * R_hat).transpose(1, 0, 2).reshape(3, 3 * N)
