"""Cost, Riemannian gradient, Hessian and retraction (test infrastructure: oracle only).

Prop. "BM Riemannian Optimization": the rank-r Burer-Monteiro problem
(Prop. "BM Factorization") is unconstrained optimisation of tr(Q U^T U) over
U = [R_1, s_2 R_2, ..., s_N R_N] with R_i on the Stiefel manifold
St(r, 3) = {R in R^{r x 3} : R^T R = I3} and s_i on the positive manifold.
Frame 0 here is the paper's frame 1 (s_0 = 1 fixed, R_0 free).

The paper fixes the manifold but not the metric or the retraction formulas
beyond "QR by Gram-Schmidt" for the Stiefel factor.  Readings used (listed in
the design notes):
  * Stiefel factor: embedded (Euclidean) metric, projection
    P_R(Z) = Z - R sym(R^T Z), Riemannian Hessian = projected directional
    derivative of the Euclidean gradient minus the Weingarten term
    P_R(Zdot - Rdot sym(R^T Z)).
  * Positive factor: metric <a, b>_s = a b / s^2 (Euclidean in log s), so
    grad_s = s^2 df/ds, Hess_s[sdot] = s^2 d(df/ds) + s (df/ds) sdot, and the
    retraction s <- s exp(sdot / s).
  * Stiefel retraction: Gram-Schmidt orthonormalisation of the columns of
    R + Rdot (QR with positive diagonal).

A point is (R [N, r, 3], s [N]); a tangent vector is (Rd [N, r, 3], sd [N])
with sd[0] = 0.  U (the paper's flat r x 3N matrix) has column 3k+c equal to
s_k R_k[:, c].

Scale regularisation (App. "Scale Regularization", eq. problem-sdp-scale):
the objective gains lam sum_{i>=2} (X_{3i,3i} - 1)^2.  On the manifold every
diagonal block of X = U^T U is s_k^2 I, so the term is
F(s) = lam sum_{k>=1} (s_k^2 - 1)^2, a function of the scales alone: its
Euclidean derivative is dF/ds_k = 4 lam s_k (s_k^2 - 1) and its second
derivative 4 lam (3 s_k^2 - 1).  Every function below takes `lam` (0: the
plain problem).
"""
from __future__ import annotations

import numpy as np


def sym(A):
    return 0.5 * (A + np.swapaxes(A, -1, -2))


def to_U(R, s):
    """U = [s_0 R_0, ..., s_{N-1} R_{N-1}]  (r x 3N)."""
    N, r, _ = R.shape
    return (s[:, None, None] * R).transpose(1, 0, 2).reshape(r, 3 * N)


def blocks(G, N):
    """Split an r x 3N matrix into its N blocks of size r x 3."""
    r = G.shape[0]
    return G.reshape(r, N, 3).transpose(1, 0, 2)


def scale_reg(s, lam):
    """F = lam sum_{k>=1} (s_k^2 - 1)^2."""
    return lam * float(np.sum((s[1:] ** 2 - 1.0) ** 2))


def cost(Q, R, s, lam=0.0):
    """f = tr(Q U^T U) + F(s)."""
    U = to_U(R, s)
    return float(np.sum(U * (U @ Q))) + scale_reg(s, lam)


def euclid_parts(Q, R, s):
    """Gamma = 2 U Q (blocks), E_k = df/dR_k = s_k Gamma_k, e_k = df/ds_k = <R_k, Gamma_k>."""
    N = R.shape[0]
    U = to_U(R, s)
    Gam = blocks(2.0 * (U @ Q), N)
    E = s[:, None, None] * Gam
    e = np.einsum("nab,nab->n", R, Gam)
    return Gam, E, e


def proj(R, Z):
    """Orthogonal projection onto the tangent space of St(r,3) at R."""
    return Z - R @ sym(np.swapaxes(R, 1, 2) @ Z)


def rgrad(Q, R, s, lam=0.0):
    """Riemannian gradient (gR [N,r,3], gs [N]) with gs[0] = 0 (s_0 anchored)."""
    Gam, E, e = euclid_parts(Q, R, s)
    gR = proj(R, E)
    gs = s * s * (e + 4.0 * lam * s * (s * s - 1.0))
    gs[0] = 0.0
    return gR, gs


def hess(Q, R, s, Rd, sd, lam=0.0):
    """Riemannian Hessian applied to the tangent vector (Rd, sd)."""
    N = R.shape[0]
    Gam, E, e = euclid_parts(Q, R, s)
    Ud = (sd[:, None, None] * R + s[:, None, None] * Rd).transpose(1, 0, 2).reshape(R.shape[1], 3 * N)
    Gd = blocks(2.0 * (Ud @ Q), N)
    Ed = sd[:, None, None] * Gam + s[:, None, None] * Gd
    ed = np.einsum("nab,nab->n", Rd, Gam) + np.einsum("nab,nab->n", R, Gd)
    HR = proj(R, Ed - Rd @ sym(np.swapaxes(R, 1, 2) @ E))
    Hs = s * s * ed + s * e * sd
    # F(s): s^2 F'' sd + s F' sd
    Hs = Hs + (s * s * 4.0 * lam * (3.0 * s * s - 1.0) + s * 4.0 * lam * s * (s * s - 1.0)) * sd
    Hs[0] = 0.0
    return HR, Hs


def inner(s, aR, as_, bR, bs):
    """Metric: sum <aR_k, bR_k> + sum_{k>=1} as_k bs_k / s_k^2."""
    return float(np.sum(aR * bR) + np.sum((as_ * bs)[1:] / (s[1:] ** 2)))


def gram_schmidt(A):
    """Columns of each r x 3 block orthonormalised in order (positive-diagonal QR)."""
    Qm = np.empty_like(A)
    for c in range(A.shape[2]):
        v = A[:, :, c].copy()
        for d in range(c):
            v -= np.sum(Qm[:, :, d] * v, axis=1, keepdims=True) * Qm[:, :, d]
        Qm[:, :, c] = v / np.linalg.norm(v, axis=1, keepdims=True)
    return Qm


def retract(R, s, Rd, sd):
    """R <- qf(R + Rd) (Gram-Schmidt), s <- s exp(sd / s); s_0 stays 1."""
    Rn = gram_schmidt(R + Rd)
    sn = s * np.exp(sd / s)
    sn[0] = 1.0
    return Rn, sn


def initial_point(N, r):
    """U^0 = [I3, ..., I3] (Algorithm "Riemannian Staircase", initialisation),
    padded with zero rows when r > 3."""
    R = np.zeros((N, r, 3))
    R[:, 0, 0] = R[:, 1, 1] = R[:, 2, 2] = 1.0
    return R, np.ones(N)


def from_U(U):
    """Split a feasible U (blocks with U_k^T U_k = alpha_k I) into (R, s), s_0 = 1."""
    r, n3 = U.shape
    N = n3 // 3
    B = blocks(U, N)
    s = np.sqrt(np.einsum("nab,nab->n", B, B) / 3.0)
    R = B / s[:, None, None]
    return R, s
