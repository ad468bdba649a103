"""Gradients of the certified optimum w.r.t. keypoints and weights (test infrastructure: oracle only).

The paper does not differentiate its solver; this is the build's reading
(listed in the design notes).  theta = (u_o, w_o) over all observations.

Cost.  f*(theta) = min over (U, t, p) of sum_o w_o ||U_i u_o + t_i - p_k||^2
(eq. sba with U_i = s_i R_i).  theta does not enter the constraints, so by
the envelope theorem, with e_o = U_i u_o + t_i - p_k at the optimum:
    df*/du_o = 2 w_o U_i^T e_o,      df*/dw_o = ||e_o||^2.

Rotations and scales.  At a tight optimum the rounded anchored solution
(R_hat, s_hat) is the unique minimiser in the chart where frame 0 is fixed.
Two references are provided:
  * ift_grad: Riemannian implicit-function theorem,
      dl/dtheta = -d/dtheta [ Df(x*; theta)[lam] ],  H lam = grad l,
    with H the Riemannian Hessian of the anchored problem (frame 0 removed).
    Df[lam] = sum_o 2 w_o <e_o, e^lam_o>, where e^lam_o uses the ambient
    direction Udot_k = lam_s,k R_k + s_k lam_R,k and the inner minimiser
    (t^lam, p^lam) for that direction, which gives
      dl/du_o = -2 w_o (U_i^T e^lam_o + Udot_i^T e_o),
      dl/dw_o = -2 <e_o, e^lam_o>.
  * dense_reference: coordinates x = (omega_k, sigma_k), k >= 1, with
    R_k = R_hat_k expm([omega_k]_x), s_k = s_hat_k exp(sigma_k); the Hessian
    of f in x is obtained exactly by polarising the quadratic Taylor term,
    the mixed derivative along a direction v of theta by central differences
    of Q(theta), and dx/dtheta . v = -H^{-1} d_theta grad f . v.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import data_matrix as dm
from . import manifold as mf


def anchored_U(R_hat, s_hat):
    N = R_hat.shape[0]
    return (s_hat[:, None, None] * R_hat).transpose(1, 0, 2).reshape(3, 3 * N)


def residuals(frame, landmark, u, Y, t, p):
    """e_o = Y_i u_o + t_i - p_k  (n x r)."""
    N = Y.shape[1] // 3
    Yb = Y.reshape(Y.shape[0], N, 3).transpose(1, 0, 2)
    return np.einsum("nab,nb->na", Yb[frame], u) + t[frame] - p[landmark]


def cost_grad(N, M, frame, landmark, u, w, Y):
    """Envelope gradient of the optimal cost: (df/du [n,3], df/dw [n])."""
    t, p = dm.recover_tp(N, M, frame, landmark, u, w, Y)
    e = residuals(frame, landmark, u, Y, t, p)
    Yb = Y.reshape(Y.shape[0], N, 3).transpose(1, 0, 2)
    gu = 2.0 * w[:, None] * np.einsum("nab,na->nb", Yb[frame], e)
    gw = np.sum(e * e, axis=1)
    return gu, gw


def anchored_hess_apply(Q, R, s, Rd, sd):
    """Riemannian Hessian of the anchored problem (frame 0 fixed)."""
    Rd = Rd.copy(); sd = sd.copy()
    Rd[0] = 0.0; sd[0] = 0.0
    HR, Hs = mf.hess(Q, R, s, Rd, sd)
    HR[0] = 0.0; Hs[0] = 0.0
    return HR, Hs


def ift_grad(N, M, frame, landmark, u, w, R_hat, s_hat, gR, gs, Q=None):
    """dl/du, dl/dw for l with Euclidean partials gR [N,3,3] (d l / d R_hat) and gs [N]."""
    if Q is None:
        Q = dm.q_block_elimination(N, M, frame, landmark, u, w)
    R, s = R_hat.copy(), s_hat.copy()
    # Riemannian gradient of l on the anchored manifold
    bR = mf.proj(R, gR)
    bs = s * s * gs
    bR[0] = 0.0; bs[0] = 0.0
    # dense solve of H lam = b in the metric: build H column by column on a basis
    dims = []
    for k in range(1, N):
        for m in range(3):
            W = np.zeros((3, 3)); a, b = [(1, 2), (0, 2), (0, 1)][m]
            W[a, b], W[b, a] = 1.0, -1.0
            dims.append(("R", k, R[k] @ W / np.sqrt(2.0)))
        dims.append(("s", k, s[k]))
    n = len(dims)

    def vec(i):
        Rd = np.zeros_like(R); sd = np.zeros_like(s)
        kind, k, val = dims[i]
        if kind == "R":
            Rd[k] = val
        else:
            sd[k] = val
        return Rd, sd

    basis = [vec(i) for i in range(n)]          # orthonormal in the metric
    H = np.zeros((n, n))
    for j in range(n):
        HR, Hs = anchored_hess_apply(Q, R, s, *basis[j])
        for i in range(n):
            H[i, j] = mf.inner(s, basis[i][0], basis[i][1], HR, Hs)
    rhs = np.array([mf.inner(s, basis[i][0], basis[i][1], bR, bs) for i in range(n)])
    coef = np.linalg.solve(0.5 * (H + H.T), rhs)
    lamR = sum(c * b[0] for c, b in zip(coef, basis))
    lams = sum(c * b[1] for c, b in zip(coef, basis))
    Y = anchored_U(R, s)
    Yd = (lams[:, None, None] * R + s[:, None, None] * lamR).transpose(1, 0, 2).reshape(3, 3 * N)
    t, p = dm.recover_tp(N, M, frame, landmark, u, w, Y)
    tl, pl = dm.recover_tp(N, M, frame, landmark, u, w, Yd)
    e = residuals(frame, landmark, u, Y, t, p)
    el = residuals(frame, landmark, u, Yd, tl, pl)
    Yb = Y.reshape(3, N, 3).transpose(1, 0, 2)
    Ydb = Yd.reshape(3, N, 3).transpose(1, 0, 2)
    gu = -2.0 * w[:, None] * (np.einsum("nab,na->nb", Yb[frame], el) + np.einsum("nab,na->nb", Ydb[frame], e))
    gw = -2.0 * np.sum(e * el, axis=1)
    return gu, gw


# ---- dense chart reference ----------------------------------------------------
def _skew(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def _chart_parts(R_hat, s_hat, x):
    """U0, U1(x), U2(x): the constant, linear and quadratic Taylor terms of U(x)."""
    N = R_hat.shape[0]
    U0 = anchored_U(R_hat, s_hat)
    U1 = np.zeros_like(U0)
    U2 = np.zeros_like(U0)
    for k in range(1, N):
        om = x[4 * (k - 1):4 * (k - 1) + 3]
        sg = x[4 * (k - 1) + 3]
        W = _skew(om)
        base = s_hat[k] * R_hat[k]
        U1[:, 3 * k:3 * k + 3] = base @ (sg * np.eye(3) + W)
        U2[:, 3 * k:3 * k + 3] = base @ (0.5 * sg * sg * np.eye(3) + sg * W + 0.5 * W @ W)
    return U0, U1, U2


def chart_hessian(Q, R_hat, s_hat):
    """Exact Hessian of f(x) = tr(Q U(x)^T U(x)) at x = 0 by polarising the
    quadratic Taylor term q(x) = <U1, Q U1> + 2 <U0, Q U2>  (f = f0 + g x + q(x))."""
    n = 4 * (R_hat.shape[0] - 1)

    def q(x):
        U0, U1, U2 = _chart_parts(R_hat, s_hat, x)
        return float(np.sum(U1 * (U1 @ Q)) + 2.0 * np.sum(U0 * (U2 @ Q)))

    E = np.eye(n)
    qd = np.array([q(E[i]) for i in range(n)])
    H = np.zeros((n, n))
    for i in range(n):
        H[i, i] = 2.0 * qd[i]
        for j in range(i + 1, n):
            H[i, j] = H[j, i] = q(E[i] + E[j]) - qd[i] - qd[j]
    return H


def chart_gradient(Q, R_hat, s_hat):
    """g_i = 2 <U0, Q U1(e_i)> (the linear Taylor term)."""
    n = 4 * (R_hat.shape[0] - 1)
    E = np.eye(n)
    U0 = anchored_U(R_hat, s_hat)
    QU0 = Q @ U0.T
    g = np.zeros(n)
    for i in range(n):
        _, U1, _ = _chart_parts(R_hat, s_hat, E[i])
        g[i] = 2.0 * np.sum(U1 * QU0.T)
    return g


def dense_reference(N, M, frame, landmark, u, w, R_hat, s_hat, gR, gs, vu, vw, h=1e-5):
    """<dl/dtheta, v> for l with partials (gR, gs) along the direction v = (vu, vw)."""
    Q = dm.q_block_elimination(N, M, frame, landmark, u, w)
    H = chart_hessian(Q, R_hat, s_hat)
    Qp = dm.q_block_elimination(N, M, frame, landmark, u + h * vu, w + h * vw)
    Qm = dm.q_block_elimination(N, M, frame, landmark, u - h * vu, w - h * vw)
    dg = (chart_gradient(Qp, R_hat, s_hat) - chart_gradient(Qm, R_hat, s_hat)) / (2 * h)
    dx = -np.linalg.solve(H, dg)
    # chain rule to (R, s): dR_k = R_hat_k [d omega]_x, ds_k = s_hat_k d sigma
    total = 0.0
    for k in range(1, N):
        om = dx[4 * (k - 1):4 * (k - 1) + 3]
        sg = dx[4 * (k - 1) + 3]
        total += float(np.sum(gR[k] * (R_hat[k] @ _skew(om)))) + gs[k] * s_hat[k] * sg
    return total
