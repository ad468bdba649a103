"""Algorithm "Riemannian Staircase" (test infrastructure: oracle only).

r = 3, U^0 = [I, ..., I]; loop: local optimisation at rank r (RTR-tCG), dual
certificate, return if Z is PSD, otherwise escape along the least eigenvector
(Theorem "Descent Direction") with step halving and move to rank r + 1.

Readings for the escape (listed in the design notes): the printed line search
compares traces of mismatched sizes and appends alpha v^T without restoring
feasibility; here the cost tr(Q U^T U) is compared, each block of
[U; alpha v^T] is retracted back onto the manifold (Gram-Schmidt of
[R_k; alpha v_k^T / s_k], scale kept), ||v|| = 1, and at most 40 halvings.
"""
from __future__ import annotations

import numpy as np

from . import certificate as cert
from . import manifold as mf
from .rtr import rtr


def escape(Q, R, s, v, max_halvings=40, lam=0.0):
    """Rank r -> r+1 along D = [0; v^T].  Returns (R+, s+, alpha) or None."""
    N, r, _ = R.shape
    f0 = mf.cost(Q, R, s, lam)
    Rh = np.concatenate([R, np.zeros((N, 1, 3))], axis=1)
    vb = v.reshape(N, 3)
    alpha = 1.0
    for _ in range(max_halvings + 1):
        Rd = np.zeros_like(Rh)
        Rd[:, r, :] = alpha * vb / s[:, None]
        Rn, sn = mf.retract(Rh, s, Rd, np.zeros(N))
        sn = s.copy()
        if mf.cost(Q, Rn, sn, lam) < f0:
            return Rn, sn, alpha
        alpha *= 0.5
    return None


def staircase(Q, r0=3, r_max=5, grad_tol=1e-10, tau=1e-8, max_outer=500, R0=None, s0=None,
              history=None, lam=0.0):
    """Run the staircase (lam > 0: the scale-regularised objective of
    eq. problem-sdp-scale).  Returns (R, s, info) with info['certified'] etc."""
    N = Q.shape[0] // 3
    if R0 is None:
        R, s = mf.initial_point(N, r0)
    else:
        R, s = R0.copy(), s0.copy()
    r = R.shape[1]
    total_outer = total_inner = 0
    while True:
        R, s, info = rtr(Q, R, s, grad_tol=grad_tol, max_outer=max_outer, lam=lam)
        total_outer += info["outer"]
        total_inner += info["inner"]
        c = cert.certify(Q, R, s, tau, lam=lam)
        if history is not None:
            history.append({"r": r, "cost": info["cost"], "lambda_min": c["lambda_min"]})
        if c["certified"] or r >= r_max:
            break
        out = escape(Q, R, s, c["v"], lam=lam)
        if out is None:
            break
        R, s, _ = out
        r += 1
    info = {"r": r, "cost": mf.cost(Q, R, s, lam), "grad_norm": info["grad_norm"],
            "certified": c["certified"], "lambda_min": c["lambda_min"],
            "lambda_min_full": c["lambda_min_full"], "primal": c["primal"], "dual": c["dual"],
            "outer": total_outer, "inner": total_inner, "qbar": c["qbar"], "Lambda": c["Lambda"]}
    return R, s, info
