"""Riemannian trust region with truncated CG (test infrastructure: oracle only).

The paper's local optimizer (Algorithm "Riemannian Staircase", the local
optimisation step; Section "C++/CUDA-based Riemannian Optimization") is
RTR-tCG as described by Absil, Mahony & Sepulchre (2008) and Boumal (2023).
The paper gives no parameters; the textbook defaults are used (listed in the
design notes): kappa = 0.1, theta = 1 for the inner stop, rho' = 0.1 for
acceptance, radius x1/4 when rho < 1/4 and x2 (capped at Delta_bar) when
rho > 3/4 and tCG stopped on the boundary, Delta_bar = sqrt(3N),
Delta_0 = Delta_bar / 8, and the usual rho regularisation
max(1, |f|) * 1e3 * eps added to both numerator and denominator.

Stopping rule (also a reading): ||grad|| <= grad_tol * qbar * ||U||_F with
qbar = tr(Q) / 3N, or the iteration caps.
"""
from __future__ import annotations

import numpy as np

from . import manifold as mf


def tcg(Q, R, s, gR, gs, Delta, kappa=0.1, theta=1.0, max_inner=None, lam=0.0):
    """Steihaug-Toint truncated CG on the trust-region subproblem.

    Returns (eta, Heta, reason, n_inner).  Inner products are the manifold
    metric, computed afresh each time (no recurrences)."""
    N = R.shape[0]
    if max_inner is None:
        max_inner = 3 * N * R.shape[1]
    ip = lambda a, b: mf.inner(s, a[0], a[1], b[0], b[1])
    eta = (np.zeros_like(gR), np.zeros_like(gs))
    Heta = (np.zeros_like(gR), np.zeros_like(gs))
    res = (gR.copy(), gs.copy())
    r_r = ip(res, res)
    norm_r0 = np.sqrt(r_r)
    delta = (-res[0], -res[1])
    reason = "maxiter"
    j = 0
    for j in range(1, max_inner + 1):
        Hd = mf.hess(Q, R, s, delta[0], delta[1], lam)
        d_Hd = ip(delta, Hd)
        alpha = r_r / d_Hd if d_Hd != 0 else np.inf
        e_Pe = ip(eta, eta)
        e_Pd = ip(eta, delta)
        d_Pd = ip(delta, delta)
        e_Pe_new = e_Pe + 2 * alpha * e_Pd + alpha * alpha * d_Pd
        if d_Hd <= 0 or e_Pe_new >= Delta * Delta:
            tau = (-e_Pd + np.sqrt(e_Pd * e_Pd + d_Pd * (Delta * Delta - e_Pe))) / d_Pd
            eta = (eta[0] + tau * delta[0], eta[1] + tau * delta[1])
            Heta = (Heta[0] + tau * Hd[0], Heta[1] + tau * Hd[1])
            reason = "negative curvature" if d_Hd <= 0 else "boundary"
            break
        eta = (eta[0] + alpha * delta[0], eta[1] + alpha * delta[1])
        Heta = (Heta[0] + alpha * Hd[0], Heta[1] + alpha * Hd[1])
        res = (res[0] + alpha * Hd[0], res[1] + alpha * Hd[1])
        r_r_new = ip(res, res)
        if np.sqrt(r_r_new) <= norm_r0 * min(norm_r0 ** theta, kappa):
            reason = "converged"
            break
        beta = r_r_new / r_r
        r_r = r_r_new
        delta = (-res[0] + beta * delta[0], -res[1] + beta * delta[1])
    return eta, Heta, reason, j


def rtr(Q, R, s, grad_tol=1e-10, max_outer=500, max_inner=None, Delta_bar=None,
        Delta0=None, rho_prime=0.1, log=None, lam=0.0):
    """Minimise tr(Q U^T U) (+ the scale regulariser lam sum_{k>=1} (s_k^2 - 1)^2)
    from (R, s).  Returns (R, s, info)."""
    N = R.shape[0]
    qbar = float(np.trace(Q)) / (3 * N)
    if Delta_bar is None:
        Delta_bar = np.sqrt(3.0 * N)
    Delta = Delta_bar / 8.0 if Delta0 is None else Delta0
    f = mf.cost(Q, R, s, lam)
    gR, gs = mf.rgrad(Q, R, s, lam)
    gnorm = np.sqrt(mf.inner(s, gR, gs, gR, gs))
    total_inner = 0
    k = 0
    for k in range(max_outer):
        Unorm = np.linalg.norm(mf.to_U(R, s))
        if gnorm <= grad_tol * qbar * Unorm:
            break
        eta, Heta, reason, nin = tcg(Q, R, s, gR, gs, Delta, max_inner=max_inner, lam=lam)
        total_inner += nin
        Rn, sn = mf.retract(R, s, eta[0], eta[1])
        fn = mf.cost(Q, Rn, sn, lam)
        mdec = -(mf.inner(s, gR, gs, eta[0], eta[1]) + 0.5 * mf.inner(s, eta[0], eta[1], Heta[0], Heta[1]))
        reg = max(1.0, abs(f)) * np.finfo(float).eps * 1e3
        rho = (f - fn + reg) / (mdec + reg)
        # a trial point whose cost is not finite is a failed step: reject, shrink
        finite = bool(np.isfinite(rho))
        if not finite or rho < 0.25:
            Delta = Delta / 4.0
        elif rho > 0.75 and reason in ("boundary", "negative curvature"):
            Delta = min(2.0 * Delta, Delta_bar)
        if log is not None:
            log.append((k, f, gnorm, Delta, rho, reason, nin))
        if finite and mdec > 0 and rho > rho_prime:
            R, s, f = Rn, sn, fn
            gR, gs = mf.rgrad(Q, R, s, lam)
            gnorm = np.sqrt(mf.inner(s, gR, gs, gR, gs))
    info = {"cost": f, "grad_norm": gnorm, "outer": k, "inner": total_inner, "qbar": qbar}
    return R, s, info
