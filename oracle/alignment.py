"""Similarity alignment of an estimate to a reference (test infrastructure:
oracle only; the library never imports it).

App. "Metrics" measures trajectory errors after aligning the estimated camera
positions to the ground truth by a point-cloud registration (rotation of each
frame ignored).  The paper uses a robust registration; on the synthetic scenes
the correspondence is known and exact, and the registration here is its
least-squares special case: the similarity (s, R, t), s > 0, R in SO(3),
minimising

    sum_i w_i | s R p_i + t - q_i |^2 .

Closed form (Umeyama's solution of this problem, written from its
derivation): with the weighted means mu_p, mu_q, the weighted cross-covariance
C = sum_i w_i (q_i - mu_q)(p_i - mu_p)^T / W and sigma^2 = sum_i w_i
|p_i - mu_p|^2 / W, the rotation maximises tr(R^T C) over SO(3) (the closest
rotation to C: with C = U D V^T, R = U diag(1, 1, det(U V^T)) V^T), then
s = tr(R^T C) / sigma^2 and t = mu_q - s R mu_p.

Functions
---------
align_similarity   (s, R, t) and the weighted RMS residual after alignment.
"""
from __future__ import annotations

import numpy as np


def align_similarity(P, Q, w=None):
    """P, Q: [n, 3]; w: [n] non-negative weights or None.  Returns
    (s, R, t, rmse) with rmse = sqrt(sum w |s R p + t - q|^2 / sum w)."""
    P = np.asarray(P, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    n = P.shape[0]
    w = np.ones(n) if w is None else np.asarray(w, dtype=np.float64)
    W = w.sum()
    if not W > 0:
        raise ValueError("the weights must have a positive sum")
    mu_p = (w[:, None] * P).sum(axis=0) / W
    mu_q = (w[:, None] * Q).sum(axis=0) / W
    Pc, Qc = P - mu_p, Q - mu_q
    sigma2 = (w * (Pc * Pc).sum(axis=1)).sum() / W
    if not sigma2 > 0:
        raise ValueError("the points to align have no spread")
    C = (w[:, None, None] * Qc[:, :, None] * Pc[:, None, :]).sum(axis=0) / W
    U, D, Vt = np.linalg.svd(C)
    S = np.diag([1.0, 1.0, np.sign(np.linalg.det(U @ Vt)) or 1.0])
    R = U @ S @ Vt
    s = np.trace(R.T @ C) / sigma2
    t = mu_q - s * R @ mu_p
    res = s * P @ R.T + t - Q
    rmse = np.sqrt((w * (res * res).sum(axis=1)).sum() / W)
    return s, R, t, rmse
