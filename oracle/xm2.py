"""XM^2: the greedy outlier loop (test infrastructure: oracle only).

Section "Structure from Motion with XM", solver paragraph: solve the SDP with
the XM solver; if needed, delete the 10% of the measurements with the largest
residuals and run the solver again (a greedy outlier-removal heuristic, run
twice).

Readings (listed in the design notes; the paper fixes none of them):
  * the residual of observation o = (i, k) is the SBA residual of eq. sba at
    the rounded, anchored optimum, e_o = s_i R_i u_o + t_i - p_k, with t and p
    the minimisers of eq. tpstar at that (R, s);
  * "largest residuals" ranks observations by a score: |e_o| (rank="world",
    the residual of eq. sba as written, weights not applied) or |e_o| / s_i
    (rank="frame", the same residual in the units of frame i's lifted
    keypoints).  Where the optimum shrinks the scales of frames 2..N (the
    collapse App. "Scale Regularization" describes) the anchored frame's
    world-frame residuals dominate, and deleting by |e_o| can strip the
    anchor of its observations; the frame-unit score is the default.  The
    number deleted is floor(frac * n_obs); ties drop the lower index first;
  * the deletion may leave a frame tied to the others by too few
    observations for its pose to be determined (its block of Q becomes
    near-singular and the second run stalls or cannot certify).  A guard
    undoes the deletion around such a frame: a kept observation is a link
    of its frame when its landmark keeps at least two observations; for a
    frame with fewer than min_links links, every observation of that frame
    and every observation of a landmark it sees is kept again (one pass;
    afterwards each frame has min_links links or all the links it can have,
    so a second pass changes nothing; min_links = 0 disables it).  Three
    points in general position fix a similarity; the default asks for twice
    that;
  * the second run is the same staircase on the kept observations (a frame
    or landmark may lose observations; the view graph must stay connected).

Functions
---------
residuals   e_o [n, 3] at (R_hat, s_hat), with t, p.
scores      the ranking score of every observation.
drop_mask   keep mask deleting the largest-score fraction.
guard_frames  restore the observations of frames left with too few links.
xm2         solve, residuals, delete, solve again (dense Q: small scenes).
"""
from __future__ import annotations

import numpy as np

from . import data_matrix as dm
from . import manifold as mf
from . import rounding as rd
from . import staircase as st


def residuals(N, M, frame, landmark, u, w, R_hat, s_hat):
    """e_o = s_i R_i u_o + t_i - p_k for every observation, (t, p) from eq. tpstar.
    Returns (e [n, 3], t [N, 3], p [M, 3])."""
    U = rd.rounded_U(R_hat, s_hat)
    t, p = dm.recover_tp(N, M, frame, landmark, u, w, U)
    Ub = U.reshape(3, N, 3).transpose(1, 0, 2)          # N x 3 x 3: s_i R_i
    e = np.einsum("nab,nb->na", Ub[frame], u) + t[frame] - p[landmark]
    return e, t, p


def drop_mask(score, frac):
    """Keep mask: False for the floor(frac n) observations with the largest
    score (ties: the lower index is dropped first)."""
    n = score.shape[0]
    k = int(np.floor(frac * n))
    keep = np.ones(n, bool)
    if k > 0:
        order = np.lexsort((np.arange(n), -score))      # score descending, then index ascending
        keep[order[:k]] = False
    return keep


def guard_frames(N, M, frame, landmark, keep, min_links):
    """The frame guard of the deletion: a kept observation of landmark k is a
    link when k keeps >= 2 observations; a frame with fewer than min_links
    links is starved; an observation is kept again when its frame is starved
    or its landmark is seen by a starved frame.  Returns (keep', number
    restored)."""
    keep = np.asarray(keep, bool)
    kept_per_landmark = np.bincount(landmark[keep], minlength=M)
    link = keep & (kept_per_landmark[landmark] >= 2)
    links_per_frame = np.bincount(frame[link], minlength=N)
    starved = links_per_frame < min_links
    rescued = np.zeros(M, bool)
    rescued[landmark[starved[frame]]] = True
    out = keep | starved[frame] | rescued[landmark]
    return out, int(np.count_nonzero(out & ~keep))


def scores(e, s_hat, frame, rank="frame"):
    """|e_o| ("world") or |e_o| / s_i ("frame")."""
    nrm = np.linalg.norm(e, axis=1)
    return nrm if rank == "world" else nrm / s_hat[frame]


def xm2(N, M, frame, landmark, u, w, frac=0.1, rank="frame", grad_tol=1e-11, tau=1e-7, r_max=5,
        min_links=6):
    """Staircase on all observations, rounding, residuals, deletion of the
    largest fraction, staircase on the rest, rounding.  Dense Q."""
    Q1 = dm.q_block_elimination(N, M, frame, landmark, u, w)
    R1, s1, info1 = st.staircase(Q1, grad_tol=grad_tol, tau=tau, r_max=r_max)
    Rh1, sh1 = rd.round_solution(mf.to_U(R1, s1))
    e, _, _ = residuals(N, M, frame, landmark, u, w, Rh1, sh1)
    keep = drop_mask(scores(e, sh1, frame, rank), frac)
    keep, _ = guard_frames(N, M, frame, landmark, keep, min_links)
    Q2 = dm.q_block_elimination(N, M, frame[keep], landmark[keep], u[keep], w[keep])
    R2, s2, info2 = st.staircase(Q2, grad_tol=grad_tol, tau=tau, r_max=r_max)
    Rh2, sh2 = rd.round_solution(mf.to_U(R2, s2))
    return {"first": (Rh1, sh1, info1), "residuals": e, "keep": keep, "second": (Rh2, sh2, info2),
            "Q2": Q2}
