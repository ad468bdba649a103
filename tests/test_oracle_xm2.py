"""Pins for the oracle's XM^2 loop (Section "Structure from Motion with XM"):
residuals against the SBA cost and ground truth, the deletion against its
definition, and the loop on a seeded scene with injected outliers."""
import numpy as np
import pytest

import scenes
from oracle import data_matrix as dm
from oracle import manifold as mf
from oracle import rounding as rd
from oracle import staircase as st
from oracle import xm2


def test_residuals_vanish_at_noise_free_ground_truth():
    sc = scenes.make_scene("tiny", 3, sigma=0.0)
    e, t, p = xm2.residuals(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w, sc.gt["R"], sc.gt["s"])
    assert np.abs(e).max() <= 1e-10 * np.abs(sc.u).max()
    assert np.abs(t - sc.gt["t"]).max() <= 1e-9 * np.abs(sc.gt["t"]).max()


def test_weighted_squared_residuals_sum_to_least_squares_cost():
    # sum_o w_o |e_o|^2 at (R, s) is the SBA cost minimised over t, p (eq. sba),
    # here by numpy lstsq over the observations, independent of Q
    sc = scenes.random_scene(6, 40, L=3, sigma=0.1, seed=31, weights=(0.5, 1.5))
    rng = np.random.default_rng(2)
    R = mf.gram_schmidt(rng.standard_normal((sc.N, 3, 3)))
    R[0] = np.eye(3)
    s = np.exp(0.3 * rng.standard_normal(sc.N))
    s[0] = 1.0
    R = np.where(np.linalg.det(R)[:, None, None] < 0, R * np.array([1, 1, -1.0]), R)
    e, _, _ = xm2.residuals(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w, R, s)
    bf = dm.brute_force_cost(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w, rd.rounded_U(R, s))
    assert abs(float(np.sum(sc.w * np.sum(e * e, axis=1))) - bf) <= 1e-10 * bf


def test_drop_mask_definition():
    rng = np.random.default_rng(0)
    score = rng.random(1000)
    score[[10, 20, 30]] = 5.0           # a tie at the top
    keep = xm2.drop_mask(score, 0.002)  # floor(2.0) = 2 dropped: the lower indices of the tie
    assert (~keep).sum() == 2 and not keep[10] and not keep[20] and keep[30]
    keep = xm2.drop_mask(score, 0.1)
    assert (~keep).sum() == 100
    assert score[~keep].min() >= score[keep].max()
    assert xm2.drop_mask(score, 0.0).all()


@pytest.mark.parametrize("rank", ["frame", "world"])
def test_xm2_removes_injected_outliers(rank):
    # noise-free scene, 1% of observations moved up to 3 units off their
    # landmark: the deletion must catch almost all of them and the second
    # solve must be far closer to the ground truth than the first
    sc = scenes.random_scene(50, 2000, L=4, sigma=0.0, seed=10, outlier=0.01, outlier_local=3.0)
    out = xm2.xm2(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w, frac=0.1, rank=rank)
    bad, keep = sc.gt["outlier"], out["keep"]
    assert (~keep).sum() == int(0.1 * sc.n_obs)
    assert (bad & keep).sum() <= 0.02 * bad.sum()
    err = [np.linalg.norm(out[k][0] - sc.gt["R"], axis=(1, 2)).max() for k in ("first", "second")]
    assert out["first"][2]["certified"] and out["second"][2]["certified"]
    assert err[1] <= 0.05 * err[0]
    # the second solve is the staircase on the kept observations
    Q2 = dm.q_block_elimination(sc.N, sc.M, sc.frame[keep], sc.landmark[keep], sc.u[keep], sc.w[keep])
    assert np.abs(Q2 - out["Q2"]).max() <= 1e-12 * np.abs(Q2).max()


def _guard_case():
    # four frames, five landmarks; observations (frame, landmark) with the two
    # partners of frame 3's landmarks deleted: frame 3 keeps both of its own
    # observations but none of them is a link any more
    obs = [(0, 0), (1, 0), (0, 1), (2, 1), (1, 2), (2, 2), (3, 3), (3, 4), (0, 3), (2, 4)]
    frame = np.array([f for f, _ in obs], np.int32)
    landmark = np.array([k for _, k in obs], np.int32)
    keep = np.ones(len(obs), bool)
    keep[[8, 9]] = False
    return frame, landmark, keep


def test_guard_frames_worked_example():
    frame, landmark, keep = _guard_case()
    # links: frames 0, 1, 2 have two each, frame 3 none
    out, n = xm2.guard_frames(4, 5, frame, landmark, keep, 1)
    assert n == 2 and out.all()             # (0, 3) and (2, 4) come back: landmarks of frame 3
    out, n = xm2.guard_frames(4, 5, frame, landmark, keep, 0)
    assert n == 0 and (out == keep).all()   # disabled
    # min_links 3: every frame is starved, so every landmark is rescued
    out, n = xm2.guard_frames(4, 5, frame, landmark, keep, 3)
    assert n == 2 and out.all()
    # frame 1 loses (1, 2): landmark 2 keeps one observation, so frames 1 and 2
    # drop to one link; with min_links 2 they are starved with frame 3
    keep2 = keep.copy()
    keep2[4] = False
    out, n = xm2.guard_frames(4, 5, frame, landmark, keep2, 2)
    assert n == 3 and out.all()
    # only frame 3 starved (min_links 1): its landmarks 3, 4 come back, the
    # deleted (1, 2) stays deleted
    out, n = xm2.guard_frames(4, 5, frame, landmark, keep2, 1)
    assert n == 2 and not out[4] and out[[0, 1, 2, 3, 5, 6, 7, 8, 9]].all()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_guard_frames_invariants(seed):
    # random deletions on a random scene: afterwards every frame has at least
    # min_links links or keeps every observation of it and of its landmarks;
    # nothing kept is deleted; a second pass changes nothing
    rng = np.random.default_rng(seed)
    N, M, n = 40, 300, 1500
    frame = rng.integers(0, N, n).astype(np.int32)
    landmark = rng.integers(0, M, n).astype(np.int32)
    keep = rng.random(n) > 0.5
    for mlinks in (1, 4, 8):
        out, nr = xm2.guard_frames(N, M, frame, landmark, keep, mlinks)
        assert nr == int((out & ~keep).sum()) and not (keep & ~out).any()
        again, nr2 = xm2.guard_frames(N, M, frame, landmark, out, mlinks)
        assert nr2 == 0 and (again == out).all()
        for i in range(N):
            mine = frame == i
            links = sum(1 for o in np.flatnonzero(mine & out)
                        if np.count_nonzero(out & (landmark == landmark[o])) >= 2)
            if links < mlinks:
                seen = np.isin(landmark, landmark[mine])
                assert out[mine].all() and out[seen].all()
