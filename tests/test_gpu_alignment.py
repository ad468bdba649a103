"""xm_align_similarity against the oracle (App. "Metrics": camera positions
registered by a similarity before trajectory errors): random, weighted,
exact, mirrored and collinear point sets, the error cases, and the anchored
gauge of a solved scene registered to its ground-truth camera centres."""
import numpy as np
import pytest

import scenes
from oracle import alignment as oal

from conftest import progress

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _xm():
    import paper_2502_04640_amd as xm
    xm.load_library()
    return xm


def _say(msg):
    print(msg, flush=True)
    progress(msg)


def _rot(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    return q if np.linalg.det(q) > 0 else -q


def _gpu(xm, P, Q, w=None):
    d = xm.align_similarity(torch.from_numpy(P).cuda(), torch.from_numpy(Q).cuda(),
                            None if w is None else torch.from_numpy(w).cuda())
    return d["s"], d["R"].numpy(), d["t"].numpy(), d["rmse"]


@pytest.mark.parametrize("n", [3, 5, 1000, 100000])
@pytest.mark.parametrize("weighted", [False, True])
def test_alignment_matches_oracle(n, weighted):
    _say(f"case: similarity alignment vs oracle, n={n}, weighted={weighted}")
    xm = _xm()
    rng = np.random.default_rng(n + weighted)
    P = rng.normal(size=(n, 3)) * np.array([4.0, 2.0, 1.0])
    Q = 1.7 * P @ _rot(rng).T + np.array([3.0, -1.0, 2.0]) + 0.3 * rng.normal(size=(n, 3))
    w = rng.uniform(0.1, 2.0, size=n) if weighted else None
    s, R, t, rmse = _gpu(xm, P, Q, w)
    so, Ro, to, rmseo = oal.align_similarity(P, Q, w)
    assert abs(s - so) <= 1e-11 * so
    assert np.abs(R - Ro).max() <= 1e-11
    assert np.abs(t - to).max() <= 1e-10 * (1 + np.abs(to).max())
    assert abs(rmse - rmseo) <= 1e-11 * rmseo
    assert abs(np.linalg.det(R) - 1.0) <= 1e-12


def test_exact_and_mirrored_sets():
    _say("case: similarity alignment, exact similarity and mirrored set")
    xm = _xm()
    rng = np.random.default_rng(7)
    P = rng.normal(size=(50, 3)) * 2.0
    R0 = _rot(rng)
    Q = 0.35 * P @ R0.T + np.array([10.0, 0.0, -5.0])
    s, R, t, rmse = _gpu(xm, P, Q)
    assert abs(s - 0.35) <= 1e-12 and np.abs(R - R0).max() <= 1e-12
    assert np.abs(t - np.array([10.0, 0.0, -5.0])).max() <= 1e-11 and rmse <= 1e-11
    # mirrored: the closest proper rotation, as the oracle's
    Qm = P * np.array([1.0, 1.0, -1.0]) * np.array([3.0, 2.0, 1.0])
    s, R, t, rmse = _gpu(xm, P, Qm)
    so, Ro, to, rmseo = oal.align_similarity(P, Qm)
    assert abs(np.linalg.det(R) - 1.0) <= 1e-12
    assert abs(s - so) <= 1e-11 * so and abs(rmse - rmseo) <= 1e-11 * rmseo
    assert np.abs(R - Ro).max() <= 1e-10


def test_collinear_points_give_the_unique_aligned_positions():
    # the rotation about the line is free: only the aligned points and the
    # residual are unique
    _say("case: similarity alignment, collinear points")
    xm = _xm()
    rng = np.random.default_rng(8)
    d = np.array([1.0, 2.0, -0.5])
    P = rng.normal(size=(20, 1)) * d
    Q = rng.normal(size=(20, 3))
    s, R, t, rmse = _gpu(xm, P, Q)
    so, Ro, to, rmseo = oal.align_similarity(P, Q)
    A, Ao = s * P @ R.T + t, so * P @ Ro.T + to
    assert np.abs(A - Ao).max() <= 1e-10 * (1 + np.abs(Ao).max())
    assert abs(rmse - rmseo) <= 1e-11 * rmseo
    assert np.abs(R @ R.T - np.eye(3)).max() <= 1e-12 and abs(np.linalg.det(R) - 1.0) <= 1e-12


def test_error_cases():
    _say("case: similarity alignment errors")
    xm = _xm()
    P = np.zeros((4, 3))
    P[:, 0] = np.arange(4.0)
    Q = P.copy()
    with pytest.raises(xm.XMError, match="XM_EINVAL"):
        _gpu(xm, P[:1], Q[:1])                      # one point: no spread
    with pytest.raises(xm.XMError, match="XM_EINVAL"):
        _gpu(xm, P, Q, np.array([1.0, -1.0, 1.0, 1.0]))
    with pytest.raises(xm.XMError, match="XM_EINVAL"):
        _gpu(xm, P, Q, np.zeros(4))
    Pn = P.copy()
    Pn[2, 1] = np.nan
    with pytest.raises(xm.XMError, match="XM_EINVAL"):
        _gpu(xm, Pn, Q)


def test_anchored_gauge_registers_to_ground_truth_centres():
    # noise-free scene: the recovered camera positions t_i (anchored gauge)
    # are the ground-truth centres up to the similarity of frame 0's pose and
    # depth scale, which the alignment returns with zero residual
    _say("case: anchored gauge registered to the ground-truth camera centres")
    xm = _xm()
    sc = scenes.random_scene(30, 1200, L=4, sigma=0.0, seed=12)
    dev = [torch.from_numpy(a).cuda() for a in (sc.frame, sc.landmark, sc.u, sc.w)]
    P = xm.build_Q(sc.N, sc.M, *dev, keep=())
    Y, info = P.solve(xm.SolveOptions(compute="f64"))
    R, s, _ = P.round(Y)
    t, _ = P.recover_tp(R, s)
    c = np.asarray(sc.gt["c"], dtype=np.float64)
    sa, Ra, ta, rmse = _gpu(xm, t.cpu().numpy(), c)
    so, Ro, to, rmseo = oal.align_similarity(t.cpu().numpy(), c)
    assert rmse <= 1e-7 * np.abs(c).max() and abs(sa - so) <= 1e-10 * so
    assert abs(sa - 1.0 / sc.gt["d"][0]) <= 1e-7 / sc.gt["d"][0]
    assert np.abs(Ra - sc.gt["R_cfg"][0].T).max() <= 1e-7
