"""Pins for the oracle's similarity alignment (App. "Metrics": positions
registered before trajectory errors): exact recovery, optimality against a
generic minimiser over (log s, rotation vector, t), the reflection case, and
weights."""
import numpy as np
from scipy.optimize import minimize
from scipy.spatial.transform import Rotation

from oracle import alignment as al


def _cost(P, Q, w, s, R, t):
    r = s * P @ R.T + t - Q
    return float((w * (r * r).sum(axis=1)).sum())


def _brute(P, Q, w, starts=20, seed=0):
    # generic minimisation over (log s, rotation vector, t) from many starts
    rng = np.random.default_rng(seed)

    def f(x):
        return _cost(P, Q, w, np.exp(x[0]), Rotation.from_rotvec(x[1:4]).as_matrix(), x[4:7])
    best = np.inf
    for _ in range(starts):
        x0 = np.concatenate([[rng.normal()], rng.normal(size=3) * 2.0, rng.normal(size=3)])
        r = minimize(f, x0, method="BFGS", options={"gtol": 1e-12, "maxiter": 2000})
        best = min(best, r.fun)
    return best


def test_exact_similarity_is_recovered():
    rng = np.random.default_rng(1)
    P = rng.normal(size=(40, 3)) * 3.0
    R0 = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    s0, t0 = 2.7, np.array([1.0, -4.0, 0.5])
    Q = s0 * P @ R0.T + t0
    s, R, t, rmse = al.align_similarity(P, Q)
    assert abs(s - s0) <= 1e-12 * s0
    assert np.abs(R - R0).max() <= 1e-12
    assert np.abs(t - t0).max() <= 1e-11
    assert rmse <= 1e-11
    assert abs(np.linalg.det(R) - 1.0) <= 1e-12


def test_noisy_weighted_alignment_is_the_global_minimum():
    rng = np.random.default_rng(2)
    P = rng.normal(size=(8, 3))
    Q = 0.6 * P @ Rotation.from_rotvec([0.3, -1.2, 2.0]).as_matrix().T + 0.4 * rng.normal(size=(8, 3))
    w = rng.uniform(0.2, 2.0, size=8)
    s, R, t, rmse = al.align_similarity(P, Q, w)
    c = _cost(P, Q, w, s, R, t)
    assert c <= _brute(P, Q, w) + 1e-10
    assert abs(rmse - np.sqrt(c / w.sum())) <= 1e-12


def test_reflected_data_gives_a_proper_rotation():
    # Q is a mirror image of P: the best proper rotation is not the
    # reflection, and the closed form must still reach the global minimum
    rng = np.random.default_rng(3)
    P = rng.normal(size=(10, 3)) * np.array([3.0, 2.0, 1.0])
    Q = P * np.array([1.0, 1.0, -1.0])
    w = np.ones(10)
    s, R, t, rmse = al.align_similarity(P, Q, w)
    assert abs(np.linalg.det(R) - 1.0) <= 1e-12
    assert np.abs(R @ R.T - np.eye(3)).max() <= 1e-12
    assert _cost(P, Q, w, s, R, t) <= _brute(P, Q, w) + 1e-10


def test_zero_weights_ignore_points():
    rng = np.random.default_rng(4)
    P = rng.normal(size=(12, 3))
    Q = 1.3 * P + 0.05 * rng.normal(size=(12, 3))
    w = np.ones(12)
    w[[2, 7]] = 0.0
    Q2 = Q.copy()
    Q2[[2, 7]] += 100.0
    a = al.align_similarity(P, Q, w)
    b = al.align_similarity(P, Q2, w)
    c = al.align_similarity(np.delete(P, [2, 7], 0), np.delete(Q, [2, 7], 0))
    for x, y in ((a, b), (a, c)):
        assert abs(x[0] - y[0]) <= 1e-12 and np.abs(x[1] - y[1]).max() <= 1e-12
        assert np.abs(x[2] - y[2]).max() <= 1e-12 and abs(x[3] - y[3]) <= 1e-12
