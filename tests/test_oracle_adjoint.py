"""Pins for the oracle's adjoint: central finite differences of re-solved optima and the
dense chart-coordinate reference (independent of the Riemannian Hessian formulas)."""
import numpy as np
import pytest

import scenes
from oracle import adjoint as oad
from oracle import data_matrix as dm
from oracle import manifold as mf
from oracle import rounding as rd
from oracle import staircase as st


def _solve(sc, u, w, R0=None, s0=None):
    Q = dm.q_block_elimination(sc.N, sc.M, sc.frame, sc.landmark, u, w)
    R, s, info = st.staircase(Q, grad_tol=1e-13, tau=1e-8, R0=R0, s0=s0)
    assert info["certified"]
    Rh, sh = rd.round_solution(mf.to_U(R, s))
    return Rh, sh, info["cost"], R, s


@pytest.fixture(scope="module")
def prob():
    sc = scenes.random_scene(8, 150, L=4, sigma=0.01, seed=31, weights=(0.5, 1.5))
    Rh, sh, f, R, s = _solve(sc, sc.u, sc.w)
    rng = np.random.default_rng(5)
    gR = rng.standard_normal((sc.N, 3, 3))
    gs = rng.standard_normal(sc.N)
    return sc, Rh, sh, f, R, s, gR, gs


def _loss(Rh, sh, gR, gs):
    return float(np.sum(gR * Rh) + np.sum(gs * sh))


def test_cost_gradient_matches_finite_differences(prob):
    sc, Rh, sh, f, R, s, gR, gs = prob
    gu, gw = oad.cost_grad(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w, oad.anchored_U(Rh, sh))
    rng = np.random.default_rng(1)
    h = 1e-4
    for _ in range(4):
        vu = rng.standard_normal(sc.u.shape)
        vw = rng.standard_normal(sc.w.shape) * 0.1
        fp = _solve(sc, sc.u + h * vu, sc.w + h * vw, R, s)[2]
        fm = _solve(sc, sc.u - h * vu, sc.w - h * vw, R, s)[2]
        fd = (fp - fm) / (2 * h)
        an = float(np.sum(gu * vu) + np.sum(gw * vw))
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an))


def test_weight_gradient_is_squared_residual(prob):
    sc, Rh, sh, f, R, s, gR, gs = prob
    Y = oad.anchored_U(Rh, sh)
    t, p = dm.recover_tp(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w, Y)
    e = oad.residuals(sc.frame, sc.landmark, sc.u, Y, t, p)
    _, gw = oad.cost_grad(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w, Y)
    assert np.allclose(gw, np.sum(e * e, axis=1), rtol=0, atol=1e-14)
    # and the cost itself is sum w ||e||^2
    assert abs(float(np.sum(sc.w * gw)) - f) <= 1e-9 * max(1.0, f)


def test_ift_matches_dense_chart_reference(prob):
    sc, Rh, sh, f, R, s, gR, gs = prob
    gu, gw = oad.ift_grad(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w, Rh, sh, gR, gs)
    rng = np.random.default_rng(2)
    for _ in range(3):
        vu = rng.standard_normal(sc.u.shape)
        vw = rng.standard_normal(sc.w.shape) * 0.1
        ref = oad.dense_reference(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w, Rh, sh, gR, gs, vu, vw)
        an = float(np.sum(gu * vu) + np.sum(gw * vw))
        assert abs(ref - an) <= 1e-6 * max(1.0, abs(ref))


def test_ift_matches_finite_differences(prob):
    sc, Rh, sh, f, R, s, gR, gs = prob
    gu, gw = oad.ift_grad(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w, Rh, sh, gR, gs)
    rng = np.random.default_rng(3)
    h = 1e-4
    for _ in range(4):
        vu = rng.standard_normal(sc.u.shape)
        vw = rng.standard_normal(sc.w.shape) * 0.1
        lp = _loss(*_solve(sc, sc.u + h * vu, sc.w + h * vw, R, s)[:2], gR, gs)
        lm = _loss(*_solve(sc, sc.u - h * vu, sc.w - h * vw, R, s)[:2], gR, gs)
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(gu * vu) + np.sum(gw * vw))
        assert abs(fd - an) <= 1e-4 * max(1.0, abs(an))


def test_chart_hessian_matches_second_differences(prob):
    # the exact polarised Hessian agrees with second differences of f in the chart
    sc, Rh, sh, f, R, s, gR, gs = prob
    Q = dm.q_block_elimination(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w)
    H = oad.chart_hessian(Q, Rh, sh)
    n = H.shape[0]
    rng = np.random.default_rng(4)
    d = rng.standard_normal(n)
    d /= np.linalg.norm(d)

    def f_of(x):
        Rx = Rh.copy(); sx = sh.copy()
        from scipy.linalg import expm
        for k in range(1, sc.N):
            Rx[k] = Rh[k] @ expm(oad._skew(x[4 * (k - 1):4 * (k - 1) + 3]))
            sx[k] = sh[k] * np.exp(x[4 * (k - 1) + 3])
        U = oad.anchored_U(Rx, sx)
        return float(np.sum(U * (U @ Q)))

    hstep = 1e-4
    second = (f_of(hstep * d) - 2 * f_of(0 * d) + f_of(-hstep * d)) / hstep ** 2
    assert abs(second - d @ H @ d) <= 1e-4 * max(1.0, abs(second))
