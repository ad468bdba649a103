"""Pins for the oracle's scale-regularised objective (App. "Scale
Regularization", eq. problem-sdp-scale): lam sum_{i>=2} (X_{3i,3i} - 1)^2 added
to tr(QX), its modified dual matrix and dual value."""
import numpy as np
import pytest

import scenes
from oracle import certificate as ce
from oracle import data_matrix as dm
from oracle import manifold as mf
from oracle import rounding as rd
from oracle import staircase as st

LAM = 3.0


def _Q(sc):
    return dm.q_block_elimination(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w)


def _rand_point(rng, N, r):
    R = mf.gram_schmidt(rng.standard_normal((N, r, 3)))
    s = np.exp(0.3 * rng.standard_normal(N))
    s[0] = 1.0
    return R, s


def _rand_tangent(rng, R, s):
    Rd = mf.proj(R, rng.standard_normal(R.shape))
    sd = rng.standard_normal(s.shape) * s
    sd[0] = 0.0
    return Rd, sd


@pytest.fixture(scope="module")
def small():
    sc = scenes.random_scene(8, 120, L=3, sigma=0.05, seed=21, weights=(0.5, 1.5))
    return sc, _Q(sc)


def test_regulariser_is_x_diagonal_term():
    # F evaluated on X = U^T U by its definition equals the scale form
    rng = np.random.default_rng(1)
    R, s = _rand_point(rng, 6, 4)
    U = mf.to_U(R, s)
    X = U.T @ U
    F = LAM * sum((X[3 * i + 2, 3 * i + 2] - 1.0) ** 2 for i in range(1, 6))
    assert abs(F - mf.scale_reg(s, LAM)) <= 1e-12 * F


@pytest.mark.parametrize("r", [3, 5])
def test_gradient_matches_finite_difference(small, r):
    sc, Q = small
    rng = np.random.default_rng(r)
    R, s = _rand_point(rng, sc.N, r)
    Rd, sd = _rand_tangent(rng, R, s)
    gR, gs = mf.rgrad(Q, R, s, LAM)
    h = 1e-6
    fp = mf.cost(Q, *mf.retract(R, s, h * Rd, h * sd), LAM)
    fm = mf.cost(Q, *mf.retract(R, s, -h * Rd, -h * sd), LAM)
    fd = (fp - fm) / (2 * h)
    assert abs(fd - mf.inner(s, gR, gs, Rd, sd)) <= 1e-6 * max(1.0, abs(fd))


def test_hessian_is_projected_derivative_of_gradient(small):
    sc, Q = small
    rng = np.random.default_rng(13)
    R, s = _rand_point(rng, sc.N, 4)
    Rd, sd = _rand_tangent(rng, R, s)
    h = 1e-5

    def grad_log(Rx, sig):
        gR, gs = mf.rgrad(Q, Rx, np.exp(sig), LAM)
        return gR, gs / np.exp(sig)

    sig, sig_d = np.log(s), sd / s
    gp = grad_log(R + h * Rd, sig + h * sig_d)
    gm = grad_log(R - h * Rd, sig - h * sig_d)
    dR = mf.proj(R, (gp[0] - gm[0]) / (2 * h))
    dsig = (gp[1] - gm[1]) / (2 * h)
    HR, Hs = mf.hess(Q, R, s, Rd, sd, LAM)
    scale = np.abs(HR).max()
    assert np.abs(HR - dR).max() <= 1e-6 * scale
    assert np.abs(Hs / s - dsig)[1:].max() <= 1e-6 * scale


def test_two_frames_closed_form_with_regulariser():
    # N = 2, every landmark in both frames: with t and p eliminated the cost is
    # A - 2 s tr(R^T C) + B s^2 (centred, c-weighted, as in the plain two-frame
    # pin), so R is the weighted Procrustes rotation for any s > 0 and s
    # minimises A - 2 m s + B s^2 + lam (s^2 - 1)^2, m = tr(R^T C): the positive
    # root of 4 lam s^3 + (2 B - 4 lam) s - 2 m = 0
    sc = scenes.random_scene(2, 60, L=2, sigma=0.05, seed=8, weights=(0.5, 1.5))
    Q = _Q(sc)
    lam = 50.0
    R, s, info = st.staircase(Q, grad_tol=1e-12, lam=lam)
    assert info["certified"]
    Rh, sh = rd.round_solution(mf.to_U(R, s))
    M = sc.M
    a = np.zeros((M, 3)); b = np.zeros((M, 3)); wa = np.zeros(M); wb = np.zeros(M)
    for o in range(sc.n_obs):
        if sc.frame[o] == 0:
            a[sc.landmark[o]] = sc.u[o]; wa[sc.landmark[o]] = sc.w[o]
        else:
            b[sc.landmark[o]] = sc.u[o]; wb[sc.landmark[o]] = sc.w[o]
    c = wa * wb / (wa + wb)
    ac = a - (c[:, None] * a).sum(0) / c.sum()
    bc = b - (c[:, None] * b).sum(0) / c.sum()
    Cm = (c[:, None, None] * ac[:, :, None] * bc[:, None, :]).sum(0)
    B = float((c * (bc ** 2).sum(1)).sum())
    Us, D, Vt = np.linalg.svd(Cm)
    S = np.diag([1, 1, np.sign(np.linalg.det(Us) * np.linalg.det(Vt))])
    Rot = Us @ S @ Vt
    m = float(np.trace(Rot.T @ Cm))
    roots = np.roots([4 * lam, 0.0, 2 * B - 4 * lam, -2 * m])
    pos = [x.real for x in roots if abs(x.imag) < 1e-12 and x.real > 0]
    g = lambda x: -2 * m * x + B * x * x + lam * (x * x - 1) ** 2
    s_cf = min(pos, key=g)
    assert np.abs(Rh[1] - Rot).max() <= 1e-9
    assert abs(sh[1] - s_cf) <= 1e-9 * s_cf
    # the plain problem's scale differs: the regulariser pulls it toward 1
    assert abs(s_cf - m / B) > 1e-3 and abs(s_cf - 1) < abs(m / B - 1)


def test_certificate_primal_dual_and_weak_duality():
    # at the certified regularised optimum: Z U^T = 0, primal = dual, and every
    # feasible X has tr(QX) + F(X) >= max(0, lambda_min) tr(X) + rho_dual
    # (the theorem of App. "Suboptimality for SDP")
    sc = scenes.make_scene("tiny", 1)
    Q = _Q(sc)
    lam = 0.5 * float(np.trace(Q)) / (3 * sc.N)
    R, s, info = st.staircase(Q, grad_tol=1e-11, lam=lam)
    assert info["certified"]
    U = mf.to_U(R, s)
    c = ce.certify(Q, R, s, 1e-7, lam=lam)
    Z = ce.dual_matrix(Q + np.diag(ce.reg_gradient(s, lam)), c["Lambda"])
    assert np.abs(Z @ U.T).max() <= 1e-7 * info["qbar"]
    assert abs(c["primal"] - c["dual"]) <= 1e-7 * max(1.0, abs(c["primal"]))
    assert abs(c["primal"] - info["cost"]) <= 1e-10 * info["cost"]
    rng = np.random.default_rng(5)
    for r in (3, 5, 8):
        for _ in range(5):
            R0, s0 = _rand_point(rng, sc.N, r)
            assert mf.cost(Q, R0, s0, lam) >= c["dual"] - 1e-9 * abs(c["dual"])
    # the scales move toward 1 as lam grows
    R2, s2, _ = st.staircase(Q, grad_tol=1e-11, lam=100 * lam)
    assert np.abs(s2 - 1).max() < np.abs(s - 1).max()
    # eq. suboptimality_new at the rounded point (tight scene: ~0)
    Rh, sh = rd.round_solution(U)
    rho_hat = mf.cost(Q, Rh, sh, lam)
    eta = ce.suboptimality_dual(rho_hat, c["dual"], c["lambda_min_full"], float(np.sum(U * U)))
    assert abs(eta) <= 1e-7
