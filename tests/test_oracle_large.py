"""Pins for the oracle's matrix-free forms (Q as an operator, the SBA cost at a
fixed factor, the eigsh certificate, the Gram rounding branch): the forms that
reach scenes whose dense Q does not fit, pinned at small sizes against the
dense constructions and against least squares."""
import numpy as np
import pytest

import scenes
from oracle import certificate as ce
from oracle import data_matrix as dm
from oracle import manifold as mf
from oracle import rounding as rd
from oracle import staircase as st


def _args(sc):
    return sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w


@pytest.fixture(scope="module")
def tiny():
    sc = scenes.make_scene("tiny", 1)
    Q = dm.q_block_elimination(*_args(sc))
    op = dm.QOperator(*_args(sc))
    R, s, _ = st.staircase(Q, grad_tol=1e-11)
    return sc, Q, op, R, s


def test_operator_products_diagonal_and_trace(tiny):
    sc, Q, op, _, _ = tiny
    rng = np.random.default_rng(0)
    for k in (1, 5):
        V = rng.standard_normal((3 * sc.N, k))
        assert np.abs(op.matmat(V) - Q @ V).max() <= 1e-12 * np.abs(Q @ V).max()
    D = op.diag_blocks()
    for k in range(sc.N):
        assert np.abs(D[k] - Q[3 * k:3 * k + 3, 3 * k:3 * k + 3]).max() <= 1e-12 * np.abs(Q).max()
    assert abs(op.trace() - np.trace(Q)) <= 1e-12 * np.trace(Q)


@pytest.mark.parametrize("r", [3, 5])
def test_operator_cost_and_sba_cost_at_equal_least_squares(r):
    # tr(Q U^T U) (operator) and the SBA cost at the minimiser of eq. tpstar
    # (per-observation residuals) both equal min over t, p by numpy lstsq
    sc = scenes.random_scene(6, 40, L=3, sigma=0.1, seed=20 + r, weights=(0.5, 1.5))
    op = dm.QOperator(*_args(sc))
    rng = np.random.default_rng(r)
    for _ in range(3):
        U = rng.standard_normal((r, 3 * sc.N))
        bf = dm.brute_force_cost(*_args(sc), U)
        assert abs(op.cost(U) - bf) <= 1e-10 * max(1.0, bf)
        assert abs(dm.sba_cost_at(op, sc.frame, sc.landmark, sc.u, sc.w, U) - bf) <= 1e-10 * max(1.0, bf)


def test_sba_cost_at_noise_free_ground_truth_is_zero():
    sc = scenes.make_scene("tiny", 3, sigma=0.0)
    op = dm.QOperator(*_args(sc))
    gt = sc.gt
    U = (gt["s"][:, None, None] * gt["R"]).transpose(1, 0, 2).reshape(3, 3 * sc.N)
    t, p = dm.recover_tp_sparse(op, sc.frame, sc.landmark, sc.u, sc.w, U)
    assert np.abs(t - gt["t"]).max() <= 1e-9 * np.abs(gt["t"]).max()
    assert dm.sba_cost_at(op, sc.frame, sc.landmark, sc.u, sc.w, U) <= 1e-18 * np.trace(op.diag_blocks().sum(0))


def _compare(c, co, qbar):
    assert abs(c["primal"] - co["primal"]) <= 1e-10 * (1 + abs(c["primal"]))
    assert abs(c["dual"] - co["dual"]) <= 1e-10 * (1 + abs(c["dual"]))
    assert abs(c["stat_res"] - co["stat_res"]) <= 1e-9 * (qbar + c["stat_res"])
    assert abs(c["defl_min"] - co["defl_min"]) <= 1e-9
    assert abs(c["defl_cross"] - co["defl_cross"]) <= 1e-9 * (1 + c["defl_cross"])
    assert abs(c["lambda_min_scaled"] - co["lambda_min_scaled"]) <= 1e-8
    assert abs(c["lambda_bound_full"] - co["lambda_bound_full"]) <= 1e-8 * c["dmax"]
    assert abs(c["lambda_min"] - co["lambda_min_plain"]) <= 1e-8 * qbar
    assert co["certified"] == bool(c["lambda_bound_full"] >= -1e-7 * qbar)


def test_eigsh_certificate_matches_dense_at_optimum_and_perturbed_point(tiny):
    sc, Q, op, R, s = tiny
    c = ce.certify(Q, R, s, 1e-7)
    co = ce.certify_op(op, mf.to_U(R, s), 1e-7, plain=True)
    _compare(c, co, c["qbar"])
    assert co["certified"]
    rng = np.random.default_rng(3)
    R2 = mf.gram_schmidt(R + 0.05 * rng.standard_normal(R.shape))
    s2 = s * np.exp(0.05 * rng.standard_normal(s.shape))
    s2[0] = 1.0
    c = ce.certify(Q, R2, s2, 1e-7)
    co = ce.certify_op(op, mf.to_U(R2, s2), 1e-7, plain=True)
    _compare(c, co, c["qbar"])
    assert not co["certified"]


def test_eigsh_certificate_at_a_spurious_minimum():
    # the seeded rank-3 local minimum of the escape pin: the smallest
    # eigenvalue is negative and matches the dense one
    from oracle import rtr
    sc = scenes.random_scene(8, 40, L=3, sigma=0.5, seed=0)
    Q = dm.q_block_elimination(*_args(sc))
    op = dm.QOperator(*_args(sc))
    rng = np.random.default_rng(0)
    R0 = mf.gram_schmidt(rng.standard_normal((sc.N, 3, 3)))
    s0 = np.exp(rng.standard_normal(sc.N) * 0.3)
    s0[0] = 1.0
    R, s, _ = rtr.rtr(Q, R0, s0, grad_tol=1e-11)
    c = ce.certify(Q, R, s, 1e-8)
    co = ce.certify_op(op, mf.to_U(R, s), 1e-8, plain=True)
    assert c["lambda_min"] < -1e-3 * c["qbar"]
    _compare(c, co, c["qbar"])
    assert not co["certified"]


def test_top3_gram_branch_equals_dense_branch():
    # the r x r Gram U U^T has the nonzero spectrum of X = U^T U: the two
    # branches give the same rank-3 factor up to the sign of each row, hence
    # the same best rank-3 approximation of X and the same rounding
    rng = np.random.default_rng(4)
    sc = scenes.make_scene("tiny", 2)
    gt = sc.gt
    Ugt = (gt["s"][:, None, None] * gt["R"]).transpose(1, 0, 2).reshape(3, 3 * sc.N)
    O, _ = np.linalg.qr(rng.standard_normal((5, 5)))
    U = O @ np.vstack([Ugt + 0.05 * rng.standard_normal(Ugt.shape), 0.3 * rng.standard_normal((2, 3 * sc.N))])
    Ud = rd.top3_factor(U, method="dense")
    Ug = rd.top3_factor(U, method="gram")
    assert np.abs(Ud.T @ Ud - Ug.T @ Ug).max() <= 1e-10 * np.abs(Ud.T @ Ud).max()
    for a in range(3):
        assert min(np.abs(Ud[a] - Ug[a]).max(), np.abs(Ud[a] + Ug[a]).max()) <= 1e-9 * np.abs(Ud).max()
    Rd, sd = rd.round_solution(U, method="dense")
    Rg, sg = rd.round_solution(U, method="gram")
    assert np.abs(Rd - Rg).max() <= 1e-9 and np.abs(sd - sg).max() <= 1e-9 * np.abs(sd).max()
