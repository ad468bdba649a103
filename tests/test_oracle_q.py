"""Pins for the oracle's data matrix Q (App. A) against things other than itself."""
import numpy as np
import pytest

import scenes
from oracle import data_matrix as dm


def _args(sc):
    return sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_paper_formula_equals_block_elimination(seed):
    sc = scenes.random_scene(7, 50, L=3, sigma=0.05, seed=seed, weights=(0.5, 1.5))
    Qa = dm.q_paper_formula(*_args(sc))
    Qb = dm.q_block_elimination(*_args(sc))
    assert np.abs(Qa - Qb).max() <= 1e-12 * np.abs(Qa).max()


@pytest.mark.parametrize("r", [3, 4, 5])
def test_brute_force_least_squares(r):
    # tr(Q U^T U) = min over t (t_0 = 0) and p of the SBA cost (eq. sba), for any U.
    sc = scenes.random_scene(6, 40, L=3, sigma=0.1, seed=10 + r, weights=(0.5, 1.5))
    Q = dm.q_block_elimination(*_args(sc))
    rng = np.random.default_rng(r)
    for _ in range(3):
        U = rng.standard_normal((r, 3 * sc.N))
        bf = dm.brute_force_cost(*_args(sc), U)
        assert abs(bf - np.sum(U * (U @ Q))) <= 1e-10 * max(1.0, bf)


def test_two_frame_closed_form():
    # N = 2 with every landmark in both frames: eliminating p_k leaves
    # c_k ||U_0 a_k - U_1 b_k - t||^2 with c_k = w0 w1 / (w0 + w1); eliminating
    # t centres a, b by the c-weighted means.  Q is then written by hand.
    rng = np.random.default_rng(3)
    M = 30
    a = rng.standard_normal((M, 3))
    b = rng.standard_normal((M, 3))
    w0 = rng.uniform(0.5, 2.0, M)
    w1 = rng.uniform(0.5, 2.0, M)
    frame = np.r_[np.zeros(M, np.int32), np.ones(M, np.int32)]
    landmark = np.r_[np.arange(M), np.arange(M)].astype(np.int32)
    u = np.r_[a, b]
    w = np.r_[w0, w1]
    Q = dm.q_block_elimination(2, M, frame, landmark, u, w)
    c = w0 * w1 / (w0 + w1)
    ac = a - (c[:, None] * a).sum(0) / c.sum()
    bc = b - (c[:, None] * b).sum(0) / c.sum()
    Qh = np.zeros((6, 6))
    Qh[:3, :3] = (c[:, None, None] * ac[:, :, None] * ac[:, None, :]).sum(0)
    Qh[3:, 3:] = (c[:, None, None] * bc[:, :, None] * bc[:, None, :]).sum(0)
    Qh[:3, 3:] = -(c[:, None, None] * ac[:, :, None] * bc[:, None, :]).sum(0)
    Qh[3:, :3] = Qh[:3, 3:].T
    assert np.abs(Q - Qh).max() <= 1e-12 * np.abs(Qh).max()


def test_psd_and_laplacian_structure():
    sc = scenes.make_scene("tiny", 0)
    Q, (A_rr, A_rt, A_tt) = dm.q_block_elimination(*_args(sc), return_parts=True)
    ev = np.linalg.eigvalsh(Q)
    assert ev[0] >= -1e-10 * ev[-1]
    # translation invariance: A_tt 1 = 0, A_rt 1 = 0 (Lemma "laplacian")
    one = np.ones(sc.N)
    assert np.abs(A_tt @ one).max() <= 1e-12 * np.abs(A_tt).max()
    assert np.abs(A_rt @ one).max() <= 1e-12 * np.abs(A_rt).max()
    # grounded Laplacian is SPD for a connected view graph
    assert np.linalg.eigvalsh(A_tt[1:, 1:])[0] > 0


def test_noise_free_null_space():
    # Without noise the anchored ground truth attains cost 0: Q U_gt^T = 0 and
    # Q has exactly three zero eigenvalues (the rows of U_gt).
    sc = scenes.random_scene(12, 300, L=4, sigma=0.0, seed=4)
    Q = dm.q_block_elimination(*_args(sc))
    gt = sc.gt
    Ugt = (gt["s"][:, None, None] * gt["R"]).transpose(1, 0, 2).reshape(3, 3 * sc.N)
    assert np.abs(Q @ Ugt.T).max() <= 1e-11 * np.abs(Q).max()
    ev = np.linalg.eigvalsh(Q)
    assert np.all(np.abs(ev[:3]) <= 1e-10 * ev[-1])
    assert ev[3] > 1e-6 * ev[-1]


def test_recover_tp_matches_cost_and_ground_truth():
    sc = scenes.random_scene(9, 120, L=3, sigma=0.0, seed=5, weights=(0.5, 1.5))
    gt = sc.gt
    Ugt = (gt["s"][:, None, None] * gt["R"]).transpose(1, 0, 2).reshape(3, 3 * sc.N)
    t, p = dm.recover_tp(*_args(sc), Ugt)
    assert np.abs(t - gt["t"]).max() <= 1e-9
    assert np.abs(p - gt["p"]).max() <= 1e-9
    rng = np.random.default_rng(1)
    U = rng.standard_normal((4, 3 * sc.N))
    Q = dm.q_block_elimination(*_args(sc))
    t, p = dm.recover_tp(*_args(sc), U)
    assert abs(dm.sba_cost(sc.frame, sc.landmark, sc.u, sc.w, U, t, p) - np.sum(U * (U @ Q))) <= 1e-9 * np.sum(U * (U @ Q))


def test_single_observation_landmark_contributes_nothing():
    sc = scenes.random_scene(5, 30, L=3, sigma=0.05, seed=6)
    Q0 = dm.q_block_elimination(*_args(sc))
    fr = np.r_[sc.frame, np.int32(2)]
    lm = np.r_[sc.landmark, np.int32(sc.M)]
    u = np.r_[sc.u, [[0.3, -1.0, 2.0]]]
    w = np.r_[sc.w, 1.7]
    Q1 = dm.q_block_elimination(sc.N, sc.M + 1, fr, lm, u, w)
    assert np.abs(Q1 - Q0).max() <= 1e-12 * np.abs(Q0).max()


def test_q_rows_equals_full_construction():
    sc = scenes.random_scene(9, 120, L=4, sigma=0.03, seed=12, weights=(0.5, 1.5))
    Q = dm.q_block_elimination(*_args(sc))
    rows = np.array([0, 4, 13, 26])
    Qr = dm.q_rows(*_args(sc), rows)
    assert np.abs(Qr - Q[rows]).max() <= 1e-12 * np.abs(Q).max()
