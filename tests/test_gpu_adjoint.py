"""GPU adjoint (xm_adjoint / XMSolve.backward) against the oracle and finite differences."""
import numpy as np
import pytest

import scenes
from oracle import adjoint as oad
from oracle import manifold as omf
from oracle import rounding as ord_
from oracle import staircase as ost
from oracle import data_matrix as odm

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _xm():
    import paper_2502_04640_amd as xm
    xm.load_library()
    return xm


def _say(msg):
    print(msg, flush=True)


def _gpu_solution(sc, u, w, tol=1e-12):
    xm = _xm()
    P = xm.build_Q(sc.N, sc.M, torch.from_numpy(sc.frame).cuda(), torch.from_numpy(sc.landmark).cuda(),
                   torch.from_numpy(u).cuda(), torch.from_numpy(w).cuda(), keep=())
    Y, info = P.solve(xm.SolveOptions(compute="f64", grad_tol=tol))
    assert info["certified"] == 1
    R, s, rho = P.round(Y)
    return P, R, s, rho


def test_adjoint_matches_oracle_small():
    _say("case: adjoint vs oracle, N=20")
    sc = scenes.random_scene(20, 400, L=4, sigma=0.01, seed=41, weights=(0.5, 1.5))
    rng = np.random.default_rng(0)
    gR = rng.standard_normal((sc.N, 3, 3))
    gs = rng.standard_normal(sc.N)
    gc = 0.7
    # oracle at its own solution
    Q = odm.q_block_elimination(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w)
    Ro, so, oinfo = ost.staircase(Q, grad_tol=1e-13, tau=1e-8)
    Rh, sh = ord_.round_solution(omf.to_U(Ro, so))
    gu_o, gw_o = oad.ift_grad(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w, Rh, sh, gR, gs, Q=Q)
    cu, cw = oad.cost_grad(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w, oad.anchored_U(Rh, sh))
    gu_o = gu_o + gc * cu
    gw_o = gw_o + gc * cw
    # GPU
    P, R, s, _ = _gpu_solution(sc, sc.u, sc.w)
    gu, gw, info = P.adjoint(R, s, torch.from_numpy(gR).cuda(), torch.from_numpy(gs).cuda(), gc)
    gu, gw = gu.cpu().numpy(), gw.cpu().numpy()
    assert info["cg_residual"] <= 1e-9
    assert np.abs(gu - gu_o).max() <= 1e-6 * np.abs(gu_o).max()
    assert np.abs(gw - gw_o).max() <= 1e-6 * np.abs(gw_o).max()
    # and against the dense chart reference in random directions
    for _ in range(3):
        vu = rng.standard_normal(sc.u.shape)
        vw = 0.1 * rng.standard_normal(sc.w.shape)
        ref = oad.dense_reference(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w, Rh, sh, gR, gs, vu, vw)
        ref += gc * float(np.sum(cu * vu) + np.sum(cw * vw))
        an = float(np.sum(gu * vu) + np.sum(gw * vw))
        assert abs(an - ref) <= 1e-6 * max(1.0, abs(ref))


def test_recover_tp_matches_oracle():
    # eq. tpstar at the rounded optimum: noise-free (ground truth) and noisy
    # (the oracle's recovery at the same rotations and scales)
    _say("case: recover t, p")
    sc = scenes.random_scene(15, 300, L=4, sigma=0.0, seed=42, weights=(0.5, 1.5))
    P, R, s, _ = _gpu_solution(sc, sc.u, sc.w)
    t, p = P.recover_tp(R, s)
    assert np.abs(t.cpu().numpy() - sc.gt["t"]).max() <= 1e-7
    assert np.abs(p.cpu().numpy() - sc.gt["p"]).max() <= 1e-7
    sc = scenes.random_scene(40, 1500, L=4, sigma=0.05, seed=44, weights=(0.5, 1.5))
    P, R, s, _ = _gpu_solution(sc, sc.u, sc.w)
    t, p = P.recover_tp(R, s)
    U = ord_.rounded_U(R.cpu().numpy(), s.cpu().numpy())
    t_o, p_o = odm.recover_tp(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w, U)
    assert np.abs(t.cpu().numpy() - t_o).max() <= 1e-9 * np.abs(t_o).max()
    assert np.abs(p.cpu().numpy() - p_o).max() <= 1e-9 * np.abs(p_o).max()


def test_autograd_refuses_a_non_tight_optimum():
    # the benchmark scene (5% outlier observations): certified, but its optimum
    # has rank 4 and rounding loses eta ~ 0.08, so the implicit-function
    # gradient of the rotations is undefined: forward must refuse
    _say("case: XMSolve on the N=10155 outlier workload (rank-4 optimum)")
    xm = _xm()
    sc = scenes.make_scene("large", 0)
    u = torch.from_numpy(sc.u).cuda().requires_grad_(True)
    w = torch.from_numpy(sc.w).cuda().requires_grad_(True)
    with pytest.raises(xm.NotTightError, match="eta"):
        xm.XMSolve.apply(u, w, torch.from_numpy(sc.frame).cuda(), torch.from_numpy(sc.landmark).cuda(),
                         sc.N, sc.M, xm.SolveOptions(compute="f32"))


def test_autograd_function_backward():
    _say("case: XMSolve autograd")
    xm = _xm()
    sc = scenes.random_scene(12, 250, L=4, sigma=0.01, seed=43, weights=(0.5, 1.5))
    u = torch.from_numpy(sc.u).cuda().requires_grad_(True)
    w = torch.from_numpy(sc.w).cuda().requires_grad_(True)
    R, s, f = xm.XMSolve.apply(u, w, torch.from_numpy(sc.frame).cuda(), torch.from_numpy(sc.landmark).cuda(),
                               sc.N, sc.M, xm.SolveOptions(compute="f64", grad_tol=1e-12))
    rng = np.random.default_rng(1)
    gR = torch.from_numpy(rng.standard_normal((sc.N, 3, 3))).cuda()
    gs = torch.from_numpy(rng.standard_normal(sc.N)).cuda()
    loss = (gR * R).sum() + (gs * s).sum() + 0.3 * f
    loss.backward()
    Q = odm.q_block_elimination(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w)
    Ro, so, _ = ost.staircase(Q, grad_tol=1e-13, tau=1e-8)
    Rh, sh = ord_.round_solution(omf.to_U(Ro, so))
    gu_o, gw_o = oad.ift_grad(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w, Rh, sh, gR.cpu().numpy(),
                              gs.cpu().numpy(), Q=Q)
    cu, cw = oad.cost_grad(sc.N, sc.M, sc.frame, sc.landmark, sc.u, sc.w, oad.anchored_U(Rh, sh))
    assert np.abs(u.grad.cpu().numpy() - (gu_o + 0.3 * cu)).max() <= 1e-6 * np.abs(gu_o).max()
    assert np.abs(w.grad.cpu().numpy() - (gw_o + 0.3 * cw)).max() <= 1e-6 * np.abs(gw_o).max()


@pytest.mark.parametrize("n_dirs", [64])
def test_adjoint_finite_differences_diff_workload(n_dirs):
    # the differentiation workload: N=500, ~225k observations, FP32 keypoints and
    # weights; central differences (h=1e-4, FP64) of the whole GPU pipeline
    # (re-solve + rounding) on random directions, relative error <= 1e-4
    _say(f"case: adjoint FD on the N=500 workload, {n_dirs} directions")
    sc = scenes.make_scene("diff", 0)
    u = sc.u.astype(np.float32).astype(np.float64)
    w = sc.w.astype(np.float32).astype(np.float64)
    P, R, s, rho = _gpu_solution(sc, u, w, tol=1e-11)
    rng = np.random.default_rng(7)
    gR = rng.standard_normal((sc.N, 3, 3))
    gs = rng.standard_normal(sc.N)
    gc = 1e-3
    gu, gw, info = P.adjoint(R, s, torch.from_numpy(gR).cuda(), torch.from_numpy(gs).cuda(), gc,
                             dtype=torch.float32)
    gu = gu.double().cpu().numpy()
    gw = gw.double().cpu().numpy()
    _say(f"  cg iters {info['cg_iters']} residual {info['cg_residual']:.2e}")
    h = 1e-4

    def loss(du, dw):
        _, Rx, sx, rx = _gpu_solution(sc, u + du, w + dw, tol=1e-11)
        return float(np.sum(gR * Rx.cpu().numpy()) + np.sum(gs * sx.cpu().numpy()) + gc * rx)

    errs = []
    for d in range(n_dirs):
        vu = rng.standard_normal(u.shape)
        vw = 0.1 * rng.standard_normal(w.shape)
        fd = (loss(h * vu, h * vw) - loss(-h * vu, -h * vw)) / (2 * h)
        an = float(np.sum(gu * vu) + np.sum(gw * vw))
        errs.append(abs(fd - an) / max(1e-12, abs(fd)))
    _say(f"  max rel err {max(errs):.2e}, median {np.median(errs):.2e}")
    assert max(errs) <= 1e-4
