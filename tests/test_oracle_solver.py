"""Pins for the oracle's manifold calculus, RTR-tCG, staircase, certificate and rounding."""
import numpy as np
import pytest

import scenes
from oracle import certificate as ce
from oracle import data_matrix as dm
from oracle import manifold as mf
from oracle import rounding as rd
from oracle import rtr
from oracle import staircase as st


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


@pytest.mark.parametrize("r", [3, 5])
def test_gradient_matches_finite_difference(small, r):
    sc, Q = small
    rng = np.random.default_rng(r)
    R, s = _rand_point(rng, sc.N, r)
    Rd, sd = _rand_tangent(rng, R, s)
    gR, gs = mf.rgrad(Q, R, s)
    h = 1e-6
    fp = mf.cost(Q, *mf.retract(R, s, h * Rd, h * sd))
    fm = mf.cost(Q, *mf.retract(R, s, -h * Rd, -h * sd))
    fd = (fp - fm) / (2 * h)
    assert abs(fd - mf.inner(s, gR, gs, Rd, sd)) <= 1e-6 * max(1.0, abs(fd))


@pytest.mark.parametrize("r", [3, 4])
def test_hessian_is_projected_derivative_of_gradient(small, r):
    # On a Riemannian submanifold of Euclidean space the Hessian is the projected
    # derivative of (any extension of) the gradient field.  In (R, log s)
    # coordinates the metric is Euclidean, so differentiate there.
    sc, Q = small
    rng = np.random.default_rng(10 + r)
    R, s = _rand_point(rng, sc.N, r)
    Rd, sd = _rand_tangent(rng, R, s)
    h = 1e-5

    def grad_log(Rx, sig):
        gR, gs = mf.rgrad(Q, Rx, np.exp(sig))
        return gR, gs / np.exp(sig)          # gradient in sigma units: s * df/ds

    sig = np.log(s)
    sig_d = sd / s
    gp = grad_log(R + h * Rd, sig + h * sig_d)
    gm = grad_log(R - h * Rd, sig - h * sig_d)
    dR = mf.proj(R, (gp[0] - gm[0]) / (2 * h))
    dsig = (gp[1] - gm[1]) / (2 * h)
    HR, Hs = mf.hess(Q, R, s, Rd, sd)
    scale = np.abs(HR).max()
    assert np.abs(HR - dR).max() <= 1e-6 * scale
    assert np.abs(Hs / s - dsig)[1:].max() <= 1e-6 * scale


def test_hessian_symmetric(small):
    sc, Q = small
    rng = np.random.default_rng(7)
    R, s = _rand_point(rng, sc.N, 4)
    a = _rand_tangent(rng, R, s)
    b = _rand_tangent(rng, R, s)
    Ha = mf.hess(Q, R, s, *a)
    Hb = mf.hess(Q, R, s, *b)
    x = mf.inner(s, *a, *Hb)
    y = mf.inner(s, *b, *Ha)
    assert abs(x - y) <= 1e-12 * max(abs(x), 1.0)


def test_noise_free_recovers_ground_truth():
    sc = scenes.make_scene("tiny", 3, sigma=0.0)
    Q = _Q(sc)
    R, s, info = st.staircase(Q, grad_tol=1e-12)
    assert info["r"] == 3 and info["certified"]
    assert info["cost"] <= 1e-9 * info["qbar"]
    Rh, sh = rd.round_solution(mf.to_U(R, s))
    assert np.abs(Rh - sc.gt["R"]).max() <= 1e-8
    assert np.abs(sh - sc.gt["s"]).max() <= 1e-8


def test_two_frames_match_umeyama():
    # N = 2, every landmark seen by both frames: SBA is weighted similarity
    # registration (Remark "Connection to Other Perception Problems"), solved in
    # closed form by Umeyama (1991) / Horn (1987) with the SO(3) determinant fix.
    sc = scenes.random_scene(2, 60, L=2, sigma=0.05, seed=8, weights=(0.5, 1.5))
    Q = _Q(sc)
    R, s, info = st.staircase(Q, grad_tol=1e-12)
    assert info["certified"]
    Rh, sh = rd.round_solution(mf.to_U(R, s))
    # closed form for: min sum_k c_k || a_k - (sigma Rot b_k + t) ||^2
    M = sc.M
    a = np.zeros((M, 3)); b = np.zeros((M, 3)); wa = np.zeros(M); wb = np.zeros(M)
    for o in range(sc.n_obs):
        if sc.frame[o] == 0:
            a[sc.landmark[o]] = sc.u[o]; wa[sc.landmark[o]] = sc.w[o]
        else:
            b[sc.landmark[o]] = sc.u[o]; wb[sc.landmark[o]] = sc.w[o]
    c = wa * wb / (wa + wb)
    C = c.sum()
    ma = (c[:, None] * a).sum(0) / C
    mb = (c[:, None] * b).sum(0) / C
    Sig = ((c[:, None, None] * (a - ma)[:, :, None] * (b - mb)[:, None, :]).sum(0)) / C
    Us, D, Vt = np.linalg.svd(Sig)
    S = np.diag([1, 1, np.sign(np.linalg.det(Us) * np.linalg.det(Vt))])
    Rot = Us @ S @ Vt
    var_b = (c * ((b - mb) ** 2).sum(1)).sum() / C
    sig = np.trace(np.diag(D) @ S) / var_b
    t = ma - sig * Rot @ mb
    cost_cf = float((c * ((a - (sig * b @ Rot.T + t)) ** 2).sum(1)).sum())
    assert np.abs(Rh[1] - Rot).max() <= 1e-9
    assert abs(sh[1] - sig) <= 1e-9 * sig
    assert abs(info["cost"] - cost_cf) <= 1e-9 * max(1.0, cost_cf)


def test_multistart_three_frames():
    # For N = 3 the certified staircase optimum must be the best of many random
    # rank-3 local solves, and none may go below it.
    sc = scenes.random_scene(3, 40, L=3, sigma=0.2, seed=9)
    Q = _Q(sc)
    R, s, info = st.staircase(Q, grad_tol=1e-12)
    assert info["certified"]
    rng = np.random.default_rng(0)
    costs = []
    for _ in range(60):
        R0, s0 = _rand_point(rng, 3, 3)
        _, _, inf = rtr.rtr(Q, R0, s0, grad_tol=1e-12)
        costs.append(inf["cost"])
    costs = np.array(costs)
    tol = 1e-9 * max(1.0, info["cost"])
    assert costs.min() >= info["cost"] - tol
    assert abs(costs.min() - info["cost"]) <= tol


def test_certificate_invariants_and_weak_duality():
    sc = scenes.make_scene("tiny", 1)
    Q = _Q(sc)
    R, s, info = st.staircase(Q, grad_tol=1e-11)
    assert info["certified"]
    U = mf.to_U(R, s)
    Lam = info["Lambda"]
    Z = ce.dual_matrix(Q, Lam)
    # Z U^T = 0 up to the gradient level; primal = dual at the critical point
    assert np.abs(Z @ U.T).max() <= 1e-7 * info["qbar"]
    assert abs(info["primal"] - info["dual"]) <= 1e-7 * max(1.0, info["primal"])
    assert info["lambda_min_full"] >= -1e-8 * info["qbar"]
    # weak duality: every feasible X of the SDP has tr(QX) >= tr(Lambda_0)
    rng = np.random.default_rng(2)
    for r in (3, 5, 8):
        R0, s0 = _rand_point(rng, sc.N, r)
        X_U = mf.to_U(R0, s0)
        assert np.sum(X_U * (X_U @ Q)) >= info["dual"] - 1e-9 * abs(info["dual"])


def test_escape_strictly_decreases_cost():
    # A seeded rank-3 local minimum with a negative dual eigenvalue (heavy noise);
    # Theorem "Descent Direction": the escape along [0; v^T] lowers the cost and
    # keeps every block feasible.
    sc = scenes.random_scene(8, 40, L=3, sigma=0.5, seed=0)
    Q = _Q(sc)
    rng = np.random.default_rng(0)
    R, s = mf.gram_schmidt(rng.standard_normal((sc.N, 3, 3))), np.exp(rng.standard_normal(sc.N) * 0.3)
    s[0] = 1.0
    R, s, info = rtr.rtr(Q, R, s, grad_tol=1e-11)
    c = ce.certify(Q, R, s, 1e-8)
    assert c["lambda_min"] < -1e-3 * c["qbar"]
    out = st.escape(Q, R, s, c["v"])
    assert out is not None
    Rn, sn, alpha = out
    assert mf.cost(Q, Rn, sn) < info["cost"]
    eye = np.einsum("nab,nac->nbc", Rn, Rn)
    assert np.abs(eye - np.eye(3)).max() <= 1e-13
    # and the staircase from there ends certified with a lower cost
    Rf, sf, inf2 = st.staircase(Q, R0=Rn, s0=sn, r_max=8, grad_tol=1e-10)
    assert inf2["certified"] and inf2["cost"] < info["cost"]


def test_rounding_exact_rank3_is_identity():
    sc = scenes.make_scene("tiny", 2)
    gt = sc.gt
    Ugt = (gt["s"][:, None, None] * gt["R"]).transpose(1, 0, 2).reshape(3, 3 * sc.N)
    rng = np.random.default_rng(4)
    # embed in rank 5 with a random orthogonal 5x5 (X unchanged), reflection included
    O, _ = np.linalg.qr(rng.standard_normal((5, 5)))
    U5 = O @ np.vstack([Ugt, np.zeros((2, 3 * sc.N))])
    Rh, sh = rd.round_solution(U5)
    assert np.abs(Rh - gt["R"]).max() <= 1e-11
    assert np.abs(sh - gt["s"]).max() <= 1e-11


def test_suboptimality_tight_scene():
    sc = scenes.make_scene("tiny", 0)
    Q = _Q(sc)
    R, s, info = st.staircase(Q, grad_tol=1e-11)
    Rh, sh = rd.round_solution(mf.to_U(R, s))
    Uh = rd.rounded_U(Rh, sh)
    rho_hat = float(np.sum(Uh * (Uh @ Q)))
    eta = ce.suboptimality(rho_hat, info["cost"])
    assert info["certified"] and info["r"] == 3
    assert 0 <= eta + 1e-12 and eta <= 1e-10


def _d_complement_gen_eig(Q, Z, U):
    """min of v^T Z v / v^T D v over v D-orthogonal to rows(U), D = blkdiag(Q_kk),
    as a generalized symmetric eigenproblem on an explicit basis (scipy)."""
    import scipy.linalg as sla
    N = Q.shape[0] // 3
    D = np.zeros_like(Q)
    for k in range(N):
        D[3 * k:3 * k + 3, 3 * k:3 * k + 3] = Q[3 * k:3 * k + 3, 3 * k:3 * k + 3]
    C = sla.null_space((D @ U.T).T)                  # basis of {v : U D v = 0}
    return float(sla.eigh(C.T @ Z @ C, C.T @ D @ C, eigvals_only=True)[0]), D


@pytest.mark.parametrize("case", ["certified", "spurious"])
def test_scaled_certificate_inertia_and_bound(case):
    # Sylvester's law of inertia: Zs = D^{-1/2} Z D^{-1/2} has the sign pattern
    # of Z; its deflated minimum equals the generalized Rayleigh minimum of
    # (Z, D) on the D-orthogonal complement of rows(U), and lambda_bound bounds
    # v^T Z v for unit v there.
    if case == "certified":
        sc = scenes.make_scene("tiny", 1)
        Q = _Q(sc)
        R, s, _ = st.staircase(Q, grad_tol=1e-11)
    else:
        sc = scenes.random_scene(8, 40, L=3, sigma=0.5, seed=0)
        Q = _Q(sc)
        rng = np.random.default_rng(0)
        R, s = mf.gram_schmidt(rng.standard_normal((sc.N, 3, 3))), np.exp(rng.standard_normal(sc.N) * 0.3)
        s[0] = 1.0
        R, s, _ = rtr.rtr(Q, R, s, grad_tol=1e-11)
    c = ce.certify(Q, R, s, 1e-8)
    U = mf.to_U(R, s)
    Z = ce.dual_matrix(Q, c["Lambda"])
    gen, D = _d_complement_gen_eig(Q, Z, U)
    assert abs(c["lambda_min_scaled"] - gen) <= 1e-9 * max(1.0, abs(gen))
    n_neg = lambda A: int(np.sum(np.linalg.eigvalsh(A) < -1e-9 * np.abs(A).max()))
    Dm = np.linalg.inv(np.linalg.cholesky(D))
    assert n_neg(Dm @ Z @ Dm.T) == n_neg(Z)
    if case == "certified":
        assert c["lambda_min_scaled"] >= -1e-9 and c["lambda_bound"] >= -1e-8 * c["qbar"]
    else:
        assert c["lambda_min"] < 0 and c["lambda_min_scaled"] < 0 and c["lambda_bound"] < 0
    rng = np.random.default_rng(5)
    P = np.eye(Q.shape[0]) - (D @ U.T) @ np.linalg.solve(U @ D @ D @ U.T, U @ D)
    for _ in range(200):
        v = P @ rng.standard_normal(Q.shape[0])
        v /= np.linalg.norm(v)
        assert v @ Z @ v >= c["lambda_bound"] - 1e-9 * c["qbar"]


@pytest.mark.parametrize("case", ["optimum", "near", "perturbed", "random", "rank5"])
def test_full_spectrum_bound_holds_at_any_point(case):
    # certificate_bound bounds the smallest eigenvalue of Zs over the whole space
    # (the exact one from a dense eigvalsh) at any point, with the spectral and the
    # (larger) Frobenius cross norm; at a critical point the deflated block
    # contributes ~0 and the bound is that smallest eigenvalue itself
    sc = scenes.make_scene("tiny", 1)
    Q = _Q(sc)
    R, s, info = st.staircase(Q, grad_tol=1e-11)
    rng = np.random.default_rng(3)
    eps = {"optimum": 0.0, "near": 1e-4, "perturbed": 0.05}.get(case)
    if case == "random":
        R, s = _rand_point(rng, sc.N, 3)
    elif eps:
        R = mf.gram_schmidt(R + eps * rng.standard_normal(R.shape))
        s = s * np.exp(eps * rng.standard_normal(s.shape))
        s[0] = 1.0
    U = mf.to_U(R, s)
    if case == "rank5":
        # a rank-5 factor of the rank-3 optimum whose two extra rows carry only
        # gradient-level residue (mixed in by a random orthogonal 5x5)
        O, _ = np.linalg.qr(rng.standard_normal((5, 5)))
        U = O @ np.vstack([U, 1e-8 * rng.standard_normal((2, U.shape[1]))])
        s = mf.from_U(U)[1]
    cb = ce.certificate_bound(Q, U)
    full = cb["lambda_min_scaled_full"]
    assert cb["bound_scaled"] <= full + 1e-12 * max(1.0, abs(full))
    assert cb["bound_scaled_fro"] <= cb["bound_scaled"] + 1e-15
    Z = ce.dual_matrix(Q, ce.dual_lambda(Q, U, s))
    lam_Z = float(np.linalg.eigvalsh(Z)[0])
    assert cb["lambda_bound"] <= lam_Z + 1e-10 * info["qbar"]
    if case in ("optimum", "rank5"):
        assert abs(cb["bound_scaled_fro"] - full) <= 1e-10
        assert cb["cross_fro"] <= 1e-7 and abs(cb["defl_min"]) <= 1e-12
    if case == "rank5":
        # keeping the residue rows in the basis would wreck the bound
        bad = ce.certificate_bound(Q, U, rel=1e-14)
        assert bad["bound_scaled_fro"] < -1e-3 and bad["bound_scaled_fro"] <= bad["lambda_min_scaled_full"]


def test_complement_alone_would_certify_a_non_critical_point():
    # A perturbed optimum: Zs is positive on the complement of D^{1/2} rows(U)
    # (the complement-only bound says "certified"), yet Z has a negative
    # eigenvalue well below the tolerance; the full-spectrum bound rejects it.
    sc = scenes.make_scene("tiny", 1)
    Q = _Q(sc)
    R, s, info = st.staircase(Q, grad_tol=1e-11)
    rng = np.random.default_rng(3)
    R = mf.gram_schmidt(R + 0.05 * rng.standard_normal(R.shape))
    s = s * np.exp(0.05 * rng.standard_normal(s.shape))
    s[0] = 1.0
    c = ce.certify(Q, R, s, 1e-7)
    tol = 1e-7 * c["qbar"]
    assert c["lambda_bound"] >= -tol                      # complement alone: PSD
    assert c["lambda_min_full"] < -1e3 * tol              # Z is not PSD
    assert c["lambda_bound_full"] < -tol                  # the full bound says so
