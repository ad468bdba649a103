"""Dual certificate (test infrastructure: oracle only).

Theorem "Dual Optimality Certificate": at a BM local optimum U there is a
unique y with Z(y) U^T = 0 (eq. bm_first_order_optimality), Z(y) = Q - sum
y_i A_i (eq. Zofy); if Z(y) is PSD the point is globally optimal for the SDP.

The A_i (App. "Proof of LICQ condition") act on the diagonal 3x3 blocks only:
for frames k >= 1 they span the traceless symmetric matrices (B^1..B^5), for
frame 0 one more constraint (unit diagonal) makes the span all of S^3.  So
sum y_i A_i = blkdiag(Lambda_k); solving Lambda_k U_k^T = (Q U^T)_k gives
Lambda_k = (Q U^T)_k U_k / alpha_k with alpha_k = s_k^2, symmetrised, and made
traceless for k >= 1.  The dual objective b^T y is tr(Lambda_0).

Readings (listed in the design notes): the PSD test uses a relative
tolerance, certified <=> lambda_min >= -tau * qbar, qbar = tr(Q)/3N; the
minimum eigenvalue is taken on the orthogonal complement of the rows of U
(Z U^T = 0 puts those directions at zero); the escape vector is normalised
to unit length with its largest-magnitude entry positive.

Block-Jacobi scaled form (what the GPU's Lanczos measures): with
D = blkdiag(Q_kk), Zs = D^{-1/2} Z D^{-1/2} is congruent to Z, so by
Sylvester's law of inertia both have the same number of negative
eigenvalues.  min_eig_scaled takes the smallest eigenvalue ls of Zs on the
orthogonal complement of D^{1/2} rows(U) (the D-orthogonal complement of
rows(U) in the coordinates of Z); for v in that complement
v^T Z v >= ls v^T D v, which gives the lower bound
lambda_bound = ls * (d_min if ls >= 0 else d_max) over unit v, d_min, d_max
the extreme eigenvalues of the Q_kk.

That bound covers the complement only, which decides PSD-ness of Z only when
Z U^T = 0.  certificate_bound folds in the deflated block itself (its
smallest eigenvalue and its coupling to the complement, both zero at a
critical point) to bound the whole spectrum, so that a U that is not a
critical point is not taken for a certificate.
"""
from __future__ import annotations

import numpy as np

from . import manifold as mf


def dual_lambda(Q, U, s, QU=None):
    """Lambda [N, 3, 3]: Lambda_k = sym((Q U^T)_k U_k) / s_k^2, traceless for k >= 1.
    QU (3N x r) may be given instead of Q (matrix-free callers)."""
    N = U.shape[1] // 3
    if QU is None:
        QU = (Q @ U.T)                              # 3N x r
    L = np.empty((N, 3, 3))
    for k in range(N):
        Uk = U[:, 3 * k:3 * k + 3]                  # r x 3
        Lk = QU[3 * k:3 * k + 3, :] @ Uk / (s[k] ** 2)
        Lk = 0.5 * (Lk + Lk.T)
        if k > 0:
            Lk = Lk - np.trace(Lk) / 3.0 * np.eye(3)
        L[k] = Lk
    return L


def dual_matrix(Q, Lam):
    """Z = Q - blkdiag(Lambda)."""
    Z = Q.copy()
    for k in range(Lam.shape[0]):
        Z[3 * k:3 * k + 3, 3 * k:3 * k + 3] -= Lam[k]
    return Z


def min_eig(Z, U):
    """Minimum eigenvalue of Z on the orthogonal complement of rows(U), with its
    eigenvector (unit norm, largest |entry| positive).  Also the minimum of the
    full spectrum.  Dense eigendecomposition."""
    n = Z.shape[0]
    Qf, _ = np.linalg.qr(U.T, mode="complete")
    r = np.linalg.matrix_rank(U)
    C = Qf[:, r:]
    lam, V = np.linalg.eigh(C.T @ Z @ C)
    v = C @ V[:, 0]
    v = v / np.linalg.norm(v)
    if v[np.argmax(np.abs(v))] < 0:
        v = -v
    full = float(np.linalg.eigvalsh(Z)[0])
    return float(lam[0]), v, full


def block_sqrt(Q):
    """Q_kk^{1/2}, Q_kk^{-1/2} per frame and (d_min, d_max) over all blocks (eigh)."""
    N = Q.shape[0] // 3
    Dh = np.empty((N, 3, 3))
    Dm = np.empty((N, 3, 3))
    lo, hi = np.inf, -np.inf
    for k in range(N):
        B = Q[3 * k:3 * k + 3, 3 * k:3 * k + 3]
        lam, V = np.linalg.eigh(0.5 * (B + B.T))
        lam = np.maximum(lam, 1e-12 * lam[-1])
        Dh[k] = (V * np.sqrt(lam)) @ V.T
        Dm[k] = (V / np.sqrt(lam)) @ V.T
        lo, hi = min(lo, lam[0]), max(hi, lam[-1])
    return Dh, Dm, float(lo), float(hi)


def _blkdiag(B):
    N = B.shape[0]
    M = np.zeros((3 * N, 3 * N))
    for k in range(N):
        M[3 * k:3 * k + 3, 3 * k:3 * k + 3] = B[k]
    return M


def min_eig_scaled(Q, Z, U):
    """Smallest eigenvalue of Zs = D^{-1/2} Z D^{-1/2} on the orthogonal
    complement of D^{1/2} rows(U), D = blkdiag(Q_kk), and the lower bound on
    v^T Z v (unit v, D-orthogonal to rows(U)) it implies.  Dense."""
    Dh, Dm, dmin, dmax = block_sqrt(Q)
    Dmh = _blkdiag(Dm)
    Zs = Dmh @ Z @ Dmh
    lam, _, _ = min_eig(0.5 * (Zs + Zs.T), U @ _blkdiag(Dh))
    bound = lam * (dmin if lam >= 0 else dmax)
    return lam, bound, dmin, dmax


def _orth_basis(A, rel=1e-10):
    """Orthonormal basis of the column space of A (columns with a singular
    value below rel times the largest are dropped)."""
    Uo, sv, _ = np.linalg.svd(A, full_matrices=False)
    if sv.size == 0 or sv[0] == 0:
        return Uo[:, :0]
    return Uo[:, sv > rel * sv[0]]


def certificate_bound(Q, U, rel=1e-3, D_from=None):
    """Lower bound on the whole spectrum of Zs = D^{-1/2} Z D^{-1/2} from the
    deflated block, valid at any U (not only at critical points).

    W: orthonormal basis of the part of D^{1/2} rows(U) whose singular values
    are at least `rel` times the largest (rows that are numerically
    combinations of the others, as a rank-5 factor of a rank-3 optimum
    carries, would add directions with a large coupling term; left out, they
    are part of the complement).  The bound holds for any W.  For unit v = x + y with x in
    span W and y orthogonal to it, v^T Zs v >= a|x|^2 + b|y|^2 - 2e|x||y|,
    with a = lambda_min(W^T Zs W), b = lambda_min of Zs on the complement and
    e = |(I - W W^T) Zs W|; minimising over |x|^2 + |y|^2 = 1 gives
    (a + b)/2 - sqrt(((a - b)/2)^2 + e^2).  Returns a, b, e (spectral norm),
    e_fro (Frobenius norm, an upper bound on e), the bound with each, the
    bound on v^T Z v for unit v it implies (d_min or d_max scaling, with the
    Frobenius form), and the exact smallest eigenvalue of Zs (dense).  Q here
    is the matrix the multipliers are taken from (Q + grad F(X) with the scale
    regulariser); D_from (default Q) gives the scaling blocks D."""
    Lam = dual_lambda(Q, U, mf.from_U(U)[1])
    Z = dual_matrix(Q, Lam)
    Dh, Dm, dmin, dmax = block_sqrt(Q if D_from is None else D_from)
    Dmh = _blkdiag(Dm)
    Zs = Dmh @ Z @ Dmh
    Zs = 0.5 * (Zs + Zs.T)
    W = _orth_basis(_blkdiag(Dh) @ U.T, rel)
    ZW = Zs @ W
    Mw = W.T @ ZW
    a = float(np.linalg.eigvalsh(0.5 * (Mw + Mw.T))[0])
    E = ZW - W @ Mw
    e = float(np.linalg.norm(E, 2))
    e_fro = float(np.linalg.norm(E))
    n = Zs.shape[0]
    Qf, _ = np.linalg.qr(W, mode="complete")
    C = Qf[:, W.shape[1]:]
    b = float(np.linalg.eigvalsh(C.T @ Zs @ C)[0])

    def comb(ee):
        return 0.5 * (a + b) - np.sqrt(0.25 * (a - b) ** 2 + ee * ee)

    full = comb(e_fro)
    return {"defl_min": a, "complement_min": b, "cross": e, "cross_fro": e_fro,
            "bound_scaled": float(comb(e)), "bound_scaled_fro": float(full),
            "lambda_bound": float(full * (dmin if full >= 0 else dmax)),
            "lambda_min_scaled_full": float(np.linalg.eigvalsh(Zs)[0]), "dmin": dmin, "dmax": dmax, "n": n}


def reg_gradient(s, lam):
    """Diagonal of grad F(X) for F = lam sum_{i>=2} (X_{3i,3i} - 1)^2
    (eq. problem-sdp-scale): 2 lam (X_{3k+2,3k+2} - 1) = 2 lam (s_k^2 - 1) at
    index 3k+2 for frames k >= 1 (0-based; the paper's index 3i), 0 elsewhere."""
    N = s.shape[0]
    g = np.zeros(3 * N)
    g[3 * np.arange(1, N) + 2] = 2.0 * lam * (s[1:] ** 2 - 1.0)
    return g


def certify(Q, R, s, tau, lam=0.0):
    """Certificate at (R, s): dict with lambda_min (complement), lambda_min_full,
    primal, dual, certified flag and escape vector.

    With the scale regulariser (lam > 0, App. "Scale Regularization") the dual
    matrix is Z = Q + grad F(X) - blkdiag(Lambda) at X = U^T U, the multipliers
    come from the same stationarity condition with Q + grad F(X) in place of Q,
    the primal value is tr(Q X) + F(X) and the dual value
    tr(Lambda_0) + F(X) - <grad F(X), X>."""
    U = mf.to_U(R, s)
    g = reg_gradient(s, lam)
    Qe = Q + np.diag(g)
    Lam = dual_lambda(Qe, U, s)
    Z = dual_matrix(Qe, Lam)
    lam_c, v, full = min_eig(Z, U)
    lam_s, bound, dmin, dmax = min_eig_scaled(Q, Z, U)
    cb = certificate_bound(Qe, U, D_from=Q)
    N = R.shape[0]
    qbar = float(np.trace(Q)) / (3 * N)
    X_diag = np.repeat(s * s, 3)
    F = mf.scale_reg(s, lam)
    primal = float(np.sum(U * (U @ Q))) + F
    dual = float(np.trace(Lam[0])) + F - float(g @ X_diag)
    return {"lambda_min": lam_c, "lambda_min_full": full, "v": v, "primal": primal,
            "dual": dual, "certified": bool(lam_c >= -tau * qbar), "qbar": qbar, "Lambda": Lam,
            "lambda_min_scaled": lam_s, "lambda_bound": bound, "dmin": dmin, "dmax": dmax,
            "defl_min": cb["defl_min"], "defl_cross": cb["cross_fro"], "lambda_bound_full": cb["lambda_bound"],
            "stat_res": float(np.linalg.norm(Z @ U.T))}


def suboptimality(rho_hat, rho_sdp):
    """eta = (rho_hat - rho_sdp) / (1 + |rho_hat| + |rho_sdp|)   (eq. suboptimality)."""
    return (rho_hat - rho_sdp) / (1.0 + abs(rho_hat) + abs(rho_sdp))


def suboptimality_dual(rho_hat, rho_dual, lambda_min, trace_X):
    """eq. suboptimality_new (App. "Suboptimality for SDP"): the lower bound
    lb = max(0, lambda_min(Z)) tr(X) + rho_dual on the SDP optimum replaces
    rho_SDP, eta = (rho_hat - lb) / (1 + |rho_hat| + |lb|)."""
    lb = max(0.0, lambda_min) * trace_X + rho_dual
    return (rho_hat - lb) / (1.0 + abs(rho_hat) + abs(lb))


# ---------------------------------------------------------------------------
# Matrix-free certificate for scenes whose dense Q does not fit: Q enters only
# through products (data_matrix.QOperator) and its diagonal blocks.

def _blk_apply(B, x):
    """blkdiag(B) x for B [N, 3, 3] and x (3N,) or (3N, k)."""
    N = B.shape[0]
    if x.ndim == 1:
        return np.einsum("nab,nb->na", B, x.reshape(N, 3)).reshape(-1)
    k = x.shape[1]
    return np.einsum("nab,nbk->nak", B, x.reshape(N, 3, k)).reshape(3 * N, k)


def _sqrt_blocks(D):
    """D_k^{1/2}, D_k^{-1/2} per 3x3 block and the extreme eigenvalues (eigh)."""
    lam, V = np.linalg.eigh(0.5 * (D + np.swapaxes(D, 1, 2)))
    lam = np.maximum(lam, 1e-12 * lam[:, -1:])
    Dh = np.einsum("nab,nb,ncb->nac", V, np.sqrt(lam), V)
    Dm = np.einsum("nab,nb,ncb->nac", V, 1.0 / np.sqrt(lam), V)
    return Dh, Dm, float(lam[:, 0].min()), float(lam[:, -1].max())


def certify_op(op, U, tau, rel=1e-3, tol=1e-10, plain=False, log=None):
    """Certificate at U with Q given as an operator (op.matmat, op.diag_blocks).

    The quantities of certify / certificate_bound, with every eigenvalue on
    the complement taken by scipy.sparse.linalg.eigsh (ARPACK Lanczos,
    smallest algebraic) on a LinearOperator:
      Lambda, Z = Q - blkdiag(Lambda), ||Z U^T|| (stationarity), primal and dual;
      the block-Jacobi scaled Zs = D^{-1/2} Z D^{-1/2}, D = blkdiag(Q_kk);
      W an orthonormal basis of D^{1/2} rows(U) (rows above `rel` of the
      largest singular value), a = lambda_min(W^T Zs W), the coupling
      e = ||(I - W W^T) Zs W||_F, b = lambda_min of Zs on the complement of W;
      the whole-spectrum bound (a + b)/2 - sqrt(((a - b)/2)^2 + e^2) and the
      bound on v^T Z v for unit v it implies (d_min / d_max scaling).
    On the complement the operator is P Zs P + sigma W W^T (P = I - W W^T) with
    sigma above the spectrum of Zs, so the deflated directions are not the
    smallest.  plain=True also takes lambda_min of Z itself on the orthogonal
    complement of rows(U) (the quantity of Theorem "Dual Optimality
    Certificate"; slower: the unscaled spectrum is wider)."""
    from scipy.sparse.linalg import LinearOperator, eigsh

    N = U.shape[1] // 3
    n = 3 * N
    s = mf.from_U(U)[1]
    QU = op.matmat(U.T)
    Lam = dual_lambda(None, U, s, QU=QU)
    primal = float(np.sum(U.T * QU))
    dual = float(np.trace(Lam[0]))
    ZU = QU - _blk_apply(Lam, U.T)
    D = op.diag_blocks()
    qbar = float(np.trace(D, axis1=1, axis2=2).sum()) / n
    Dh, Dm, dmin, dmax = _sqrt_blocks(D)

    def zs(x):
        y = _blk_apply(Dm, x)
        return _blk_apply(Dm, op.matmat(y) - _blk_apply(Lam, y))

    W = _orth_basis(_blk_apply(Dh, U.T), rel)
    ZW = zs(W)
    Mw = W.T @ ZW
    a = float(np.linalg.eigvalsh(0.5 * (Mw + Mw.T))[0])
    e = float(np.linalg.norm(ZW - W @ Mw))
    count = [0]

    def top(fn):
        A = LinearOperator((n, n), matvec=lambda x: (count.__setitem__(0, count[0] + 1), fn(x))[1],
                           dtype=np.float64)
        return float(eigsh(A, k=1, which="LA", tol=1e-3, return_eigenvectors=False)[0])

    sigma = 1.05 * top(zs) + 1.0

    def zc(x):
        x = x.reshape(-1)
        px = x - W @ (W.T @ x)
        y = zs(px)
        return (y - W @ (W.T @ y)) + sigma * (W @ (W.T @ x))

    A = LinearOperator((n, n), matvec=lambda x: (count.__setitem__(0, count[0] + 1), zc(x))[1],
                       dtype=np.float64)
    v0 = np.ones(n) - W @ (W.T @ np.ones(n))
    vals, vecs = eigsh(A, k=1, which="SA", tol=tol, v0=v0, ncv=40)
    b = float(vals[0])
    x = vecs[:, 0]
    res = float(np.linalg.norm(zc(x) - b * x))
    full = 0.5 * (a + b) - np.sqrt(0.25 * (a - b) ** 2 + e * e)
    out = {"primal": primal, "dual": dual, "qbar": qbar, "Lambda": Lam,
           "stat_res": float(np.linalg.norm(ZU)), "defl_min": a, "defl_cross": e,
           "lambda_min_scaled": b, "ritz_residual": res, "bound_scaled": float(full),
           "lambda_bound_full": float(full * (dmin if full >= 0 else dmax)),
           "dmin": dmin, "dmax": dmax, "deflated_rank": int(W.shape[1]), "matvecs": count[0]}
    out["certified"] = bool(out["lambda_bound_full"] >= -tau * qbar)
    if plain:
        Wp = _orth_basis(U.T, 1e-10)

        def zp(x):
            x = x.reshape(-1)
            px = x - Wp @ (Wp.T @ x)
            y = op.matmat(px) - _blk_apply(Lam, px)
            return y - Wp @ (Wp.T @ y)

        sig_p = 1.05 * top(zp) + 1.0

        def zpc(x):
            x = x.reshape(-1)
            return zp(x) + sig_p * (Wp @ (Wp.T @ x))

        Ap = LinearOperator((n, n), matvec=lambda x: (count.__setitem__(0, count[0] + 1), zpc(x))[1],
                            dtype=np.float64)
        v0 = np.ones(n) - Wp @ (Wp.T @ np.ones(n))
        out["lambda_min_plain"] = float(eigsh(Ap, k=1, which="SA", tol=tol, v0=v0, ncv=40,
                                              return_eigenvectors=False)[0])
        out["matvecs"] = count[0]
    return out
