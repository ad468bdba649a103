"""The data matrix Q (test infrastructure: oracle only).

Prop. "Scaled-Rotation-Only Formulation" and its proof (App. A) eliminate the
translations t and the landmarks p from the SBA cost (eq. sba) and leave
rho = min tr(Q U^T U).  The proof writes the cost with six matrices
Q1, Q2, Q3, V1, V2, V3, solves the stationarity condition for y = [t; p] with
frame 1 anchored (t_1 = 0), and substitutes back.

Readings of the printed proof (each one listed in the design notes):
  * the Q1 sum carries (e_i^T kron p_ik^T); the lifted keypoint u_ik is meant,
    so Q1 = blkdiag_i( sum_k w_ik u_ik u_ik^T );
  * the printed stationarity system has the opposite sign to the gradient of
    the restated quadratic; A is taken exactly as printed and the final
    formula Q = A^T Q_tp A + V_tp A + A^T V_tp^T + Q1 is consistent with that A;
  * "p_1; ...; p_{N+M}" in the definition of the reduced unknown means p_1..p_M.

Functions
---------
paper_matrices        Q1, Q2, Q3, V1, V2, V3 as sparse matrices (App. A).
q_paper_formula       Q by the paper's A-formula (dense; small scenes only).
q_block_elimination   Q by eliminating p (Q3 diagonal) and then t (frame 0
                      grounded), using the same matrices; any size that fits.
recover_tp            [t; p] = (A kron I3) vec(U)   (eq. tpstar), any r.
sba_cost              the SBA objective of eq. sba evaluated directly.
brute_force_cost      min over t, p of the SBA cost for fixed U by least squares.
q_rows                selected rows of Q (sparse elimination, any size).
sparse_parts          A_rr, A_rt, A_tt kept sparse (landmarks eliminated).
QOperator             Q V without forming Q (sparse parts + one Cholesky of
                      the grounded Laplacian); its diagonal blocks; tr(Q U^T U).
recover_tp_sparse     eq. tpstar with the sparse parts.
sba_cost_at           min over t, p of the SBA cost at fixed U, evaluated from
                      the per-observation residuals (any size).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def paper_matrices(N, M, frame, landmark, u, w):
    """Q1 (3N x 3N), Q2 (N x N), Q3 (M x M), V1 (3N x N), V2 (3N x M), V3 (N x M).

    Definitions of App. A with e_i, ebar_k the unit vectors of frames and
    landmarks; the Kronecker products (e_i kron u) place u in rows 3i..3i+2."""
    n = frame.shape[0]
    fr = frame.astype(np.int64)
    lm = landmark.astype(np.int64)
    rows3 = (3 * fr[:, None] + np.arange(3)[None, :])            # [n, 3]
    # Q1 = sum w (e_i kron u)(e_i^T kron u^T)
    r1 = np.repeat(rows3, 3, axis=1).ravel()
    c1 = np.tile(rows3, (1, 3)).ravel()
    v1 = (w[:, None, None] * u[:, :, None] * u[:, None, :]).ravel()
    Q1 = sp.coo_matrix((v1, (r1, c1)), shape=(3 * N, 3 * N)).tocsr()
    Q2 = sp.coo_matrix((w, (fr, fr)), shape=(N, N)).tocsr()
    Q3 = sp.coo_matrix((w, (lm, lm)), shape=(M, M)).tocsr()
    wu = (w[:, None] * u).ravel()
    V1 = sp.coo_matrix((wu, (rows3.ravel(), np.repeat(fr, 3))), shape=(3 * N, N)).tocsr()
    V2 = sp.coo_matrix((wu, (rows3.ravel(), np.repeat(lm, 3))), shape=(3 * N, M)).tocsr()
    V3 = sp.coo_matrix((w, (fr, lm)), shape=(N, M)).tocsr()
    return Q1, Q2, Q3, V1, V2, V3


def q_paper_formula(N, M, frame, landmark, u, w):
    """Q = A^T Q_tp A + V_tp A + A^T V_tp^T + Q1 with the printed A (App. A).

    Q_tp = [[Q2, -V3], [-V3^T, Q3]] (the view-graph Laplacian, Lemma
    "laplacian"), V_tp = [-V1, V2], Qbar_tp = Q_tp without its first column
    (t_1 = 0), A = [0_{1 x 3N}; -(Qbar^T Qbar)^{-1} Qbar^T V_tp^T].
    Dense; meant for N + M up to a few thousand."""
    Q1, Q2, Q3, V1, V2, V3 = paper_matrices(N, M, frame, landmark, u, w)
    Qtp = sp.bmat([[Q2, -V3], [-V3.T, Q3]]).toarray()
    Vtp = sp.hstack([-V1, V2]).toarray()
    Qbar = Qtp[:, 1:]
    Abar = -np.linalg.solve(Qbar.T @ Qbar, Qbar.T @ Vtp.T)
    A = np.vstack([np.zeros((1, 3 * N)), Abar])
    Q = A.T @ Qtp @ A + Vtp @ A + A.T @ Vtp.T + Q1.toarray()
    return 0.5 * (Q + Q.T)


def block_parts(N, M, frame, landmark, u, w):
    """Eliminate the landmarks: Schur complement of the diagonal block Q3.

    With the full quadratic [r; t; p]^T [[Q1, V1, -V2], [V1^T, Q2, -V3],
    [-V2^T, -V3^T, Q3]] [r; t; p] (App. A), removing p gives
        A_rr = Q1 - V2 Q3^-1 V2^T,  A_rt = V1 - V2 Q3^-1 V3^T,
        A_tt = Q2 - V3 Q3^-1 V3^T   (the frame co-visibility Laplacian).
    Returned dense (A_rr 3N x 3N, A_rt 3N x N, A_tt N x N)."""
    Q1, Q2, Q3, V1, V2, V3 = paper_matrices(N, M, frame, landmark, u, w)
    q3 = Q3.diagonal()
    inv = sp.diags(np.where(q3 > 0, 1.0 / np.where(q3 > 0, q3, 1.0), 0.0))
    A_rr = (Q1 - V2 @ inv @ V2.T).toarray()
    A_rt = (V1 - V2 @ inv @ V3.T).toarray()
    A_tt = (Q2 - V3 @ inv @ V3.T).toarray()
    return A_rr, A_rt, A_tt


def q_block_elimination(N, M, frame, landmark, u, w, return_parts=False):
    """Q = A_rr - A_rt[:,1:] A_tt[1:,1:]^{-1} A_rt[:,1:]^T (translations out, t_1 = 0).

    Same Q as q_paper_formula (block Gaussian elimination of the same
    quadratic, p first because Q3 is diagonal); the grounded Laplacian
    A_tt[1:,1:] is SPD for a connected view graph (Lemma "laplacian")."""
    A_rr, A_rt, A_tt = block_parts(N, M, frame, landmark, u, w)
    G = A_tt[1:, 1:]
    B = A_rt[:, 1:]
    cf = sla.cho_factor(G, lower=True)
    Q = A_rr - B @ sla.cho_solve(cf, B.T)
    Q = 0.5 * (Q + Q.T)
    if return_parts:
        return Q, (A_rr, A_rt, A_tt)
    return Q


def q_rows(N, M, frame, landmark, u, w, rows):
    """Selected rows of Q, for scenes too large for the dense constructions.

    Same block elimination as q_block_elimination, kept sparse: A_rr, A_rt
    and A_tt from the paper's matrices, then
    Q[rows, :] = A_rr[rows, :] - (A_tt[1:,1:]^{-1} A_rt[rows, 1:]^T)^T A_rt[:, 1:]^T
    with one dense Cholesky of the grounded Laplacian (N - 1 squared)."""
    Q1, Q2, Q3, V1, V2, V3 = paper_matrices(N, M, frame, landmark, u, w)
    q3 = Q3.diagonal()
    inv = sp.diags(np.where(q3 > 0, 1.0 / np.where(q3 > 0, q3, 1.0), 0.0))
    rows = np.asarray(rows)
    V2r = V2[rows]
    A_rr_rows = (Q1[rows] - V2r @ inv @ V2.T).toarray()
    A_rt = (V1 - V2 @ inv @ V3.T).tocsr()
    A_tt = (Q2 - V3 @ inv @ V3.T).toarray()
    cf = sla.cho_factor(A_tt[1:, 1:], lower=True)
    B = A_rt[:, 1:]
    X = sla.cho_solve(cf, B[rows].toarray().T)          # (N-1) x |rows|
    return A_rr_rows - (B @ X).T


def recover_tp(N, M, frame, landmark, u, w, Y):
    """[t; p] for a given U (r x 3N): eq. tpstar, solved blockwise.

    Returns t (N x r) and p (M x r): rows are the r coordinates, so for r = 3
    t[i] is t_i and p[k] is p_k.  t_0 = 0 (anchor)."""
    Q1, Q2, Q3, V1, V2, V3 = paper_matrices(N, M, frame, landmark, u, w)
    A_rr, A_rt, A_tt = block_parts(N, M, frame, landmark, u, w)
    r = Y.shape[0]
    # stationarity in t (p eliminated): A_tt t = -A_rt^T Y^T (columns = coords)
    rhs = -(A_rt.T @ Y.T)                           # N x r
    t = np.zeros((N, r))
    t[1:] = sla.cho_solve(sla.cho_factor(A_tt[1:, 1:], lower=True), rhs[1:])
    # stationarity in p: Q3 p = V3^T t + V2^T vec  (p_k = weighted mean of Y_i u + t_i)
    q3 = Q3.diagonal()
    p = (V3.T @ t + V2.T @ Y.T) / np.where(q3 > 0, q3, 1.0)[:, None]
    return t, p


def sba_cost(frame, landmark, u, w, Y, t, p):
    """sum w_ik || Y_i u_ik + t_i - p_k ||^2   (eq. sba with Y_i = s_i R_i, any r).

    Y is r x 3N, t is N x r, p is M x r."""
    N = Y.shape[1] // 3
    Yb = Y.reshape(Y.shape[0], N, 3).transpose(1, 0, 2)          # N x r x 3
    e = np.einsum("nab,nb->na", Yb[frame], u) + t[frame] - p[landmark]
    return float(np.sum(w * np.sum(e * e, axis=1)))


def brute_force_cost(N, M, frame, landmark, u, w, Y):
    """min_{t, p; t_0 = 0} of the SBA cost at fixed U, by dense least squares.

    Independent of every formula above: builds the residual operator of eq. sba
    row by row and calls numpy.linalg.lstsq.  Tiny scenes only."""
    n = frame.shape[0]
    r = Y.shape[0]
    N_t = N - 1
    nvar = N_t + M
    A = np.zeros((n, nvar))
    sw = np.sqrt(w)
    for o in range(n):
        i, k = frame[o], landmark[o]
        if i > 0:
            A[o, i - 1] = sw[o]
        A[o, N_t + k] = -sw[o]
    total = 0.0
    Yb = Y.reshape(r, N, 3).transpose(1, 0, 2)
    for a in range(r):
        b = -sw * np.einsum("nb,nb->n", Yb[frame, a, :], u)
        sol, *_ = np.linalg.lstsq(A, b, rcond=None)
        res = A @ sol - b
        total += float(res @ res)
    return total


# ---------------------------------------------------------------------------
# Matrix-free forms for scenes whose dense Q does not fit (tens of thousands of
# rows): the same block elimination, with A_rr, A_rt, A_tt kept sparse and the
# grounded Laplacian factored once.

def sparse_parts(N, M, frame, landmark, u, w):
    """A_rr (3N x 3N), A_rt (3N x N), A_tt (N x N) as scipy CSR matrices:
    the landmark elimination of block_parts, without densifying."""
    Q1, Q2, Q3, V1, V2, V3 = paper_matrices(N, M, frame, landmark, u, w)
    q3 = Q3.diagonal()
    inv = sp.diags(np.where(q3 > 0, 1.0 / np.where(q3 > 0, q3, 1.0), 0.0))
    A_rr = (Q1 - V2 @ inv @ V2.T).tocsr()
    A_rt = (V1 - V2 @ inv @ V3.T).tocsr()
    A_tt = (Q2 - V3 @ inv @ V3.T).tocsr()
    return A_rr, A_rt, A_tt


class QOperator:
    """Q V = A_rr V - B (G^{-1} (B^T V)),  B = A_rt[:, 1:],  G = A_tt[1:, 1:].

    The formula of q_block_elimination applied to a block of vectors instead
    of formed: one dense Cholesky of the grounded Laplacian (N - 1 squared),
    sparse products with A_rr and B.  Exact up to rounding order."""

    def __init__(self, N, M, frame, landmark, u, w):
        self.N, self.M = N, M
        self.A_rr, self.A_rt, self.A_tt = sparse_parts(N, M, frame, landmark, u, w)
        self.B = self.A_rt[:, 1:].tocsr()
        self.Bt = self.B.T.tocsr()
        self.cf = sla.cho_factor(self.A_tt[1:, 1:].toarray(), lower=True, overwrite_a=True)
        self.n = 3 * N
        self._diag = None

    def matmat(self, V):
        """Q V for V of shape (3N,) or (3N, k)."""
        return self.A_rr @ V - self.B @ sla.cho_solve(self.cf, self.Bt @ V)

    def trace(self):
        """tr(Q) = sum of the diagonal 3x3 blocks."""
        return float(sum(np.trace(b) for b in self.diag_blocks()))

    def diag_blocks(self):
        """Q_kk [N, 3, 3]: A_rr's diagonal block minus B_k G^{-1} B_k^T, B_k the
        three rows of frame k (sparse), with G^{-1} from the Cholesky factor."""
        if self._diag is None:
            import scipy.linalg.lapack as lap
            L = np.tril(self.cf[0])
            Ginv, info = lap.dpotri(L, lower=1)
            assert info == 0
            Ginv = np.tril(Ginv) + np.tril(Ginv, -1).T
            D = np.empty((self.N, 3, 3))
            ip, ix, dv = self.B.indptr, self.B.indices, self.B.data
            C = self.A_rr.tocoo()
            on = (C.row // 3) == (C.col // 3)
            Arr = np.zeros((self.N, 3, 3))
            np.add.at(Arr, (C.row[on] // 3, C.row[on] % 3, C.col[on] % 3), C.data[on])
            for k in range(self.N):
                lo, hi = ip[3 * k], ip[3 * k + 3]
                cols, pos = np.unique(ix[lo:hi], return_inverse=True)
                Bd = np.zeros((3, cols.size))
                rows = np.repeat(np.arange(3), np.diff(ip[3 * k:3 * k + 4]))
                np.add.at(Bd, (rows, pos), dv[lo:hi])
                D[k] = Arr[k] - Bd @ Ginv[np.ix_(cols, cols)] @ Bd.T
                D[k] = 0.5 * (D[k] + D[k].T)
            self._diag = D
        return self._diag

    def cost(self, U):
        """tr(Q U^T U) = sum over rows y of U of y Q y^T."""
        return float(np.sum(U.T * self.matmat(U.T)))


def recover_tp_sparse(op, frame, landmark, u, w, Y):
    """eq. tpstar with the sparse parts (any size): t from the grounded
    Laplacian, t_0 = 0, then each landmark the weighted mean of Y_i u + t_i.
    Returns t (N x r), p (M x r)."""
    r = Y.shape[0]
    N, M = op.N, op.M
    rhs = -(op.A_rt.T @ Y.T)
    t = np.zeros((N, r))
    t[1:] = sla.cho_solve(op.cf, rhs[1:])
    Yb = Y.reshape(r, N, 3).transpose(1, 0, 2)
    x = np.einsum("nab,nb->na", Yb[frame], u) + t[frame]         # Y_i u + t_i per observation
    W = np.bincount(landmark, weights=w, minlength=M)
    p = np.stack([np.bincount(landmark, weights=w * x[:, a], minlength=M) for a in range(r)], axis=1)
    p = p / np.where(W > 0, W, 1.0)[:, None]
    return t, p


def sba_cost_at(op, frame, landmark, u, w, Y):
    """min over t, p (t_0 = 0) of the SBA cost at fixed U = Y (eq. sba),
    evaluated from the residuals of every observation at the minimiser of
    eq. tpstar.  Equals tr(Q Y^T Y) (Prop. "Scaled-Rotation-Only Formulation");
    the two are computed by different routes."""
    t, p = recover_tp_sparse(op, frame, landmark, u, w, Y)
    return sba_cost(frame, landmark, u, w, Y, t, p)
