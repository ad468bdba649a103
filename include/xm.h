/*
 * xm.h -- C ABI of the MI355X (gfx950) XM library.
 *
 * Solves scaled bundle adjustment (SBA, eq. sba of Han & Yang, "Building Rome
 * with Convex Optimization", arXiv 2502.04640) to certified global optimality:
 *
 *   xm_build_Q   eliminate translations and landmarks in closed form and
 *                assemble the 3N x 3N rotation-only data matrix Q
 *                (Prop. "Scaled-Rotation-Only Formulation", App. A);
 *   xm_bm_solve  Burer-Monteiro factorisation of the SDP relaxation
 *                (Prop. "SDP Relaxation", Prop. "BM Factorization") solved by
 *                the Riemannian staircase (Algorithm "Riemannian Staircase")
 *                with a trust-region / truncated-CG local optimiser
 *                (Prop. "BM Riemannian Optimization");
 *   xm_certify   dual certificate Z = Q - blkdiag(Lambda) and its minimum
 *                eigenvalue (Theorem "Dual Optimality Certificate");
 *   xm_round     rounding of the low-rank factor to anchored scaled rotations
 *                and the suboptimality gap (eq. suboptimality).
 *
 * Conventions (all entry points):
 *  - Every pointer argument named "device" is GPU memory owned by the caller
 *    (for example torch.Tensor.data_ptr()).  Host pointers are marked "host".
 *  - `stream` is a hipStream_t passed as void*.  Work is enqueued on it; the
 *    entry points that return scalars (info structs) synchronise that stream
 *    before returning.  NULL means the default stream.
 *  - Indices are 0-based.  Frame 0 is the anchor (the paper's frame 1:
 *    R = I, t = 0, s = 1, Section "Anchoring").
 *  - A low-rank factor Y (the paper's U) is a device array of doubles,
 *    row-major [r][3N]: column 3k+c of row a is (s_k R_k)[a][c] for the r x 3
 *    Stiefel block R_k of frame k.
 *  - Rotations are returned row-major [N][3][3] in the SBA camera->world
 *    convention (footnote to eq. sba): R_i (s_i u_ik) + t_i = p_k.
 *  - Return value: XM_OK (0) or a negative xm_status; xm_last_error() then
 *    gives a message (thread-local, valid until the next call on the thread).
 *    On XM_EINVAL / XM_EGRAPH no output has been written.
 *  - The library is not re-entrant on one problem handle: calls that use the
 *    same handle must be serialised by the caller.
 */
#ifndef XM_H_
#define XM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  XM_OK = 0,
  XM_EINVAL = -1,   /* bad argument: sizes, NaN/Inf keypoint, weight <= 0, index out of range */
  XM_ENOMEM = -2,   /* device allocation failed */
  XM_EHIP = -3,     /* a HIP runtime call failed */
  XM_EGRAPH = -4,   /* a frame without observations, or a disconnected view graph */
  XM_ENOCONV = -5   /* iteration cap reached; outputs hold the last iterate */
} xm_status;

typedef enum { XM_F64 = 0, XM_F32 = 1, XM_BF16 = 2 } xm_dtype;

/* Opaque problem handle: device-resident Q (FP64 master and optional FP32 /
 * BF16 copies) plus the workspaces of the solver.  Owned by the library,
 * released with xm_free. */
typedef struct xm_problem xm_problem;

/* Bits of `copies` in xm_build_Q. */
#define XM_KEEP_F32 (1u << 1)
#define XM_KEEP_BF16 (1u << 2)

/*
 * Assemble Q from the observations of the view graph.
 *
 * Operation (Prop. "Scaled-Rotation-Only Formulation", App. A): the SBA cost
 * sum_{(i,k)} w_ik || R_i (s_i u_ik) + t_i - p_k ||^2 is minimised over the
 * landmarks p_k and translations t_i (t_0 = 0) in closed form, leaving
 * tr(Q U^T U).  The landmarks are eliminated per landmark (Schur complement
 * of the diagonal landmark block), the translations by the inverse of the
 * grounded frame Laplacian.  Q is built in FP64.
 *
 * N        number of frames (>= 2, < 65536)
 * M        number of landmarks (>= 1); landmark ids lie in [0, M)
 * n_obs    number of observations (>= 1, < 2^31)
 * frame    device int32 [n_obs], frame index of each observation
 * landmark device int32 [n_obs], landmark index of each observation
 * u        device [n_obs][3] lifted keypoints u_ik (eq. 3D-lifting), dtype u_dtype
 * u_dtype  XM_F64 or XM_F32
 * w        device [n_obs] weights w_ik > 0, dtype w_dtype, or NULL for all ones
 * w_dtype  XM_F64 or XM_F32 (ignored when w is NULL)
 * copies   XM_KEEP_F32 | XM_KEEP_BF16: reduced-precision copies of Q to keep
 *          for xm_bm_solve with compute = XM_F32 / XM_BF16
 * stream   hipStream_t
 * out      host: receives the new handle
 *
 * Observations may come in any order; a landmark seen once contributes
 * nothing.  Errors: XM_EINVAL (sizes, index out of range, non-finite u,
 * w <= 0), XM_EGRAPH (frame without observations, disconnected graph).
 * Synchronises `stream`.  The inversion of the grounded Laplacian also uses a
 * private second stream (default priority), ordered against `stream` by
 * events and finished before the call returns.
 */
xm_status xm_build_Q(int32_t N, int32_t M, int64_t n_obs, const int32_t* frame,
                     const int32_t* landmark, const void* u, xm_dtype u_dtype,
                     const void* w, xm_dtype w_dtype, uint32_t copies, void* stream,
                     xm_problem** out);

/*
 * xm_build_Q on the observations whose mask byte is nonzero (mask: device
 * uint8 [n_obs], or NULL for all): the rebuild step of the XM^2 loop
 * (Section "Structure from Motion with XM": after the first solve, the
 * measurements with the largest residuals are deleted and the solver runs
 * again).  Every input array keeps its full length n_obs; observations with
 * mask 0 are validated but left out of Q.  Per-observation outputs of the
 * handle (xm_residuals, xm_adjoint) keep the caller's full indexing and give 0
 * for the left-out observations.  Errors as xm_build_Q, plus XM_EINVAL when the
 * mask keeps nothing; XM_EGRAPH when what is kept leaves a frame without a
 * shared landmark or the view graph disconnected.
 */
xm_status xm_build_Q_masked(int32_t N, int32_t M, int64_t n_obs, const int32_t* frame,
                            const int32_t* landmark, const void* u, xm_dtype u_dtype, const void* w,
                            xm_dtype w_dtype, const uint8_t* mask, uint32_t copies, void* stream,
                            xm_problem** out);

/* Release a handle and all device memory it owns.  NULL is allowed.  The
 * memory goes back to the library's device pool (below), not to the runtime. */
void xm_free(xm_problem* p);

/*
 * Device memory of the library.  Every buffer the library allocates (problem
 * handles, solver and certificate workspaces) comes from a per-device pool:
 * freed blocks are kept and handed out again to requests of about the same
 * size (at most 1.25x), so repeated builds and solves of one problem shape take
 * no memory from the runtime after the first.  A freed block is recycled only
 * after the device has finished its queued work (the ordering hipFree gives).
 * Cached blocks are capped at 64 GiB over all devices (environment variable
 * XM_POOL_CACHE_GB overrides; the largest are released first); an allocation
 * that fails releases the device's cached blocks and retries once.
 *
 * xm_memory_info  bytes in live blocks and in cached (free) blocks, over all
 *                 devices (host outputs; either may be NULL, not both).
 * xm_memory_trim  wait for the devices to go idle and release every cached
 *                 block to the runtime; returns the bytes released.
 */
xm_status xm_memory_info(int64_t* live_bytes, int64_t* cached_bytes);
int64_t xm_memory_trim(void);

typedef struct {
  int32_t N, M;
  int64_t n_obs;         /* observations in Q (those the mask kept) */
  int64_t n_in;          /* observations passed in (the length of per-observation outputs) */
  int64_t nnz_blocks;    /* co-visibility blocks (frame pairs sharing a landmark, incl. diagonal) */
  int64_t n_pairs;       /* per-landmark observation pairs reduced into the blocks */
  int32_t ld;            /* leading dimension (elements) of the dense row-major Q copies */
  int32_t copies;        /* bitmask: 1 (FP64) | XM_KEEP_F32 | XM_KEEP_BF16 */
  double qbar;           /* tr(Q) / 3N, the scale used by the relative tolerances */
  double build_ms;       /* device time of the last xm_build_Q, milliseconds */
  double scale_reg;      /* lambda of xm_set_scale_reg (0: the plain objective) */
} xm_problem_info;

/*
 * Scale regularisation (App. "Scale Regularization", eq. problem-sdp-scale):
 * the objective becomes tr(Q X) + lambda sum_{i>=2} (X_{3i,3i} - 1)^2, which
 * keeps the scales of frames 2..N from collapsing toward 0 on data where the
 * plain optimum shrinks them.  On the Burer-Monteiro manifold the term is
 * lambda sum_{k>=1} (s_k^2 - 1)^2.  Applies to every later xm_bm_solve,
 * xm_certify (Z = Q + grad F(X) - blkdiag(Lambda); primal tr(QX) + F(X); dual
 * tr(Lambda_0) + F(X) - <grad F(X), X>) and xm_round (rho_hat includes F) on
 * the handle.  xm_adjoint refuses a regularised handle (XM_EINVAL).  lambda
 * must be finite and >= 0 (0 restores the plain objective).
 */
xm_status xm_set_scale_reg(xm_problem* p, double lambda);

/* Fill `info` (host) for a handle. */
xm_status xm_get_info(const xm_problem* p, xm_problem_info* info);

/*
 * Device time of the main kernels of the handle's xm_build_Q (HIP events on
 * the build stream around every launch): the Laplacian inversion's trailing
 * update and the two sparse-dense products of the translation elimination.
 * `bytes` and `flops` are algorithmic totals over all launches (unique HBM
 * bytes the kernel must move; FP64 flops).  Up to `cap` entries are written to
 * `out` (host); *count receives the number available.
 */
typedef struct {
  char name[40];
  int32_t launches;
  double total_ms;
  double bytes;
  double flops;
} xm_kernel_stat;
xm_status xm_build_stats(const xm_problem* p, xm_kernel_stat* out, int32_t cap, int32_t* count);

/*
 * Copy rows [row0, row0 + nrows) of the FP64 Q into `out` (device, row-major
 * [nrows][3N]), rows and columns in frame-index order (the library stores Q
 * with its frames in a Cuthill-McKee order of the co-visibility graph and
 * gathers the rows back).  For checks against a reference.  Synchronises
 * `stream`.
 */
xm_status xm_get_Q_rows(const xm_problem* p, int32_t row0, int32_t nrows, double* out,
                        void* stream);

/*
 * Y Q product with the stored Q of precision `dtype` (XM_F64 / XM_F32 /
 * XM_BF16 copy): out[a][j] = sum_i Y[a][i] Q[i][j] for a < r, the block-
 * sparse product of the local solver (Euclidean gradient Gamma = 2 Y Q,
 * Section "C++/CUDA-based Riemannian Optimization").  Y and out are device
 * [r][3N] doubles, 1 <= r <= 8.  Accumulation is FP64 for XM_F64 and FP32
 * otherwise.  Exposed for measurement and checks.
 */
xm_status xm_spmm(xm_problem* p, xm_dtype dtype, const double* Y, int32_t r, double* out,
                  void* stream);

/*
 * The product of xm_spmm for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, kernels and result (bitwise) as xm_spmm, with
 * every temporary taken from a fixed device array of the library
 * (XM_NOALLOC_SCRATCH_MIB MiB per GPU, held from the library's first use on
 * that GPU until the process ends) instead of the handle's buffers.  It calls
 * no hipMalloc / hipFree and does not synchronise: the work is enqueued on
 * `stream` and `out` is ready when the stream reaches that point.  Every call
 * on one GPU uses the same array, so calls that may overlap on a GPU (other
 * streams, other threads) race and must be serialised by the caller.  The
 * handle's kernel choice for residual products of `dtype` applies
 * (xm_set_product_kind).  Errors: XM_EINVAL for a NULL argument, r outside
 * [1, 8], an unknown dtype, a precision the handle did not keep, or a product
 * whose temporaries exceed the array (xm_spmm_noalloc_bytes tells the need);
 * nothing is enqueued then.  HIP event timing (xm_spmm_timing) does not see
 * these products.
 */
#define XM_NOALLOC_SCRATCH_MIB 128
xm_status xm_spmm_noalloc(xm_problem* p, xm_dtype dtype, const double* Y, int32_t r, double* out,
                          void* stream);
/* Bytes of the fixed array that xm_spmm_noalloc(p, dtype, ., r, ...) needs
 * (host output `bytes`); XM_EINVAL for bad arguments. */
xm_status xm_spmm_noalloc_bytes(const xm_problem* p, xm_dtype dtype, int32_t r, int64_t* bytes);

/*
 * Which kernel computes the Y Q product for the stored Q of precision `dtype`
 * (every product on the handle: solver, certificate, xm_spmm).  Q is
 * symmetric, so the product can be formed from the upper triangle alone:
 *   XM_SPMM_FULL   every element of Q is read once ((3N)^2 elements);
 *   XM_SPMM_UPPER  only Q[i][j], j >= i, is read (3N(3N+1)/2 elements), each
 *                  feeding both out[j] and out[i]: half the HBM bytes, with
 *                  twice the arithmetic per byte and a cross-lane reduction.
 *   XM_SPMM_FACTORED (FP64, FP32)  Q is not read at all: Q Y^T is formed from
 *                  the factors of its elimination, Q = A_rr - A_rt' G^{-1} A_rt'^T
 *                  (App. A; A_rt' = A_rt without the anchored frame's column,
 *                  G the grounded Laplacian), as A_rr Y^T (sparse 3x3 blocks
 *                  on the co-visibility pattern) - A_rt' (G^{-1} (A_rt'^T Y^T))
 *                  with the dense symmetric G^{-1} read through its upper
 *                  triangle: (N-1)N/2 + 15 nnz(blocks) values per product
 *                  instead of 3N(3N+1)/2.  The paper names sparse products as
 *                  its future work.  The two terms cancel near the optimum
 *                  (A_rr Y^T is up to ~30x larger than Q Y^T there), so the
 *                  factored form carries that much more rounding: fine in FP64
 *                  for products of directions, not for the residual at the
 *                  iterate (an FP64 solve then stalls near 1e-7 relative
 *                  gradient).  FP32 (needs XM_KEEP_F32, which also keeps FP32
 *                  factors) reaches ~1e-3 relative error on a 2000-frame loop:
 *                  too coarse for residuals, usable for the curvature of a
 *                  trust-region model, whose steps are accepted on the
 *                  residual-role cost.  No BF16 form.
 * All are deterministic; their results differ by rounding order only.
 */
typedef enum { XM_SPMM_FULL = 0, XM_SPMM_UPPER = 1, XM_SPMM_FACTORED = 2 } xm_spmm_kind;
/* Products play two roles.  XM_ROLE_RESIDUAL: Y Q at the iterate itself
 * (cost, gradient, multipliers, xm_spmm), whose entries cancel heavily near
 * the optimum, so they need the most accurate form.  XM_ROLE_CURVATURE:
 * products of directions (Hessian-vector products of truncated CG and of the
 * adjoint, Lanczos steps of the certificate).  Defaults: residual products
 * XM_SPMM_UPPER (FP64, FP32) / XM_SPMM_FULL (BF16); curvature products
 * XM_SPMM_FACTORED for FP64; for FP32, XM_SPMM_FACTORED once the stored
 * upper triangle of the FP32 Q (3N(3N+1)/2 values) exceeds 256 MiB, the
 * GPU's last-level cache, below which the dense read stays cache-resident
 * across products and XM_SPMM_UPPER is the default; BF16 as its residual. */
typedef enum { XM_ROLE_RESIDUAL = 0, XM_ROLE_CURVATURE = 1 } xm_product_role;
/* xm_set_spmm_kind sets the kernel of both roles; xm_set_product_kind of one;
 * xm_get_product_kind reads the kernel in use (the defaults above are set by
 * xm_build_Q).  XM_EINVAL for an unknown role, dtype or kernel, a NULL
 * argument, or a BF16 factored product. */
xm_status xm_set_spmm_kind(xm_problem* p, xm_dtype dtype, xm_spmm_kind kind);
xm_status xm_set_product_kind(xm_problem* p, xm_product_role role, xm_dtype dtype, xm_spmm_kind kind);
xm_status xm_get_product_kind(const xm_problem* p, xm_product_role role, xm_dtype dtype, xm_spmm_kind* kind);

typedef struct {
  int32_t r0;          /* initial rank (>= 3); the staircase starts here */
  int32_t r_max;       /* maximum rank (r0 <= r_max <= 7) */
  double lift;         /* start point when Y0 is NULL: U^0 = [I, ..., I] padded
                          with zero rows (the paper's initialisation) perturbed
                          by a seeded uniform [-lift, lift] and re-orthonormalised
                          per block; 0 gives the paper's U^0 exactly */
  xm_dtype compute;    /* XM_F64: FP64 everywhere; XM_F32: FP32 products and
                          manifold arithmetic, then the FP64 stage (grad_tol);
                          XM_BF16: as XM_F32 with the BF16-stored Q for the
                          first stage's Hessian products */
  double grad_tol;     /* stop when ||grad|| <= grad_tol * qbar * ||Y||_F
                          (<= 0: 1e-9 for XM_F64, 1e-6 otherwise); a stage
                          also stops at the arithmetic's floor (6 consecutive
                          rejected trust-region steps while ||grad|| <= 30
                          grad_tol * qbar * ||Y||_F, or 12 at any gradient).
                          XM_F32 / XM_BF16 solves then continue in an FP64
                          stage (FP64 iterate, manifold arithmetic and
                          gradient products; truncated-CG products with the
                          FP32 Q) down to grad_tol / 1000.  A point whose
                          certificate fails only through the stationarity
                          terms of its bound is polished at the same rank
                          (up to 3 times; FP64 Hessian products) to the
                          reached |g| times (cert tol qbar / 2|bound|)^(1/k),
                          k in [1, 2] fitted to the bound's fall with |g|
                          (2 at first), and at least 10x below the previous
                          tolerance.  The
                          FP64 stage exists because the dual certificate needs
                          a point closer to stationary than a reduced-precision
                          iterate's own rounding allows */
  double cert_tol;     /* certified iff the lower bound on lambda_min(Z) >= -cert_tol * qbar
                          (<= 0: 1e-7 for XM_F64, 1e-5 otherwise) */
  int32_t max_outer;   /* trust-region iterations per rank (<= 0: 1000) */
  int32_t max_inner;   /* truncated-CG iterations per outer step (<= 0: 3N*r) */
  double delta0;       /* initial trust radius (<= 0: sqrt(3N)/8) */
  int32_t lanczos_max; /* Lanczos iterations per certificate (<= 0: 400) */
  double lanczos_tol;  /* Ritz residual tolerance relative to qbar (<= 0: 1e-6) */
  int32_t precondition;/* 1: per-frame diagonal preconditioner in truncated CG */
  int32_t verbose;     /* 1: one line per outer iteration on stderr */
} xm_solve_opts;

/* Fill `opts` with the defaults: compute = XM_F64, r0 = 5, r_max = 7,
 * lift = 1 (a lifted start; set r0 = 3, lift = 0 for the paper's U^0),
 * precondition = 1, every other field 0 (= the documented default). */
void xm_default_opts(xm_solve_opts* opts);

typedef struct {
  int32_t r;             /* final rank */
  int32_t certified;     /* 1 if the final certificate holds */
  int32_t outer_iters;   /* trust-region iterations, all ranks */
  int32_t inner_iters;   /* truncated-CG iterations, all ranks */
  int32_t stair_steps;   /* rank increases taken */
  int32_t spmm_count;    /* Y Q products in the solve (excluding the certificate) */
  int32_t lanczos_iters; /* Lanczos iterations, all certificates */
  int32_t converged;     /* 1 if the gradient tolerance was met at the final rank,
                            2 if the solve stopped at the precision floor (grad_tol) */
  double cost;           /* f = tr(Q Y^T Y), FP64 */
  double grad_norm;      /* final Riemannian gradient norm from FP64 products */
  double lambda_min;     /* lower bound on the minimum eigenvalue of Z at the final
                            point (xm_cert.lambda_bound of the last certificate) */
  double primal, dual;   /* tr(Q Y^T Y) and tr(Lambda_0) */
  double solve_ms;       /* wall time of the local solves, milliseconds */
  double cert_ms;        /* wall time of the certificates, milliseconds */
} xm_solve_info;

/*
 * Riemannian staircase (Algorithm "Riemannian Staircase").
 *
 * Y0     device [r_in][3N] initial factor (feasible: Y0_k^T Y0_k = alpha_k I,
 *        alpha_0 = 1), or NULL for U^0 = [I, ..., I] at rank opts->r0.
 * r_in   rank of Y0 (ignored when Y0 is NULL).
 * Y_out  device [opts->r_max][3N]; rows [0, info->r) hold the solution, the
 *        rest are zero.
 * info   host, filled on return.
 * Returns XM_OK, or XM_ENOCONV if an iteration cap or a stagnation stopped the
 * final local solve short of its tolerance and the point is not certified
 * (Y_out still holds the last iterate).  Synchronises `stream`.
 */
xm_status xm_bm_solve(xm_problem* p, const xm_solve_opts* opts, const double* Y0, int32_t r_in,
                      double* Y_out, xm_solve_info* info, void* stream);

typedef struct {
  double lambda_min;     /* smallest Ritz value of the block-Jacobi scaled dual
                            Zs = D^{-1/2} Z D^{-1/2} (D = blkdiag(Q_kk)) on the
                            complement of D^{1/2} rows(Y) */
  double ritz_residual;  /* residual norm of the Ritz pair of lambda_min */
  double lambda_bound;   /* lower bound on v^T Z v over ALL unit v:
                            b * (d_min if b >= 0 else d_max), d_min/d_max the
                            extreme eigenvalues of the Q_kk, with
                            b = (a + c)/2 - sqrt(((a - c)/2)^2 + e^2),
                            c = lambda_min - ritz_residual, a = defl_min,
                            e = defl_cross; exact given that Lanczos found the
                            smallest eigenvalue on the complement */
  double primal;         /* tr(Q Y^T Y), the relaxation's value at Y (rho_SDP) */
  double dual;           /* tr(Lambda_0), the dual objective b^T y */
  double qbar;           /* tr(Q) / 3N */
  double grad_norm;      /* || Z Y^T ||_F, the stationarity residual */
  double defl_min;       /* smallest eigenvalue of W^T Zs W, W an orthonormal basis
                            of D^{1/2} rows(Y) (0 at a critical point) */
  double defl_cross;     /* || (I - W W^T) Zs W ||_F (0 at a critical point) */
  double rho_hat;        /* cost tr(Q Uhat^T Uhat) of the rounded point (xm_round);
                            NaN when r < 3 */
  double eta;            /* eq. suboptimality: (rho_hat - primal) /
                            (1 + |rho_hat| + |primal|); NaN when r < 3 */
  int32_t certified;     /* lambda_bound >= -tol * qbar */
  int32_t iters;         /* Lanczos iterations */
} xm_cert;

/*
 * Dual certificate at Y (Theorem "Dual Optimality Certificate").
 * Lambda_k = sym((Q Y^T)_k Y_k) / alpha_k (traceless for k >= 1),
 * Z = Q - blkdiag(Lambda).  PSD-ness of Z is decided by FP64 Lanczos with full
 * reorthogonalisation on the congruent D^{-1/2} Z D^{-1/2} (same inertia,
 * narrower spectrum), deflated against D^{1/2} rows(Y), with the deflated block
 * and its coupling to the complement folded into a bound on the whole spectrum
 * (so a Y that is not a critical point is not certified by its complement
 * alone); certified iff lambda_bound >= -tol * qbar.  Also rounds Y (r >= 3)
 * for rho_hat and eta (eq. suboptimality).
 * Y      device [r][3N], 1 <= r <= 8;  tol: relative tolerance (<= 0: 1e-7)
 * v_min  device [3N] unit direction D^{-1/2} x of the Ritz vector x of lambda_min
 *        (v^T Z v < 0 when lambda_min < 0), or NULL.
 * Synchronises `stream`.
 */
xm_status xm_certify(xm_problem* p, const double* Y, int32_t r, double tol, int32_t max_iter,
                     double* v_min, xm_cert* cert, void* stream);

/*
 * Rounding (Prop. "SDP Relaxation" and the text after it): top-3 eigenvectors
 * of X = Y^T Y (through the r x r Gram Y Y^T), projection of each 3x3 block
 * to a scaled rotation with the majority determinant sign, anchoring
 * R_k <- R_0^T R_k, s_k <- s_k / s_0, and rho_hat = tr(Q Uhat^T Uhat) in FP64.
 * Y      device [r][3N], 3 <= r <= 8
 * R_out  device [N][3][3] row-major rotations;  s_out device [N] scales
 * rho_hat host: cost of the rounded point (may be NULL)
 * Synchronises `stream`.
 */
xm_status xm_round(xm_problem* p, const double* Y, int32_t r, double* R_out, double* s_out,
                   double* rho_hat, void* stream);

/*
 * Translations and landmarks of an anchored rank-3 solution (eq. tpstar):
 * t[1:] = -A_tt[1:,1:]^{-1} A_rt[:,1:]^T U^T with t_0 = 0, and each landmark
 * the weighted mean p_k = (1/W_k) sum_o w_o (U_i u_o + t_i), for
 * U = [s_0 R_0, ..., s_{N-1} R_{N-1}].
 * R  device [N][3][3] row-major rotations, s device [N] scales (frame 0: I, 1
 *    as returned by xm_round)
 * t  device [N][3] or NULL;  pts device [M][3] or NULL (landmarks with no
 *    observation get 0).  Synchronises `stream`.
 */
xm_status xm_recover_tp(xm_problem* p, const double* R, const double* s, double* t, double* pts,
                        void* stream);

/*
 * Similarity alignment of an estimate to a reference, the registration App.
 * "Metrics" applies to camera positions before trajectory errors (there a
 * robust registration; here its least-squares form, the correspondence being
 * known): s > 0, R in SO(3), t minimising sum_i w_i |s R P_i + t - Q_i|^2, in
 * closed form (R the rotation closest to the weighted cross-covariance of the
 * centred points, s = tr(R^T C) / the weighted spread of P, t from the means).
 * Used with the camera positions t of xm_recover_tp it gives the anchored
 * gauge's similarity to a ground truth.
 * n  number of points (>= 1);  P, Q device [n][3] FP64 (row i: point i);
 * w  device [n] FP64 weights >= 0, or NULL for all 1.
 * out host [14]: s, R (row-major, 9), t (3), and the weighted RMS residual
 *    sqrt(sum_i w_i |s R P_i + t - Q_i|^2 / sum_i w_i).
 * Errors: XM_EINVAL for n < 1, NULL P / Q / out, a negative or non-finite
 * weight or point, a zero weight sum, or points P with no spread.  One
 * workgroup, fixed-order sums (bitwise reproducible).  Synchronises `stream`.
 */
xm_status xm_align_similarity(int64_t n, const double* P, const double* Q, const double* w, double* out,
                              void* stream);

/*
 * Residuals of eq. sba at anchored scaled rotations (R, s) (as from
 * xm_round), with the translations and landmarks of eq. tpstar:
 * e_o = s_i R_i u_o + t_i - p_k for every observation o = (i, k), and the
 * score that ranks them for the XM^2 deletion: |e_o| (frame_units = 0) or
 * |e_o| / s_i (frame_units = 1: the residual in the units of frame i's lifted
 * keypoints, which does not favour deleting the anchored frame's
 * observations when the optimum shrinks the other frames' scales).
 * R device [N][3][3], s device [N]; e device [n_in][3] or NULL; score device
 * [n_in] or NULL (not both NULL); caller's observation order, 0 for
 * observations a masked build left out.  Synchronises `stream`.
 */
xm_status xm_residuals(xm_problem* p, const double* R, const double* s, int32_t frame_units, double* e,
                       double* score, void* stream);

/*
 * The XM^2 deletion: keep[o] = 0 for the floor(frac * n) observations with the
 * largest score, 1 for the others (ties: the lower index is deleted first).
 * score device [n] (finite, >= 0), keep device uint8 [n]; *n_dropped (host,
 * may be NULL) receives the number deleted.  Deterministic (stable radix sort
 * of the 64-bit score keys).  XM_EINVAL for frac outside [0, 1], n outside
 * [1, 2^31) or a negative / non-finite score.  Synchronises `stream`.
 */
xm_status xm_drop_largest(const double* score, int64_t n, double frac, uint8_t* keep, int64_t* n_dropped,
                          void* stream);

/*
 * Frame guard of the XM^2 deletion (Section "Structure from Motion with XM",
 * solver paragraph; the paper leaves open what happens to a frame the
 * deletion leaves undetermined).  A kept observation of landmark k is a link
 * of its frame when k keeps at least two observations; a frame with fewer
 * than min_links links is starved, and every observation of a starved frame
 * or of a landmark a starved frame sees is kept again.  One pass; afterwards
 * every frame has min_links links or all the links it can have, so a second
 * call changes nothing.  frame, landmark device int32 [n] (frame in [0, N),
 * landmark in [0, M)); keep device uint8 [n], nonzero = kept, updated in place
 * (restored entries become 1); *n_restored (host, may be NULL) receives the
 * number of entries restored.  Deterministic (integer counts).  XM_EINVAL for
 * N or M < 1, n outside [1, 2^31), min_links < 0 or an index out of range
 * (keep untouched).  Synchronises `stream`.
 */
xm_status xm_guard_frames(int32_t N, int32_t M, int64_t n, const int32_t* frame, const int32_t* landmark,
                          int32_t min_links, uint8_t* keep, int64_t* n_restored, void* stream);

typedef struct {
  int32_t cg_iters;    /* CG iterations of the Hessian solve */
  double cg_residual;  /* final relative CG residual */
  double cost;         /* f = tr(Q U^T U) at (R, s) */
} xm_adjoint_info;

/*
 * Adjoint of the certified optimum with respect to the lifted keypoints u_o
 * and the weights w_o.  For a scalar loss l(R, s, f*) with partials
 * gR = dl/dR [N][3][3], gs = dl/ds [N] and gcost = dl/d(f*), writes
 * gu = dl/du [n_obs][3] and gw = dl/dw [n_obs] in the caller's observation
 * order.  The cost term uses the envelope theorem (d(f*) / du_o = 2 w_o U_i^T e_o,
 * d(f*) / dw_o = |e_o|^2, e_o the residual of eq. sba at the optimum); the
 * rotation/scale term solves H lam = grad l by CG on the Riemannian Hessian of
 * the problem with frame 0 held fixed (FP64 products) and then
 * dl/du_o = -2 w_o (U_i^T e^lam_o + Udot_i^T e_o), dl/dw_o = -2 <e_o, e^lam_o>,
 * where Udot_k = lam_s,k R_k + s_k lam_R,k and e^lam the residual of that
 * direction.  Valid at a tight certified optimum (rank-3, from xm_round).
 * gR / gs may be NULL (no rotation/scale loss); gu, gw are device buffers of
 * dtype g_dtype (XM_F64 or XM_F32).  cg_tol (<= 0: 1e-10) is relative to
 * |grad l|; cg_max <= 0 means 4N.  For callers that differentiate through the
 * solver (the torch autograd Function of the Python binding).
 * Returns XM_ENOCONV (outputs written from the last CG iterate) when CG meets a
 * direction of non-positive curvature (the point is not a tight certified
 * optimum) or stops at cg_max above cg_tol; info->cg_residual tells which.
 */
xm_status xm_adjoint(xm_problem* p, const double* R, const double* s, const double* gR,
                     const double* gs, double gcost, void* gu, void* gw, xm_dtype g_dtype,
                     double cg_tol, int32_t cg_max, xm_adjoint_info* info, void* stream);

/*
 * Measurement hooks for the Y Q product kernels (the HBM-bound kernels of the
 * local solver and of the Lanczos certificate).  With timing enabled, every
 * product on a handle is bracketed by HIP events on the stream it runs on.
 * xm_spmm_stats synchronises those events and returns, per slot, the number of
 * launches, their total device time and the algorithmic bytes of one launch
 * (averaged over the recorded launches): the values the product must read
 * (see xm_set_spmm_kind) times their size.  Slots: xm_dtype (0..2) for the
 * dense kernel over the stored Q of that precision (the main kernel only, not
 * the pass that adds its partial sums); XM_STATS_FACTORED (3) and 4 for the
 * FP64 and FP32 factored products, bracketed whole (all their kernels);
 * XM_STATS_GINV (5) and 6 for the symmetric dense kernel over G^{-1} inside
 * the FP64 and FP32 factored products (that kernel alone); XM_STATS_FACT_ROWS
 * (7) and 8 for the pass of the FP64 and FP32 factored products that forms
 * A_rr Y^T and B^T Y^T (its bytes: the factor values and indices it streams,
 * each padded Y^T or staged union row once, and its outputs).  reset != 0
 * forgets the recorded launches.
 */
#define XM_STATS_FACTORED 3
#define XM_STATS_GINV 5
#define XM_STATS_FACT_ROWS 7
#define XM_STATS_SLOTS 9
typedef struct {
  int64_t launches[XM_STATS_SLOTS];
  double total_ms[XM_STATS_SLOTS];
  double bytes_per_launch[XM_STATS_SLOTS];
} xm_spmm_counters;
xm_status xm_spmm_timing(xm_problem* p, int32_t enable);
xm_status xm_spmm_stats(xm_problem* p, xm_spmm_counters* out, int32_t reset);

/* Message for the last failure on this thread ("" if none). */
const char* xm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* XM_H_ */
