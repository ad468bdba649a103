// The problem handle and the internal launch interfaces of libxm.
#pragma once

#include <deque>
#include <memory>

#include "common.h"

struct xm_problem {
  int32_t N = 0, M = 0;
  int64_t n_obs = 0;   // observations used (those the build's mask kept)
  int64_t n_in = 0;    // observations the caller passed (the length of per-observation outputs)
  int32_t n3 = 0;   // 3N
  int32_t ld = 0;   // leading dimension of the dense Q copies (multiple of 64)
  uint32_t copies = 1;
  double qbar = 0.0;
  double build_ms = 0.0;
  // scale regulariser lam of App. "Scale Regularization" (xm_set_scale_reg)
  double scale_reg = 0.0;
  int64_t nnzb = 0, n_pairs = 0;
  // device time of the main assembly kernels of the build (xm_build_stats)
  struct KernelStat {
    const char* name;
    int launches;
    double ms, bytes, flops;
  };
  std::vector<KernelStat> build_stats;

  // Q, row-major [3N][ld], zero padding columns
  // Q, rows and columns in the frame order (`order` / `pos` below): row 3 pos[k] + c
  // of the stored matrix is row 3k + c of Q
  xm::DevBuf<double> Q64;
  xm::DevBuf<float> Q32;
  xm::DevBuf<uint16_t> Q16;

  // observations sorted by landmark (kept for recovery of t, p and the adjoint)
  xm::DevBuf<int32_t> fr_s, lm_s;
  xm::DevBuf<double> u_s, w_s;     // [n][3], [n]
  xm::DevBuf<int64_t> perm;        // sorted position -> original index
  xm::DevBuf<int64_t> lm_ptr;      // [M+1]
  xm::DevBuf<double> Wl;           // per-landmark weight sum
  // co-visibility pattern (rows = frames), with the eliminated-landmark blocks
  xm::DevBuf<int32_t> row_ptr, col;  // [N+1], [nnzb]
  // Cuthill-McKee order of the co-visibility graph: position -> frame, frame -> position
  xm::DevBuf<int32_t> order, pos;
  xm::DevBuf<double> Art;            // [nnzb][3]: A_rt[3i+a][j]
  // factors of the factored product, structure of arrays [15][nnzb]: for the
  // block s = (i, j), rows 3a+b (a, b < 3): A_rr[3i+a][3j+b]; rows 9+a:
  // A_rt[3i+a][j]; rows 12+a: A_rt[3j+a][i] (the transposed block's entry)
  xm::DevBuf<double> fac;
  xm::DevBuf<double> fact_scratch;   // padded Y^T, W and V of the factored product
  // groups of 16 frames consecutive in the Cuthill-McKee order: the union of
  // each group's co-visible frames j >= 1 (frame indices, increasing, from
  // grp_ustart[g]), the largest union, and per stored block s the position of
  // col[s] in its row's group union (-1 for frame 0); grp_maxu < 0: not built
  xm::DevBuf<int32_t> grp_uid, lidx;
  xm::DevBuf<int64_t> grp_ustart;
  int32_t grp_maxu = -1;
  size_t lds_max = 0;  // LDS bytes a workgroup may take on the build's device
  xm::DevBuf<double> perm_scratch;   // Y^T and Y^T Q in the frame order (dense products)
  xm::DevBuf<float> mixed_scratch;   // FP32 copies of an FP64 operand and result (mixed products)
  // FP32 copies of the factors (with XM_KEEP_F32): fac as above, -G^{-1}
  xm::DevBuf<float> fac32, Gm32;
  xm::DevBuf<double> Att;            // [nnzb]:    A_tt[i][j]
  // -(A_tt[1:,1:])^{-1}, row-major [N-1][ldg]
  xm::DevBuf<double> Gm;
  int32_t ldg = 0;

  // tr(Q_kk) / 3 per frame
  xm::DevBuf<double> qkk;
  // Q_kk^{1/2} and Q_kk^{-1/2} per frame ([N][3][3]) and the extreme
  // eigenvalues over all Q_kk (the block-Jacobi scaling of the certificate)
  xm::DevBuf<double> Dhalf, Dmhalf;
  double dmin = 1.0, dmax = 1.0;

  // split-row partial sums of the Y Q product (grown on demand)
  xm::DevBuf<char> spmm_scratch;

  // optional HIP-event timing of the Y Q product kernel (xm_spmm_timing)
  struct TimedLaunch {
    hipEvent_t start, stop;
    int dtype;
    double bytes;  // algorithmic bytes of Q the launch reads
  };
  // product kernel per role (xm_product_role) and Q precision (xm_dtype)
  int spmm_kind[2][3] = {{XM_SPMM_UPPER, XM_SPMM_UPPER, XM_SPMM_FULL},
                         {XM_SPMM_FACTORED, XM_SPMM_UPPER, XM_SPMM_FULL}};
  bool timing = false;
  std::deque<TimedLaunch> events;  // deque: a pointer to one stays valid while more are added
  size_t events_used = 0;

  ~xm_problem();
};

namespace xm {

// frames per group (consecutive in the Cuthill-McKee order) of the assembly's
// correction products and of the grouped passes of the factored product
constexpr int kFrameGroup = 16;

// Temporary device memory of one Y Q product.  Without a fixed region (the
// normal entry points) the handle's grow-only buffers serve, allocated on
// first use; with one (xm_spmm_noalloc) every temporary is carved from it in
// order, 256-byte aligned, and nothing is allocated: a request beyond its end
// throws XM_EINVAL.
struct Scratch {
  char* base = nullptr;
  size_t cap = 0, used = 0;
};

template <typename T, typename B>
T* take(Scratch* sc, DevBuf<B>& own, size_t count, hipStream_t s) {
  const size_t bytes = count * sizeof(T);
  if (sc && sc->base) {
    const size_t off = (sc->used + 255) & ~static_cast<size_t>(255);
    require(off + bytes <= sc->cap, XM_EINVAL, "the product needs more temporary memory than the fixed scratch holds");
    sc->used = off + bytes;
    return reinterpret_cast<T*>(sc->base + off);
  }
  const size_t n = (bytes + sizeof(B) - 1) / sizeof(B);
  if (own.n < n) {
    XM_HIP(hipStreamSynchronize(s));
    own.alloc(n);
  }
  return reinterpret_cast<T*>(own.ptr);
}

// build_q.hip
std::unique_ptr<xm_problem> build_problem(int32_t N, int32_t M, int64_t n_obs, const int32_t* frame,
                                          const int32_t* landmark, const void* u, xm_dtype u_dtype,
                                          const void* w, xm_dtype w_dtype, const uint8_t* mask, uint32_t copies,
                                          hipStream_t s);

// spmm.hip: out (3N x r, row-major, frame-major "Yt" layout, ld = r) = Q * Yt.
// Yt is [3N][r] (row i holds Y[0..r)[i]).  T is the vector precision.
// role: XM_ROLE_RESIDUAL (gradient, cost, multipliers: accuracy at the optimum)
// or XM_ROLE_CURVATURE (Hessian-vector and Lanczos products of directions).
// sc: temporaries from a fixed region (NULL: the handle's buffers).
template <typename T>
void spmm_yt(const xm_problem* p, xm_dtype qtype, const T* Yt, int r, T* out, hipStream_t s,
             int role = XM_ROLE_RESIDUAL, Scratch* sc = nullptr);
// Bytes of temporaries spmm_yt<T> takes from a fixed region for this product
// (alignment included).
size_t product_scratch_bytes(const xm_problem* p, xm_dtype qtype, int r, int role, bool fp64_vectors);

// noalloc.hip: size and per-device address of the fixed scratch of
// xm_spmm_noalloc (the address is looked up on the first call on a device)
constexpr size_t kNoallocScratchBytes = static_cast<size_t>(XM_NOALLOC_SCRATCH_MIB) << 20;
char* noalloc_scratch_base();

// layout conversions between the ABI layout Y[r][3N] and the internal Yt[3N][r]
template <typename Ts, typename Td>
void transpose_rows(const Ts* in, int rows, int cols, Td* out, hipStream_t s);

// certify.hip: certificate at Yt (FP64, [3N][r]).
struct CertResult {
  double lambda_min = 0, ritz_residual = 0, lambda_bound = 0, primal = 0, dual = 0, stat_res = 0;
  double defl_min = 0, defl_cross = 0;
  int iters = 0;
  bool certified = false;
  // the bound from the complement of rows(Y) alone (Lanczos lower bound, no
  // deflated block or coupling) passes the threshold
  bool complement_ok = false;
};
CertResult certify_yt(xm_problem* p, const double* Yt, int r, double tol, int max_iter, double lanczos_tol,
                      double* v_out, hipStream_t s);

// solver.hip
xm_status bm_solve(xm_problem* p, const xm_solve_opts& o, const double* Y0, int r_in, double* Y_out,
                   xm_solve_info* info, hipStream_t s);

// round.hip
void round_yt(xm_problem* p, const double* Y, int r, double* R_out, double* s_out, double* rho_hat,
              hipStream_t s);
// similarity alignment of n points P to Q (device [n][3], weights device [n]
// or NULL); out (host, 14): s, R row-major, t, weighted RMS residual
void align_similarity(int64_t n, const double* P, const double* Q, const double* w, double* out, hipStream_t s);

// adjoint.hip
struct AdjointResult {
  int cg_iters = 0;
  double cg_residual = 0.0, cost = 0.0;
  bool converged = true, negative_curvature = false;
};
void recover_tp(xm_problem* p, const double* R, const double* s, double* t_out, double* p_out, hipStream_t st);
// residuals e_o of eq. sba at (R, s) with t, p of eq. tpstar, in the caller's
// order ([n_in][3] and [n_in]; observations left out by the build's mask get 0);
// score_o = |e_o| (frame_units 0) or |e_o| / s_i (1)
void residuals(xm_problem* p, const double* R, const double* s, int frame_units, double* e_out, double* score_out,
               hipStream_t st);
AdjointResult adjoint(xm_problem* p, const double* R, const double* s, const double* gR, const double* gs,
                      double gcost, void* gu, void* gw, xm_dtype gdt, double cg_tol, int cg_max, hipStream_t st);

// Host sum of per-block partials [blocks][nq] (fixed order) after a stream sync.
void read_partials(const double* dev, int blocks, int nq, double* out, hipStream_t s);
// the same for `dev`, and the n2 plain values at dev + off2 (off2 >= blocks *
// nq) into out2, in one copy
void read_partials2(const double* dev, int blocks, int nq, double* out, int64_t off2, int n2, double* out2,
                    hipStream_t s);
// rows row0 .. row0 + nrows of Q (frame-index order) into out [nrows][3N]
void get_q_rows(const xm_problem* p, int32_t row0, int32_t nrows, double* out, hipStream_t s);

}  // namespace xm
