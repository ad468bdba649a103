// Dual certificate (Theorem "Dual Optimality Certificate"), FP64.
//
// The constraint matrices act on the diagonal 3x3 blocks only (App. "Proof of
// LICQ condition"): sum y_i A_i = blkdiag(Lambda_k), with Lambda_0 symmetric and
// Lambda_k (k >= 1) symmetric traceless.  Z(y) Y^T = 0 then gives, block by
// block, Lambda_k = sym((Q Y^T)_k Y_k) / alpha_k (alpha_k = |Y_k|^2 / 3), made
// traceless for k >= 1.  The dual objective b^T y is tr(Lambda_0).
//
// PSD-ness of Z is decided on the congruent operator
//   Zs = D^{-1/2} Z D^{-1/2},   D = blkdiag(Q_kk)   (3x3 SPD diagonal blocks of Q),
// which by Sylvester's law of inertia has the same signature as Z but a much
// narrower spectrum (block-Jacobi scaling), so Lanczos needs far fewer
// products.  Its smallest eigenvalue ls with Ritz residual res bounds the
// spectrum of Zs on the complement of D^{1/2} rows(Y) from below by ls - res
// (given that the Ritz value belongs to the smallest eigenvalue, which the
// stop rule below guards).  The deflated block itself (its smallest eigenvalue
// and its coupling to the complement, both zero at a critical point) extends
// that to a bound b on the whole spectrum of Zs, so the point need not be
// stationary for the test to be sound; then
// v^T Z v >= b * (d_min if b >= 0, else d_max) for every unit v, d_min/d_max
// the extreme eigenvalues of the Q_kk; certified iff that is >= -tol * qbar.
//
// Lanczos runs on the orthogonal complement of D^{1/2} rows(Y) (Zs D^{1/2} Y^T
// = D^{-1/2} Z Y^T = 0 at a critical point): the first r basis vectors are an
// orthonormal basis of D^{1/2} rows(Y), every new Lanczos vector is
// orthogonalised against all previous ones twice (classical Gram-Schmidt,
// "twice is enough"), and alpha_j, beta_j stay on the device so that
// iterations run without host synchronisation.  Every few iterations the host
// takes the smallest eigenvalue of the tridiagonal T_j by Sturm bisection and
// its eigenvector by inverse iteration; the Ritz residual is beta_j |y_j|.
// Convergence needs a small residual at two consecutive checks with the
// smallest Ritz value unchanged between them (a converged Ritz value above a
// not yet resolved smaller eigenvalue moves when the latter appears).
#include <algorithm>
#include <cmath>
#include <vector>

#include "problem.h"

namespace xm {
namespace {

constexpr int kB = 256;
// rows of D^{1/2} Y kept in the deflation basis: residual above this fraction
// of the largest row norm
constexpr double kDeflRel = 1e-3;

// Lambda_k from (Q Y^T)_k.  With the scale regulariser (lam > 0, App. "Scale
// Regularization") the stationarity condition carries Q + grad F(X), grad F
// the diagonal 2 lam (X_{3k+2,3k+2} - 1) = 2 lam (alpha_k - 1) at row 3k+2 for
// k >= 1; Z = Q + grad F - blkdiag(Lambda) is stored as Q - blkdiag(Lambda'),
// Lambda'_k = Lambda_k - grad F_k.  part: {|Z Y^T|^2, tr(QX), tr(Lambda_0),
// F(X), <grad F, X>}.
template <int R>
__global__ __launch_bounds__(kB) void lambda_kernel(int32_t N, const double* __restrict__ Yt,
                                                    const double* __restrict__ G, double lam,
                                                    double* __restrict__ Lam, double* part) {
  const int k = blockIdx.x * kB + threadIdx.x;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (k < N) {
    double y[3][R], g[3][R];
    double nn = 0.0;
    for (int c = 0; c < 3; ++c)
      for (int a = 0; a < R; ++a) {
        y[c][a] = Yt[(3 * static_cast<int64_t>(k) + c) * R + a];
        g[c][a] = G[(3 * static_cast<int64_t>(k) + c) * R + a];
        nn += y[c][a] * y[c][a];
        v[1] += y[c][a] * g[c][a];
      }
    const double alpha = nn / 3.0;
    const double gF = (k == 0) ? 0.0 : 2.0 * lam * (alpha - 1.0);
    if (gF != 0.0)
      for (int a = 0; a < R; ++a) g[2][a] += gF * y[2][a];
    v[3] = (k == 0) ? 0.0 : lam * (alpha - 1.0) * (alpha - 1.0);
    v[4] = gF * alpha;
    double L[3][3];
    for (int c = 0; c < 3; ++c)
      for (int d = 0; d < 3; ++d) {
        double s = 0.0;
        for (int a = 0; a < R; ++a) s += g[c][a] * y[d][a];
        L[c][d] = s / alpha;
      }
    for (int c = 0; c < 3; ++c)
      for (int d = c + 1; d < 3; ++d) L[c][d] = L[d][c] = 0.5 * (L[c][d] + L[d][c]);
    const double tr = L[0][0] + L[1][1] + L[2][2];
    if (k > 0)
      for (int c = 0; c < 3; ++c) L[c][c] -= tr / 3.0;
    else
      v[2] = tr;
    for (int c = 0; c < 3; ++c)
      for (int d = 0; d < 3; ++d)
        Lam[9 * static_cast<int64_t>(k) + 3 * c + d] = L[c][d] - ((c == 2 && d == 2) ? gF : 0.0);
    // stationarity residual ((Q + grad F) Y^T)_k - Lambda_k Y_k^T
    for (int c = 0; c < 3; ++c)
      for (int a = 0; a < R; ++a) {
        double s = g[c][a];
        for (int d = 0; d < 3; ++d) s -= L[c][d] * y[d][a];
        v[0] += s * s;
      }
  }
  __shared__ double lds[5 * (kB / 64)];
  block_sum<5>(v, lds);
  if (threadIdx.x == 0)
    for (int q = 0; q < 5; ++q) part[blockIdx.x * 5 + q] = v[q];
}

// w = Qx - blkdiag(Lambda) x
__global__ void zapply_kernel(int32_t N, const double* __restrict__ Lam, const double* __restrict__ x,
                              const double* __restrict__ Qx, double* __restrict__ w) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (i >= 3 * static_cast<int64_t>(N)) return;
  const int64_t k = i / 3;
  const int c = static_cast<int>(i % 3);
  const double* L = Lam + 9 * k + 3 * c;
  w[i] = Qx[i] - (L[0] * x[3 * k] + L[1] * x[3 * k + 1] + L[2] * x[3 * k + 2]);
}

// y_k = M_k x_k per frame (M: [N][3][3] row-major)
__global__ void blockmul_kernel(int32_t N, const double* __restrict__ Mb, const double* __restrict__ x,
                                double* __restrict__ y) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (i >= 3 * static_cast<int64_t>(N)) return;
  const int64_t k = i / 3;
  const int c = static_cast<int>(i % 3);
  const double* m = Mb + 9 * k + 3 * c;
  y[i] = m[0] * x[3 * k] + m[1] * x[3 * k + 1] + m[2] * x[3 * k + 2];
}

// w = Dm (Qy - blkdiag(Lambda) y)   (y = Dm x already formed)
__global__ void zapply_scaled_kernel(int32_t N, const double* __restrict__ Lam, const double* __restrict__ Dm,
                                     const double* __restrict__ y, const double* __restrict__ Qy,
                                     double* __restrict__ w) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  double t[3];
  for (int c = 0; c < 3; ++c) {
    const double* L = Lam + 9 * static_cast<int64_t>(k) + 3 * c;
    t[c] = Qy[3 * static_cast<int64_t>(k) + c] -
           (L[0] * y[3 * static_cast<int64_t>(k)] + L[1] * y[3 * static_cast<int64_t>(k) + 1] +
            L[2] * y[3 * static_cast<int64_t>(k) + 2]);
  }
  for (int c = 0; c < 3; ++c) {
    const double* m = Dm + 9 * static_cast<int64_t>(k) + 3 * c;
    w[3 * static_cast<int64_t>(k) + c] = m[0] * t[0] + m[1] * t[1] + m[2] * t[2];
  }
}

// c[b] = <V[b], w> (one block per basis vector)
// part[b][g] = sum over segment g of V[b][i] w[i]  (grid: basis vector b x
// segment g, so that a few dozen vectors still fill the chip)
constexpr int kDotSeg = 16;
__global__ __launch_bounds__(kB) void multidot_kernel(const double* __restrict__ V, int64_t n,
                                                      const double* __restrict__ w, double* __restrict__ part) {
  const int64_t seg = (n + kDotSeg - 1) / kDotSeg;
  const int64_t i0 = blockIdx.y * seg, i1 = std::min(n, i0 + seg);
  const double* Vb = V + static_cast<int64_t>(blockIdx.x) * n;
  double v[1] = {0.0};
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kB) v[0] += Vb[i] * w[i];
  __shared__ double lds[kB / 64];
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x * kDotSeg + blockIdx.y] = v[0];
}

// c[b] = sum_g part[b][g], in segment order
__global__ void multidot_sum_kernel(const double* __restrict__ part, int nv, double* __restrict__ c) {
  const int b = blockIdx.x * kB + threadIdx.x;
  if (b >= nv) return;
  double t = 0.0;
  for (int g = 0; g < kDotSeg; ++g) t += part[b * kDotSeg + g];
  c[b] = t;
}

// w[i] += sign * sum_b c[b] V[b][i]
__global__ __launch_bounds__(kB) void multiaxpy_kernel(const double* __restrict__ V, int nv, int64_t n,
                                                       const double* __restrict__ c, double sign,
                                                       double* __restrict__ w) {
  __shared__ double cs[2048];
  for (int b = threadIdx.x; b < nv; b += kB) cs[b] = c[b];
  __syncthreads();
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int b = 0; b < nv; ++b) acc += cs[b] * V[static_cast<int64_t>(b) * n + i];
  w[i] += sign * acc;
}

// alpha[j] = c1[jj] + c2[jj]; beta[j] = |w|; out = w / beta (single block)
__global__ __launch_bounds__(1024) void normalize_kernel(const double* __restrict__ w, int64_t n,
                                                         const double* __restrict__ c1,
                                                         const double* __restrict__ c2, int jj, double* alpha,
                                                         double* beta, int j, double* __restrict__ out) {
  double v[1] = {0.0};
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) v[0] += w[i] * w[i];
  __shared__ double lds[1024 / 64];
  __shared__ double bsh;
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) {
    const double b = sqrt(v[0]);
    bsh = b;
    if (beta) beta[j] = b;
    if (alpha) alpha[j] = c1[jj] + c2[jj];
  }
  __syncthreads();
  const double b = bsh;
  const double inv = (b > 0.0) ? 1.0 / b : 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) out[i] = w[i] * inv;
}

// column a of Yt ([n][r]) -> w
__global__ void column_kernel(const double* __restrict__ Yt, int r, int a, int64_t n, double* w) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (i < n) w[i] = Yt[i * r + a];
}

// deterministic pseudo-random start vector in [-1, 1] (splitmix64 of the index)
__global__ void random_kernel(int64_t n, uint64_t seed, double* w) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (i >= n) return;
  uint64_t z = static_cast<uint64_t>(i) + seed * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  w[i] = static_cast<double>(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// ---- host side --------------------------------------------------------------
// smallest eigenvalue of the symmetric tridiagonal (d, e) by Sturm bisection
double tridiag_min_eig(const std::vector<double>& d, const std::vector<double>& e, int n) {
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i < n - 1 ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  const double scale = std::max(std::fabs(lo), std::fabs(hi)) + 1e-300;
  auto count_below = [&](double x) {
    int cnt = 0;
    double q = d[0] - x;
    if (q < 0) ++cnt;
    for (int i = 1; i < n; ++i) {
      if (q == 0.0) q = 1e-300 * scale;
      q = d[i] - x - e[i - 1] * e[i - 1] / q;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * scale; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= 1) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// eigenvector of the tridiagonal for the eigenvalue theta (inverse iteration;
// T - sigma I with sigma just below the smallest eigenvalue is positive definite)
std::vector<double> tridiag_min_vec(const std::vector<double>& d, const std::vector<double>& e, int n,
                                    double theta) {
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale = std::max(scale, std::fabs(d[i]) + (i < n - 1 ? std::fabs(e[i]) : 0.0));
  const double sigma = theta - 1e-10 * (scale + 1e-300);
  std::vector<double> y(n, 1.0), piv(n), rhs(n);
  for (int it = 0; it < 3; ++it) {
    // LDL^T-free Thomas solve of (T - sigma I) x = y
    std::vector<double> cp(n), dp(n);
    double den = d[0] - sigma;
    cp[0] = (n > 1) ? e[0] / den : 0.0;
    dp[0] = y[0] / den;
    for (int i = 1; i < n; ++i) {
      den = (d[i] - sigma) - e[i - 1] * cp[i - 1];
      cp[i] = (i < n - 1) ? e[i] / den : 0.0;
      dp[i] = (y[i] - e[i - 1] * dp[i - 1]) / den;
    }
    std::vector<double> x(n);
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
    double nn = 0.0;
    for (double v : x) nn += v * v;
    nn = std::sqrt(nn);
    for (int i = 0; i < n; ++i) y[i] = x[i] / nn;
  }
  return y;
}

// eigenvalues (returned) and eigenvectors (columns of V, row-major n x n) of a
// small symmetric matrix by cyclic Jacobi rotations
std::vector<double> small_sym_eig(std::vector<double> A, int n, std::vector<double>* V) {
  std::vector<double> E(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) E[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += A[i * n + i] * A[i * n + i];
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    }
    if (off <= 1e-30 * (diag + 1e-300)) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (apq == 0.0) continue;
        const double th = 0.5 * (A[q * n + q] - A[p * n + p]) / apq;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - sn * akq;
          A[k * n + q] = sn * akp + c * akq;
          const double ekp = E[k * n + p], ekq = E[k * n + q];
          E[k * n + p] = c * ekp - sn * ekq;
          E[k * n + q] = sn * ekp + c * ekq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - sn * aqk;
          A[q * n + k] = sn * apk + c * aqk;
        }
      }
  }
  std::vector<double> lam(n);
  for (int i = 0; i < n; ++i) lam[i] = A[i * n + i];
  if (V) *V = E;
  return lam;
}

double small_sym_min_eig(const std::vector<double>& A, int n) {
  if (n == 0) return 0.0;
  const std::vector<double> lam = small_sym_eig(A, n, nullptr);
  return *std::min_element(lam.begin(), lam.end());
}

template <int R>
void launch_lambda(int32_t N, const double* Yt, const double* G, double lam, double* Lam, double* part,
                   hipStream_t s) {
  hipLaunchKernelGGL((lambda_kernel<R>), dim3(cdiv(N, kB)), dim3(kB), 0, s, N, Yt, G, lam, Lam, part);
  XM_LAUNCH_CHECK("lambda_kernel");
}

}  // namespace

// The solver reads a few hundred partial sums per iteration: through a pinned
// (page-locked) staging buffer, one per host thread, the copy is a single DMA
// instead of a staged pageable transfer.  The buffer lives until the process
// ends (it is not freed at thread exit, when the runtime may be gone).
namespace {
// the calling thread's pinned staging buffer, grown to at least n doubles
double* staging(size_t n) {
  static thread_local double* h = nullptr;
  static thread_local size_t cap = 0;
  if (n > cap) {
    void* ptr = nullptr;
    XM_HIP(hipHostMalloc(&ptr, n * sizeof(double), hipHostMallocDefault));
    if (h) (void)hipHostFree(h);
    h = static_cast<double*>(ptr);
    cap = n;
  }
  return h;
}

void sum_blocks(const double* h, int blocks, int nq, double* out) {
  for (int q = 0; q < nq; ++q) {
    double acc = 0.0;
    for (int b = 0; b < blocks; ++b) acc += h[static_cast<size_t>(b) * nq + q];
    out[q] = acc;
  }
}
}  // namespace

void read_partials(const double* dev, int blocks, int nq, double* out, hipStream_t s) {
  const size_t n = static_cast<size_t>(blocks) * nq;
  double* h = staging(n);
  XM_HIP(hipMemcpyAsync(h, dev, n * sizeof(double), hipMemcpyDeviceToHost, s));
  XM_HIP(hipStreamSynchronize(s));
  sum_blocks(h, blocks, nq, out);
}

void read_partials2(const double* dev, int blocks, int nq, double* out, int64_t off2, int n2, double* out2,
                    hipStream_t s) {
  double* h = staging(static_cast<size_t>(off2) + n2);
  XM_HIP(hipMemcpyAsync(h, dev, (static_cast<size_t>(off2) + n2) * sizeof(double), hipMemcpyDeviceToHost, s));
  XM_HIP(hipStreamSynchronize(s));
  sum_blocks(h, blocks, nq, out);
  for (int k = 0; k < n2; ++k) out2[k] = h[off2 + k];
}

CertResult certify_yt(xm_problem* p, const double* Yt, int r, double tol, int max_iter, double lanczos_tol,
                      double* v_out, hipStream_t s) {
  require(r >= 1 && r <= 8, XM_EINVAL, "certificate: rank must be in [1, 8]");
  const int32_t N = p->N;
  const int64_t n = p->n3;
  const double qbar = p->qbar;
  require(n > r, XM_EINVAL, "certificate: 3N must exceed the rank");
  if (max_iter <= 0) max_iter = 400;
  max_iter = std::min<int>(max_iter, static_cast<int>(std::min<int64_t>(n - r, 2000 - 8)));
  if (lanczos_tol <= 0) lanczos_tol = 1e-6;
  CertResult out;

  DevBuf<double> G(n * r), Lam(9 * static_cast<size_t>(N)), part(static_cast<size_t>(cdiv(N, kB)) * 5);
  spmm_yt<double>(p, XM_F64, Yt, r, G.ptr, s);
  switch (r) {
    case 1: launch_lambda<1>(N, Yt, G.ptr, p->scale_reg, Lam.ptr, part.ptr, s); break;
    case 2: launch_lambda<2>(N, Yt, G.ptr, p->scale_reg, Lam.ptr, part.ptr, s); break;
    case 3: launch_lambda<3>(N, Yt, G.ptr, p->scale_reg, Lam.ptr, part.ptr, s); break;
    case 4: launch_lambda<4>(N, Yt, G.ptr, p->scale_reg, Lam.ptr, part.ptr, s); break;
    case 5: launch_lambda<5>(N, Yt, G.ptr, p->scale_reg, Lam.ptr, part.ptr, s); break;
    case 6: launch_lambda<6>(N, Yt, G.ptr, p->scale_reg, Lam.ptr, part.ptr, s); break;
    case 7: launch_lambda<7>(N, Yt, G.ptr, p->scale_reg, Lam.ptr, part.ptr, s); break;
    case 8: launch_lambda<8>(N, Yt, G.ptr, p->scale_reg, Lam.ptr, part.ptr, s); break;
  }
  double sums[5];
  read_partials(part.ptr, cdiv(N, kB), 5, sums, s);
  out.stat_res = std::sqrt(sums[0]);
  // primal tr(QX) + F(X); dual tr(Lambda_0) + F(X) - <grad F(X), X> (F = 0 without the regulariser)
  out.primal = sums[1] + sums[3];
  out.dual = sums[2] + sums[3] - sums[4];

  // basis: [deflation rows D^{1/2} Y | Lanczos vectors of Zs]
  const int cap = r + max_iter + 1;
  DevBuf<double> V(static_cast<size_t>(cap) * n), w(n), Qx(n), yv(n), c1(cap), c2(cap), alpha(max_iter),
      beta(max_iter);
  const unsigned gb = cdiv(n, kB);
  DevBuf<double> dpart(static_cast<size_t>(cap) * kDotSeg);
  auto multidot = [&](int nv, double* c) {  // c = V[0..nv) w
    hipLaunchKernelGGL(multidot_kernel, dim3(nv, kDotSeg), dim3(kB), 0, s, V.ptr, n, w.ptr, dpart.ptr);
    hipLaunchKernelGGL(multidot_sum_kernel, dim3(cdiv(nv, kB)), dim3(kB), 0, s, dpart.ptr, nv, c);
  };
  auto orthogonalize = [&](int nv) {  // w -= V[0..nv) (V^T w), twice
    if (nv == 0) return;
    multidot(nv, c1.ptr);
    hipLaunchKernelGGL(multiaxpy_kernel, dim3(gb), dim3(kB), 0, s, V.ptr, nv, n, c1.ptr, -1.0, w.ptr);
    multidot(nv, c2.ptr);
    hipLaunchKernelGGL(multiaxpy_kernel, dim3(gb), dim3(kB), 0, s, V.ptr, nv, n, c2.ptr, -1.0, w.ptr);
    XM_LAUNCH_CHECK("orthogonalize");
  };
  // Deflation basis: the left singular vectors of D^{1/2} Y^T (3N x r) whose
  // singular values exceed kDeflRel times the largest, from the eigenpairs of
  // the r x r Gram matrix (sigma_j^2, e_j): w_j = D^{1/2} Y^T e_j / sigma_j.
  // Directions of Y's row space that are (numerically) combinations of the
  // others -- a rank-5 factor of a rank-3 optimum carries two such at the level
  // of the solver's gradient -- would add directions that are neither null
  // vectors of Z nor small in the coupling term below; they stay in the
  // complement, where Lanczos sees them.
  auto norm_of_w = [&](double* out_vec) {  // out_vec = w / |w|
    hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(1024), 0, s, w.ptr, n, c1.ptr, c2.ptr, 0,
                       static_cast<double*>(nullptr), beta.ptr, 0, out_vec);
    XM_LAUNCH_CHECK("normalize_kernel");
  };
  DevBuf<double> rows(static_cast<size_t>(r) * n);
  for (int a = 0; a < r; ++a) {
    hipLaunchKernelGGL(column_kernel, dim3(gb), dim3(kB), 0, s, Yt, r, a, n, yv.ptr);
    hipLaunchKernelGGL(blockmul_kernel, dim3(gb), dim3(kB), 0, s, N, p->Dhalf.ptr, yv.ptr,
                       rows.ptr + static_cast<int64_t>(a) * n);
    XM_LAUNCH_CHECK("blockmul_kernel");
  }
  std::vector<double> gram(static_cast<size_t>(r) * r);
  for (int a = 0; a < r; ++a) {
    hipLaunchKernelGGL(multidot_kernel, dim3(r, kDotSeg), dim3(kB), 0, s, rows.ptr, n,
                       rows.ptr + static_cast<int64_t>(a) * n, dpart.ptr);
    hipLaunchKernelGGL(multidot_sum_kernel, dim3(1), dim3(kB), 0, s, dpart.ptr, r, c1.ptr);
    XM_LAUNCH_CHECK("multidot_kernel");
    XM_HIP(hipMemcpyAsync(gram.data() + static_cast<size_t>(a) * r, c1.ptr, r * sizeof(double),
                          hipMemcpyDeviceToHost, s));
  }
  XM_HIP(hipStreamSynchronize(s));
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < a; ++b) gram[a * r + b] = gram[b * r + a] = 0.5 * (gram[a * r + b] + gram[b * r + a]);
  std::vector<double> E;
  const std::vector<double> sig2 = small_sym_eig(gram, r, &E);
  std::vector<int> idx(r);
  for (int a = 0; a < r; ++a) idx[a] = a;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return sig2[x] > sig2[y]; });
  const double smax = std::sqrt(std::max(0.0, sig2[idx[0]]));
  const double keep_min = std::max(kDeflRel * smax, 1e-10 * std::sqrt(static_cast<double>(N) * p->dmax));
  int nb = 0;
  std::vector<double> coef(r);
  for (int jj = 0; jj < r; ++jj) {
    const int j = idx[jj];
    const double sj = std::sqrt(std::max(0.0, sig2[j]));
    if (!(sj > keep_min)) break;
    for (int a = 0; a < r; ++a) coef[a] = E[a * r + j] / sj;
    XM_HIP(hipMemcpyAsync(c1.ptr, coef.data(), r * sizeof(double), hipMemcpyHostToDevice, s));
    XM_HIP(hipMemsetAsync(w.ptr, 0, n * sizeof(double), s));
    hipLaunchKernelGGL(multiaxpy_kernel, dim3(gb), dim3(kB), 0, s, rows.ptr, r, n, c1.ptr, 1.0, w.ptr);
    XM_LAUNCH_CHECK("multiaxpy_kernel");
    orthogonalize(nb);  // exact up to rounding; keeps the basis orthonormal to machine precision
    norm_of_w(V.ptr + static_cast<int64_t>(nb) * n);
    ++nb;
  }
  // The deflated block.  W = V[0..nb) is an orthonormal basis of D^{1/2} rows(Y).
  // With a = lambda_min(W^T Zs W), e = |(I - W W^T) Zs W| and b the smallest
  // eigenvalue of Zs on the complement of W (the Lanczos run below), every unit
  // vector v = x + y (x in span W, y orthogonal to it) has
  //   v^T Zs v >= a |x|^2 + b |y|^2 - 2 e |x| |y| >= (a+b)/2 - sqrt(((a-b)/2)^2 + e^2),
  // a lower bound on the whole spectrum of Zs.  At a critical point Z Y^T = 0, so
  // a = e = 0 and the bound is min(0, b); away from one, e carries the
  // stationarity residual into the bound (the complement alone would not
  // decide PSD-ness).  Each column of Zs W costs one FP64 product in the
  // residual role (the accurate one: Zs W cancels heavily near the optimum).
  double defl_min = 0.0, defl_cross = 0.0;
  if (nb > 0) {
    std::vector<double> Mw(static_cast<size_t>(nb) * nb);
    double fro2 = 0.0;
    for (int a = 0; a < nb; ++a) {
      const double* x = V.ptr + static_cast<int64_t>(a) * n;
      hipLaunchKernelGGL(blockmul_kernel, dim3(gb), dim3(kB), 0, s, N, p->Dmhalf.ptr, x, yv.ptr);
      XM_LAUNCH_CHECK("blockmul_kernel");
      spmm_yt<double>(p, XM_F64, yv.ptr, 1, Qx.ptr, s, XM_ROLE_RESIDUAL);
      hipLaunchKernelGGL(zapply_scaled_kernel, dim3(cdiv(N, kB)), dim3(kB), 0, s, N, Lam.ptr, p->Dmhalf.ptr, yv.ptr,
                         Qx.ptr, w.ptr);
      XM_LAUNCH_CHECK("zapply_scaled_kernel");
      multidot(nb, c1.ptr);
      hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(1024), 0, s, w.ptr, n, c1.ptr, c2.ptr, 0,
                         static_cast<double*>(nullptr), beta.ptr, 0, Qx.ptr);
      XM_LAUNCH_CHECK("normalize_kernel");
      double bn = 0.0;
      XM_HIP(hipMemcpyAsync(Mw.data() + static_cast<size_t>(a) * nb, c1.ptr, nb * sizeof(double),
                            hipMemcpyDeviceToHost, s));
      XM_HIP(hipMemcpyAsync(&bn, beta.ptr, sizeof(double), hipMemcpyDeviceToHost, s));
      XM_HIP(hipStreamSynchronize(s));
      fro2 += bn * bn;
    }
    double m2 = 0.0;
    std::vector<double> Ms(Mw.size());
    for (int a = 0; a < nb; ++a)
      for (int b = 0; b < nb; ++b) {
        m2 += Mw[a * nb + b] * Mw[a * nb + b];
        Ms[a * nb + b] = 0.5 * (Mw[a * nb + b] + Mw[b * nb + a]);
      }
    defl_min = small_sym_min_eig(Ms, nb);
    defl_cross = std::sqrt(std::max(0.0, fro2 - m2));
  }
  out.defl_min = defl_min;
  out.defl_cross = defl_cross;

  hipLaunchKernelGGL(random_kernel, dim3(gb), dim3(kB), 0, s, n, static_cast<uint64_t>(12345), w.ptr);
  orthogonalize(nb);
  hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(1024), 0, s, w.ptr, n, c1.ptr, c2.ptr, 0,
                     static_cast<double*>(nullptr), static_cast<double*>(nullptr), 0,
                     V.ptr + static_cast<int64_t>(nb) * n);
  XM_LAUNCH_CHECK("normalize_kernel");
  // tolerances in the units of Zs
  const double tol_s = tol * qbar / p->dmax;
  const double ltol_s = lanczos_tol * qbar / p->dmax;

  std::vector<double> ha, hbv, d, e, y;
  double theta = 0.0, res = 0.0, theta_prev = 0.0;
  bool prev_small = false;
  int j = 0;
  bool done = false;
  for (j = 0; j < max_iter && !done; ++j) {
    const double* x = V.ptr + static_cast<int64_t>(nb + j) * n;
    hipLaunchKernelGGL(blockmul_kernel, dim3(gb), dim3(kB), 0, s, N, p->Dmhalf.ptr, x, yv.ptr);
    XM_LAUNCH_CHECK("blockmul_kernel");
    spmm_yt<double>(p, XM_F64, yv.ptr, 1, Qx.ptr, s, XM_ROLE_CURVATURE);
    hipLaunchKernelGGL(zapply_scaled_kernel, dim3(cdiv(N, kB)), dim3(kB), 0, s, N, Lam.ptr, p->Dmhalf.ptr, yv.ptr,
                       Qx.ptr, w.ptr);
    XM_LAUNCH_CHECK("zapply_scaled_kernel");
    const int nv = nb + j + 1;
    orthogonalize(nv);
    hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(1024), 0, s, w.ptr, n, c1.ptr, c2.ptr, nb + j, alpha.ptr,
                       beta.ptr, j, V.ptr + static_cast<int64_t>(nv) * n);
    XM_LAUNCH_CHECK("normalize_kernel");
    const int m = j + 1;
    if (m % 5 == 0 || m == max_iter) {
      ha.resize(m);
      hbv.resize(m);
      XM_HIP(hipMemcpyAsync(ha.data(), alpha.ptr, m * sizeof(double), hipMemcpyDeviceToHost, s));
      XM_HIP(hipMemcpyAsync(hbv.data(), beta.ptr, m * sizeof(double), hipMemcpyDeviceToHost, s));
      XM_HIP(hipStreamSynchronize(s));
      d.assign(ha.begin(), ha.end());
      e.assign(hbv.begin(), hbv.end());  // e[i] couples i and i+1; e[m-1] = beta_{m-1} is the residual factor
      theta = tridiag_min_eig(d, e, m);
      y = tridiag_min_vec(d, e, m, theta);
      res = std::fabs(hbv[m - 1] * y[m - 1]);
      const bool breakdown = hbv[m - 1] <= 1e-14 * (std::fabs(theta) + 1.0);
      const bool small = res <= ltol_s || res <= 1e-3 * std::fabs(theta);
      const bool stable = std::fabs(theta - theta_prev) <= 1e-6 * std::fabs(theta) + ltol_s;
      const bool converged = small && prev_small && stable;
      const bool negative = theta + res < -tol_s;
      if (breakdown || converged || negative) done = true;
      prev_small = small;
      theta_prev = theta;
    }
  }
  out.iters = j;
  out.lambda_min = theta;
  out.ritz_residual = res;
  const double lo = theta - res;
  double full = lo;
  if (nb > 0) {
    const double h = 0.5 * (defl_min - lo);
    full = 0.5 * (defl_min + lo) - std::sqrt(h * h + defl_cross * defl_cross);
  }
  // v^T Z v = (D^{1/2} v)^T Zs (D^{1/2} v) and d_min |v|^2 <= |D^{1/2} v|^2 <= d_max |v|^2
  out.lambda_bound = full * (full >= 0.0 ? p->dmin : p->dmax);
  out.certified = out.lambda_bound >= -tol * qbar;
  out.complement_ok = lo * (lo >= 0.0 ? p->dmin : p->dmax) >= -tol * qbar;
  if (v_out) {
    const int m = static_cast<int>(y.size());
    DevBuf<double> yd(m);
    XM_HIP(hipMemcpyAsync(yd.ptr, y.data(), m * sizeof(double), hipMemcpyHostToDevice, s));
    XM_HIP(hipMemsetAsync(w.ptr, 0, n * sizeof(double), s));
    hipLaunchKernelGGL(multiaxpy_kernel, dim3(gb), dim3(kB), 0, s, V.ptr + static_cast<int64_t>(nb) * n, m, n,
                       yd.ptr, 1.0, w.ptr);
    XM_LAUNCH_CHECK("multiaxpy_kernel");
    // Ritz vector of Zs -> direction in the coordinates of Z: v = D^{-1/2} vs (v^T Z v = vs^T Zs vs)
    hipLaunchKernelGGL(blockmul_kernel, dim3(gb), dim3(kB), 0, s, N, p->Dmhalf.ptr, w.ptr, yv.ptr);
    hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(1024), 0, s, yv.ptr, n, c1.ptr, c2.ptr, 0,
                       static_cast<double*>(nullptr), static_cast<double*>(nullptr), 0, v_out);
    XM_LAUNCH_CHECK("normalize_kernel");
    XM_HIP(hipStreamSynchronize(s));
  }
  XM_HIP(hipStreamSynchronize(s));
  return out;
}

}  // namespace xm
