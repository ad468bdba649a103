// Rounding of the low-rank factor to anchored scaled rotations (Prop. "SDP
// Relaxation" and the text after it), FP64.
//
// X = Y^T Y has the same nonzero eigenvalues as the r x r Gram Y Y^T = V mu V^T;
// its best rank-3 factor is Ubar = V_3^T Y (V_3: top-3 eigenvectors).
//   1. Gram Y Y^T by FP64 matrix cores (v_mfma_f64_16x16x4f64): each wave
//      multiplies 16 x 4 slices of Y (rows padded to 16) by their transposes;
//      the per-wave partial Grams are added in a fixed order.
//   2. Cyclic Jacobi eigendecomposition of the r x r Gram (one thread).
//   3. Per frame: Ubar_k = V_3^T Y_k and det(Ubar_k); the host counts the
//      negative determinants and, if they are the majority, negates the third
//      row of Ubar (X is unchanged) -- the sign reading of this build.
//   4. Per frame: nearest scaled rotation by SVD through the 3x3 Jacobi
//      eigendecomposition of Ubar_k^T Ubar_k: R = [a1, a2, det(B) a1 x a2] B^T,
//      s = tr(R^T Ubar_k) / 3.
//   5. Anchor: R_k <- R_0^T R_k, s_k <- s_k / s_0; rho_hat = tr(Q Uhat^T Uhat)
//      by one FP64 product.
#include <cmath>
#include <vector>

#include "problem.h"

namespace xm {
namespace {

constexpr int kB = 256;
typedef double v4d __attribute__((ext_vector_type(4)));

template <int R>
__global__ __launch_bounds__(kB) void gram_mfma_kernel(const double* __restrict__ Yt, int64_t n,
                                                       double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * (kB / 64) + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * (kB / 64);
  const int row = lane & 15, kk = lane >> 4;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = static_cast<int64_t>(wave) * 4; k0 < n; k0 += static_cast<int64_t>(nwaves) * 4) {
    const int64_t k = k0 + kk;
    const double a = (row < R && k < n) ? Yt[k * R + row] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, acc, 0, 0, 0);
  }
  double* out = part + static_cast<int64_t>(wave) * 256;
  // v_mfma_f64_16x16x4f64 returns D[(lane / 16) + 4 q][lane % 16] in register q
#pragma unroll
  for (int q = 0; q < 4; ++q) out[((lane >> 4) + 4 * q) * 16 + (lane & 15)] = acc[q];
}

template <int NN>
__device__ void jacobi_eig(double (&A)[NN][NN], double (&V)[NN][NN], int n) {
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) V[p][q] = (p == q) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int p = 0; p < n; ++p) {
      dia += A[p][p] * A[p][p];
      for (int q = p + 1; q < n; ++q) off += A[p][q] * A[p][q];
    }
    if (off <= 1e-32 * dia || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
}

// Sum the per-wave Grams, eigendecompose, keep the top-3 eigenvectors.
// out: V3 [8][3] (row a, column i), mu [8] eigenvalues in descending order.
// One workgroup of kB threads: thread t adds entry t % 64 of the waves
// w = t / 64 (mod 4) in wave order, and the four sums are added in a fixed
// order (deterministic); then one thread runs the small eigensolver.
__global__ __launch_bounds__(kB) void gram_eig_kernel(const double* __restrict__ part, int nwaves, int r,
                                                      double* V3, double* mu) {
  __shared__ double sums[4][64];
  const int e = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int ei = e >> 3, ej = e & 7;
  double acc = 0.0;
  if (ei < r && ej < r) {
#pragma unroll 8
    for (int w = g; w < nwaves; w += 4) acc += part[static_cast<int64_t>(w) * 256 + ei * 16 + ej];
  }
  sums[g][e] = acc;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double A[8][8], V[8][8];
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) {
      const int k = i * 8 + j;
      A[i][j] = (sums[0][k] + sums[1][k]) + (sums[2][k] + sums[3][k]);
    }
  for (int i = 0; i < r; ++i)
    for (int j = i + 1; j < r; ++j) A[i][j] = A[j][i] = 0.5 * (A[i][j] + A[j][i]);
  jacobi_eig<8>(A, V, r);
  int idx[8];
  for (int i = 0; i < r; ++i) idx[i] = i;
  for (int i = 0; i < r; ++i)
    for (int j = i + 1; j < r; ++j)
      if (A[idx[j]][idx[j]] > A[idx[i]][idx[i]]) {
        const int t = idx[i];
        idx[i] = idx[j];
        idx[j] = t;
      }
  for (int i = 0; i < r; ++i) mu[i] = A[idx[i]][idx[i]];
  for (int a = 0; a < r; ++a)
    for (int i = 0; i < 3; ++i) V3[a * 3 + i] = V[a][idx[i]];
}

__device__ __forceinline__ double det3(const double (&M)[3][3]) {
  return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
         M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
}

// Ubar_k[i][c] = sum_a V3[a][i] Y_k[a][c]; partial count of negative determinants
__global__ __launch_bounds__(kB) void project_kernel(int32_t N, int r, const double* __restrict__ Yt,
                                                     const double* __restrict__ V3, double* __restrict__ Ub,
                                                     double* part) {
  const int k = blockIdx.x * kB + threadIdx.x;
  double v[1] = {0.0};
  if (k < N) {
    double M[3][3];
    for (int i = 0; i < 3; ++i)
      for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (int a = 0; a < r; ++a) s += V3[a * 3 + i] * Yt[(3 * static_cast<int64_t>(k) + c) * r + a];
        M[i][c] = s;
        Ub[9 * static_cast<int64_t>(k) + 3 * i + c] = s;
      }
    v[0] = (det3(M) < 0.0) ? 1.0 : 0.0;
  }
  __shared__ double lds[kB / 64];
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// The rotation closest to M in the Frobenius norm (the SO(3) factor of its
// polar decomposition): eigenvectors b_i of M^T M by decreasing eigenvalue,
// a_i = M b_i / |M b_i| for the two largest (Gram-Schmidt), a_3 = a_1 x a_2,
// R = a_1 b_1^T + a_2 b_2^T + det(B) a_3 b_3^T.  Exact when the smallest
// singular value of M vanishes; for M of rank 1, one of the closest rotations.
__device__ void so3_project(const double (&M)[3][3], double (&Rm)[3][3]) {
  double S[3][3], B[3][3];
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) S[p][q] = M[0][p] * M[0][q] + M[1][p] * M[1][q] + M[2][p] * M[2][q];
  jacobi_eig<3>(S, B, 3);
  int idx[3] = {0, 1, 2};
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (S[idx[j]][idx[j]] > S[idx[i]][idx[i]]) {
        const int t = idx[i];
        idx[i] = idx[j];
        idx[j] = t;
      }
  double b[3][3];  // columns b_i sorted by decreasing singular value
  for (int i = 0; i < 3; ++i)
    for (int p = 0; p < 3; ++p) b[i][p] = B[p][idx[i]];
  double a1[3], a2[3];
  for (int p = 0; p < 3; ++p) {
    a1[p] = M[p][0] * b[0][0] + M[p][1] * b[0][1] + M[p][2] * b[0][2];
    a2[p] = M[p][0] * b[1][0] + M[p][1] * b[1][1] + M[p][2] * b[1][2];
  }
  double n1 = sqrt(a1[0] * a1[0] + a1[1] * a1[1] + a1[2] * a1[2]);
  for (int p = 0; p < 3; ++p) a1[p] /= n1;
  const double d12 = a1[0] * a2[0] + a1[1] * a2[1] + a1[2] * a2[2];
  for (int p = 0; p < 3; ++p) a2[p] -= d12 * a1[p];
  double n2 = sqrt(a2[0] * a2[0] + a2[1] * a2[1] + a2[2] * a2[2]);
  if (!(n2 > 1e-13 * n1)) {
    // M of rank 1: every rotation taking b_1 to a_1 is closest; complete a_1
    // by the unit vector orthogonal to it from the axis least aligned with it
    int e = 0;
    for (int p = 1; p < 3; ++p)
      if (fabs(a1[p]) < fabs(a1[e])) e = p;
    for (int p = 0; p < 3; ++p) a2[p] = ((p == e) ? 1.0 : 0.0) - a1[e] * a1[p];
    n2 = sqrt(a2[0] * a2[0] + a2[1] * a2[1] + a2[2] * a2[2]);
  }
  for (int p = 0; p < 3; ++p) a2[p] /= n2;
  const double a3[3] = {a1[1] * a2[2] - a1[2] * a2[1], a1[2] * a2[0] - a1[0] * a2[2], a1[0] * a2[1] - a1[1] * a2[0]};
  double Bm[3][3];
  for (int p = 0; p < 3; ++p)
    for (int i = 0; i < 3; ++i) Bm[p][i] = b[i][p];
  const double detB = det3(Bm) < 0.0 ? -1.0 : 1.0;
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) Rm[p][q] = a1[p] * b[0][q] + a2[p] * b[1][q] + detB * a3[p] * b[2][q];
}

__global__ __launch_bounds__(kB) void polar_kernel(int32_t N, const double* __restrict__ Ub, int flip,
                                                   double* __restrict__ Rk, double* __restrict__ sk) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  double M[3][3];
  for (int i = 0; i < 3; ++i)
    for (int c = 0; c < 3; ++c) M[i][c] = Ub[9 * static_cast<int64_t>(k) + 3 * i + c] * ((flip && i == 2) ? -1.0 : 1.0);
  double Rm[3][3];
  so3_project(M, Rm);
  double tr = 0.0;
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) tr += Rm[p][q] * M[p][q];
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) Rk[9 * static_cast<int64_t>(k) + 3 * p + q] = Rm[p][q];
  sk[k] = tr / 3.0;
}

// R_out[k] = R_0^T R_k (row-major), s_out[k] = s_k / s_0, Ut (Yt layout, r = 3) = s_out R_out
__global__ void anchor_kernel(int32_t N, const double* __restrict__ Rk, const double* __restrict__ sk,
                              double* __restrict__ R_out, double* __restrict__ s_out, double* __restrict__ Ut) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  double A[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int p = 0; p < 3; ++p) s += Rk[3 * p + i] * Rk[9 * static_cast<int64_t>(k) + 3 * p + j];
      A[i][j] = s;
    }
  const double sc = sk[k] / sk[0];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R_out[9 * static_cast<int64_t>(k) + 3 * i + j] = A[i][j];
  s_out[k] = sc;
  for (int c = 0; c < 3; ++c)
    for (int a = 0; a < 3; ++a) Ut[(3 * static_cast<int64_t>(k) + c) * 3 + a] = sc * A[a][c];
}

__global__ __launch_bounds__(kB) void dot_kernel(const double* __restrict__ a, const double* __restrict__ b,
                                                 int64_t n, double* part) {
  double v[1] = {0.0};
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x; i < n; i += static_cast<int64_t>(gridDim.x) * kB)
    v[0] += a[i] * b[i];
  __shared__ double lds[kB / 64];
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

template <int R>
void launch_gram(const double* Yt, int64_t n, double* part, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((gram_mfma_kernel<R>), dim3(blocks), dim3(kB), 0, s, Yt, n, part);
  XM_LAUNCH_CHECK("gram_mfma_kernel");
}

}  // namespace

void round_yt(xm_problem* p, const double* Y, int r, double* R_out, double* s_out, double* rho_hat,
              hipStream_t s) {
  require(r >= 3 && r <= 8, XM_EINVAL, "rounding: rank must be in [3, 8]");
  require(Y && R_out && s_out, XM_EINVAL, "rounding: NULL pointer");
  const int N = p->N;
  const int64_t n = p->n3;
  DevBuf<double> Yt(n * r);
  transpose_rows<double, double>(Y, r, static_cast<int>(n), Yt.ptr, s);
  const int blocks = 64;
  const int nwaves = blocks * (kB / 64);
  DevBuf<double> part(static_cast<size_t>(nwaves) * 256), V3(24), mu(8);
  switch (r) {
    case 3: launch_gram<3>(Yt.ptr, n, part.ptr, blocks, s); break;
    case 4: launch_gram<4>(Yt.ptr, n, part.ptr, blocks, s); break;
    case 5: launch_gram<5>(Yt.ptr, n, part.ptr, blocks, s); break;
    case 6: launch_gram<6>(Yt.ptr, n, part.ptr, blocks, s); break;
    case 7: launch_gram<7>(Yt.ptr, n, part.ptr, blocks, s); break;
    case 8: launch_gram<8>(Yt.ptr, n, part.ptr, blocks, s); break;
  }
  hipLaunchKernelGGL(gram_eig_kernel, dim3(1), dim3(kB), 0, s, part.ptr, nwaves, r, V3.ptr, mu.ptr);
  XM_LAUNCH_CHECK("gram_eig_kernel");
  const unsigned fb = cdiv(N, kB);
  DevBuf<double> Ub(9 * static_cast<size_t>(N)), Rk(9 * static_cast<size_t>(N)), sk(N), dpart(fb);
  hipLaunchKernelGGL(project_kernel, dim3(fb), dim3(kB), 0, s, N, r, Yt.ptr, V3.ptr, Ub.ptr, dpart.ptr);
  XM_LAUNCH_CHECK("project_kernel");
  double nneg = 0.0;
  read_partials(dpart.ptr, fb, 1, &nneg, s);
  const int flip = (nneg > 0.5 * N) ? 1 : 0;
  hipLaunchKernelGGL(polar_kernel, dim3(fb), dim3(kB), 0, s, N, Ub.ptr, flip, Rk.ptr, sk.ptr);
  XM_LAUNCH_CHECK("polar_kernel");
  DevBuf<double> Ut(n * 3), G(n * 3);
  hipLaunchKernelGGL(anchor_kernel, dim3(fb), dim3(kB), 0, s, N, Rk.ptr, sk.ptr, R_out, s_out, Ut.ptr);
  XM_LAUNCH_CHECK("anchor_kernel");
  if (rho_hat) {
    spmm_yt<double>(p, XM_F64, Ut.ptr, 3, G.ptr, s);
    const int db = 64;
    DevBuf<double> pp(db);
    hipLaunchKernelGGL(dot_kernel, dim3(db), dim3(kB), 0, s, Ut.ptr, G.ptr, n * 3, pp.ptr);
    XM_LAUNCH_CHECK("dot_kernel");
    read_partials(pp.ptr, db, 1, rho_hat, s);
    if (p->scale_reg != 0.0) {  // + lam sum_{k>=1} (s_k^2 - 1)^2 of the rounded scales
      std::vector<double> hs(N);
      XM_HIP(hipMemcpyAsync(hs.data(), s_out, N * sizeof(double), hipMemcpyDeviceToHost, s));
      XM_HIP(hipStreamSynchronize(s));
      double F = 0.0;
      for (int k = 1; k < N; ++k) F += (hs[k] * hs[k] - 1.0) * (hs[k] * hs[k] - 1.0);
      *rho_hat += p->scale_reg * F;
    }
  }
  XM_HIP(hipStreamSynchronize(s));
}


namespace {

// Similarity alignment: (s, R, t) minimising sum_i w_i |s R p_i + t - q_i|^2
// (the registration of estimated camera positions to a reference before
// trajectory errors).  One workgroup (the point count is a frame count): pass 1
// the weighted means, pass 2 the centred spread and cross-covariance C, then
// R = the rotation closest to C, s = tr(R^T C) / spread, t = mu_q - s R mu_p;
// pass 3 the weighted squared residual.  Fixed-order sums: deterministic.
// out: s, R (row-major), t, rmse, then the weight sum, the spread and the
// count of invalid inputs (negative or non-finite weights, non-finite points).
__global__ __launch_bounds__(kB) void align_kernel(int64_t n, const double* __restrict__ P,
                                                   const double* __restrict__ Q, const double* __restrict__ w,
                                                   double* __restrict__ out) {
  __shared__ double lds[10 * (kB / 64)];
  __shared__ double par[20];  // mu_p, mu_q, W, then s, R (row-major), t after pass 2
  double v1[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = threadIdx.x; i < n; i += kB) {
    const double wi = w ? w[i] : 1.0;
    bool bad = !(wi >= 0.0) || !isfinite(wi);
    for (int c = 0; c < 3; ++c) bad = bad || !isfinite(P[3 * i + c]) || !isfinite(Q[3 * i + c]);
    if (bad) {
      v1[7] += 1.0;
      continue;
    }
    v1[0] += wi;
    for (int c = 0; c < 3; ++c) {
      v1[1 + c] += wi * P[3 * i + c];
      v1[4 + c] += wi * Q[3 * i + c];
    }
  }
  block_sum<8>(v1, lds);
  if (threadIdx.x == 0) {
    for (int c = 0; c < 6; ++c) par[c] = v1[1 + c] / v1[0];
    par[6] = v1[0];
    out[16] = v1[7];
  }
  __syncthreads();
  double v2[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = threadIdx.x; i < n; i += kB) {
    const double wi = w ? w[i] : 1.0;
    double pc[3], qc[3];
    for (int c = 0; c < 3; ++c) {
      pc[c] = P[3 * i + c] - par[c];
      qc[c] = Q[3 * i + c] - par[3 + c];
    }
    v2[0] += wi * (pc[0] * pc[0] + pc[1] * pc[1] + pc[2] * pc[2]);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) v2[1 + 3 * a + b] += wi * qc[a] * pc[b];
  }
  block_sum<10>(v2, lds);
  if (threadIdx.x == 0) {
    const double W = par[6], sigma2 = v2[0] / W;
    double C[3][3], Rm[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) C[a][b] = v2[1 + 3 * a + b] / W;
    so3_project(C, Rm);
    double tr = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) tr += Rm[a][b] * C[a][b];
    const double sc = tr / sigma2;
    par[7] = sc;
    for (int a = 0; a < 3; ++a) {
      double rm = 0.0;
      for (int b = 0; b < 3; ++b) {
        par[8 + 3 * a + b] = Rm[a][b];
        rm += Rm[a][b] * par[b];
      }
      par[17 + a] = par[3 + a] - sc * rm;
    }
    for (int k = 0; k < 13; ++k) out[k] = par[7 + k];
    out[14] = W;
    out[15] = sigma2;
  }
  __syncthreads();
  const double sc = par[7];
  double Rm[3][3], t[3];
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b) Rm[a][b] = par[8 + 3 * a + b];
    t[a] = par[17 + a];
  }
  double v3[1] = {0.0};
  for (int64_t i = threadIdx.x; i < n; i += kB) {
    const double wi = w ? w[i] : 1.0;
    double e2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double r = sc * (Rm[a][0] * P[3 * i] + Rm[a][1] * P[3 * i + 1] + Rm[a][2] * P[3 * i + 2]) + t[a] -
                       Q[3 * i + a];
      e2 += r * r;
    }
    v3[0] += wi * e2;
  }
  block_sum<1>(v3, lds);
  if (threadIdx.x == 0) out[13] = sqrt(v3[0] / par[6]);
}

}  // namespace

void align_similarity(int64_t n, const double* P, const double* Q, const double* w, double* out, hipStream_t s) {
  require(n >= 1, XM_EINVAL, "alignment: n must be >= 1");
  require(P && Q && out, XM_EINVAL, "alignment: NULL argument");
  DevBuf<double> o(17);
  hipLaunchKernelGGL(align_kernel, dim3(1), dim3(kB), 0, s, n, P, Q, w, o.ptr);
  XM_LAUNCH_CHECK("align_kernel");
  double h[17];
  XM_HIP(hipMemcpyAsync(h, o.ptr, sizeof(h), hipMemcpyDeviceToHost, s));
  XM_HIP(hipStreamSynchronize(s));
  require(h[16] == 0.0, XM_EINVAL, "alignment: weights must be finite and >= 0, points finite");
  require(h[14] > 0.0, XM_EINVAL, "alignment: the weights sum to zero");
  require(h[15] > 0.0, XM_EINVAL, "alignment: the points to align have no spread");
  for (int k = 0; k < 14; ++k) out[k] = h[k];
}

}  // namespace xm
