// Recovery of translations and landmarks (eq. tpstar) and the adjoint of the
// certified optimum with respect to the lifted keypoints u_o and weights w_o.
//
// Recovery at a factor U (r = 3 rows, frame 0 anchored):
//   t[1:] = -A_tt[1:,1:]^{-1} A_rt[:,1:]^T U^T   (the stored -G^{-1} times the
//           transposed A_rt pattern applied to U),  t_0 = 0,
//   p_k   = (1/W_k) sum_{o in k} w_o (U_i u_o + t_i)   (weighted landmark mean).
//
// Adjoint (envelope theorem for the cost, implicit-function theorem for the
// rotations and scales in the chart where frame 0 is fixed):
//   residuals e_o = U_i u_o + t_i - p_k;
//   df*/du_o = 2 w_o U_i^T e_o,  df*/dw_o = |e_o|^2;
//   H lam = grad l (CG on the anchored Riemannian Hessian, same product and
//   per-frame kernels as the solver), Udot_k = lam_s,k R_k + s_k lam_R,k,
//   e^lam_o from (Udot, t^lam, p^lam) recovered like (U, t, p);
//   dl/du_o = -2 w_o (U_i^T e^lam_o + Udot_i^T e_o),  dl/dw_o = -2 <e_o, e^lam_o>.
#include <cmath>
#include <vector>

#include "manifold.h"
#include "problem.h"

namespace xm {
namespace {

constexpr int kB = 256;

// Rt / Yt (rank 3, frame-major) from row-major R [N][3][3] and s [N]
__global__ void from_rs_kernel(int32_t N, const double* __restrict__ R, const double* __restrict__ s,
                               double* __restrict__ Rt, double* __restrict__ sv, double* __restrict__ Yt) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  for (int c = 0; c < 3; ++c)
    for (int a = 0; a < 3; ++a) {
      const double v = R[9 * static_cast<int64_t>(k) + 3 * a + c];
      Rt[(3 * static_cast<int64_t>(k) + c) * 3 + a] = v;
      Yt[(3 * static_cast<int64_t>(k) + c) * 3 + a] = s[k] * v;
    }
  sv[k] = s[k];
}

// mirror[s] = position of (j, i) for the pattern entry s = (i, j)
__global__ void mirror_kernel(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int32_t N,
                              int32_t* __restrict__ mirror) {
  const int i = blockIdx.x;
  if (i >= N) return;
  for (int32_t s = row_ptr[i] + threadIdx.x; s < row_ptr[i + 1]; s += blockDim.x) {
    const int j = col[s];
    int32_t lo = row_ptr[j], hi = row_ptr[j + 1] - 1, pos = -1;
    while (lo <= hi) {
      const int32_t mid = (lo + hi) >> 1;
      const int c = col[mid];
      if (c == i) { pos = mid; break; }
      if (c < i) lo = mid + 1;
      else hi = mid - 1;
    }
    mirror[s] = pos;
  }
}

// b[j-1][a'] = sum_{i in nb(j)} sum_a A_rt[3i+a][j] Yt[(3i+a)*3 + a'],  j >= 1
__global__ void art_t_kernel(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                             const int32_t* __restrict__ mirror, const double* __restrict__ Art, int32_t N,
                             const double* __restrict__ Yt, double* __restrict__ b) {
  const int j = blockIdx.x * kB + threadIdx.x;
  if (j < 1 || j >= N) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int32_t s = row_ptr[j]; s < row_ptr[j + 1]; ++s) {
    const int i = col[s];
    const int32_t m = mirror[s];  // entry (i, j)
    for (int a = 0; a < 3; ++a) {
      const double v = Art[3 * static_cast<int64_t>(m) + a];
      for (int q = 0; q < 3; ++q) acc[q] += v * Yt[(3 * static_cast<int64_t>(i) + a) * 3 + q];
    }
  }
  for (int q = 0; q < 3; ++q) b[3 * static_cast<int64_t>(j - 1) + q] = acc[q];
}

// t[0] = 0; t[j][q] = sum_l Gm[j-1][l] b[l][q] (one block per row of -G^{-1})
__global__ __launch_bounds__(kB) void gm_apply_kernel(const double* __restrict__ Gm, int32_t ldg, int32_t ng,
                                                      const double* __restrict__ b, double* __restrict__ t) {
  const int j = blockIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  const double* g = Gm + static_cast<int64_t>(j) * ldg;
  for (int l = threadIdx.x; l < ng; l += kB) {
    const double gl = g[l];
    v[0] += gl * b[3 * l];
    v[1] += gl * b[3 * l + 1];
    v[2] += gl * b[3 * l + 2];
  }
  __shared__ double lds[3 * (kB / 64)];
  block_sum<3>(v, lds);
  if (threadIdx.x == 0) {
    if (j == 0) t[0] = t[1] = t[2] = 0.0;
    for (int q = 0; q < 3; ++q) t[3 * static_cast<int64_t>(j + 1) + q] = v[q];
  }
}

// p_k = (1/W_k) sum_o w_o (Y_i u_o + t_i)
__global__ void landmark_mean_kernel(const int64_t* __restrict__ lm_ptr, int32_t M, const int32_t* __restrict__ fr_s,
                                     const double* __restrict__ u_s, const double* __restrict__ w_s,
                                     const double* __restrict__ Wl, const double* __restrict__ Yt,
                                     const double* __restrict__ t, double* __restrict__ pk) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= M) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t o = lm_ptr[k]; o < lm_ptr[k + 1]; ++o) {
    const int64_t i = fr_s[o];
    const double* u = u_s + 3 * o;
    for (int q = 0; q < 3; ++q) {
      double v = t[3 * i + q];
      for (int c = 0; c < 3; ++c) v += Yt[(3 * i + c) * 3 + q] * u[c];
      acc[q] += w_s[o] * v;
    }
  }
  const double W = Wl[k];
  for (int q = 0; q < 3; ++q) pk[3 * static_cast<int64_t>(k) + q] = (W > 0.0) ? acc[q] / W : 0.0;
}

__device__ __forceinline__ void residual(int64_t o, const int32_t* fr_s, const int32_t* lm_s, const double* u_s,
                                         const double* Yt, const double* t, const double* pk, double (&e)[3]) {
  const int64_t i = fr_s[o], k = lm_s[o];
  const double* u = u_s + 3 * o;
  for (int q = 0; q < 3; ++q) {
    double v = t[3 * i + q] - pk[3 * k + q];
    for (int c = 0; c < 3; ++c) v += Yt[(3 * i + c) * 3 + q] * u[c];
    e[q] = v;
  }
}

template <typename TG>
__global__ void obs_grad_kernel(int64_t n, const int32_t* __restrict__ fr_s, const int32_t* __restrict__ lm_s,
                                const double* __restrict__ u_s, const double* __restrict__ w_s,
                                const int64_t* __restrict__ perm, const double* __restrict__ Yt,
                                const double* __restrict__ t, const double* __restrict__ pk,
                                const double* __restrict__ Yd, const double* __restrict__ td,
                                const double* __restrict__ pd, double gcost, double rot_coef,
                                TG* __restrict__ gu, TG* __restrict__ gw) {
  const int64_t o = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (o >= n) return;
  const int64_t i = fr_s[o];
  const double w = w_s[o];
  double e[3];
  residual(o, fr_s, lm_s, u_s, Yt, t, pk, e);
  double g_u[3], g_w;
  // cost part: gcost * (2 w U_i^T e, |e|^2)
  for (int c = 0; c < 3; ++c) {
    double v = 0.0;
    for (int q = 0; q < 3; ++q) v += Yt[(3 * i + c) * 3 + q] * e[q];
    g_u[c] = gcost * 2.0 * w * v;
  }
  g_w = gcost * (e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
  if (rot_coef != 0.0) {
    // (Yd, td, pd) describe the direction eta = -lam, so rot_coef = +1 turns
    // -2 w (U^T e^lam + Udot^T e) into +2 w (U^T e^eta + Ueta^T e)
    double el[3];
    residual(o, fr_s, lm_s, u_s, Yd, td, pd, el);
    for (int c = 0; c < 3; ++c) {
      double v = 0.0;
      for (int q = 0; q < 3; ++q) v += Yt[(3 * i + c) * 3 + q] * el[q] + Yd[(3 * i + c) * 3 + q] * e[q];
      g_u[c] += rot_coef * 2.0 * w * v;
    }
    g_w += rot_coef * 2.0 * (e[0] * el[0] + e[1] * el[1] + e[2] * el[2]);
  }
  const int64_t orig = perm[o];
  for (int c = 0; c < 3; ++c) gu[3 * orig + c] = static_cast<TG>(g_u[c]);
  gw[orig] = static_cast<TG>(g_w);
}

// residual export: e_o and its score in the caller's order (perm)
__global__ void residual_out_kernel(int64_t n, const int32_t* __restrict__ fr_s, const int32_t* __restrict__ lm_s,
                                    const double* __restrict__ u_s, const int64_t* __restrict__ perm,
                                    const double* __restrict__ Yt, const double* __restrict__ t,
                                    const double* __restrict__ pk, const double* __restrict__ s, int frame_units,
                                    double* __restrict__ e_out, double* __restrict__ score_out) {
  const int64_t o = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (o >= n) return;
  double e[3];
  residual(o, fr_s, lm_s, u_s, Yt, t, pk, e);
  const int64_t orig = perm[o];
  if (e_out)
    for (int q = 0; q < 3; ++q) e_out[3 * orig + q] = e[q];
  if (score_out) {
    const double nrm = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    score_out[orig] = frame_units ? nrm / s[fr_s[o]] : nrm;
  }
}

template <typename T>
__global__ void fill_kernel(int64_t n, T v, T* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (i < n) out[i] = v;
}

// b = Riemannian gradient of l in the anchored chart: P_R(gR) (Stiefel), s^2 gs; frame 0 zero
__global__ void rgrad_loss_kernel(int32_t N, const double* __restrict__ Rt, const double* __restrict__ s,
                                  const double* __restrict__ gR, const double* __restrict__ gs,
                                  double* __restrict__ bR, double* __restrict__ bs) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  double Rm[3][3], G[3][3];  // Rm[a][c] = R_k[a][c]
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) {
      Rm[a][c] = Rt[(3 * static_cast<int64_t>(k) + c) * 3 + a];
      G[a][c] = gR ? gR[9 * static_cast<int64_t>(k) + 3 * a + c] : 0.0;
    }
  double S[3][3];
  for (int c = 0; c < 3; ++c)
    for (int d = 0; d < 3; ++d) {
      double v = 0.0;
      for (int a = 0; a < 3; ++a) v += Rm[a][c] * G[a][d];
      S[c][d] = v;
    }
  for (int c = 0; c < 3; ++c)
    for (int d = c + 1; d < 3; ++d) S[c][d] = S[d][c] = 0.5 * (S[c][d] + S[d][c]);
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) {
      double v = G[a][c];
      for (int d = 0; d < 3; ++d) v -= Rm[a][d] * S[d][c];
      bR[(3 * static_cast<int64_t>(k) + c) * 3 + a] = (k == 0) ? 0.0 : v;
    }
  bs[k] = (k == 0 || !gs) ? 0.0 : s[k] * s[k] * gs[k];
}

struct Recovered {
  DevBuf<double> t, pk;
};

void recover(xm_problem* p, const double* Yt, const int32_t* mirror, Recovered& out, hipStream_t st) {
  const int N = p->N, M = p->M, ng = N - 1;
  DevBuf<double> b(3 * static_cast<size_t>(ng) + 3);
  out.t.ensure(3 * static_cast<size_t>(N));
  out.pk.ensure(3 * static_cast<size_t>(M));
  hipLaunchKernelGGL(art_t_kernel, dim3(cdiv(N, kB)), dim3(kB), 0, st, p->row_ptr.ptr, p->col.ptr, mirror,
                     p->Art.ptr, N, Yt, b.ptr);
  XM_LAUNCH_CHECK("art_t_kernel");
  hipLaunchKernelGGL(gm_apply_kernel, dim3(ng), dim3(kB), 0, st, p->Gm.ptr, p->ldg, ng, b.ptr, out.t.ptr);
  XM_LAUNCH_CHECK("gm_apply_kernel");
  hipLaunchKernelGGL(landmark_mean_kernel, dim3(cdiv(M, kB)), dim3(kB), 0, st, p->lm_ptr.ptr, M, p->fr_s.ptr,
                     p->u_s.ptr, p->w_s.ptr, p->Wl.ptr, Yt, out.t.ptr, out.pk.ptr);
  XM_LAUNCH_CHECK("landmark_mean_kernel");
  XM_HIP(hipStreamSynchronize(st));
}

DevBuf<int32_t> build_mirror(xm_problem* p, hipStream_t st) {
  DevBuf<int32_t> m(p->nnzb);
  hipLaunchKernelGGL(mirror_kernel, dim3(p->N), dim3(64), 0, st, p->row_ptr.ptr, p->col.ptr, p->N, m.ptr);
  XM_LAUNCH_CHECK("mirror_kernel");
  return m;
}

}  // namespace

void recover_tp(xm_problem* p, const double* R, const double* s, double* t_out, double* p_out, hipStream_t st) {
  require(R && s, XM_EINVAL, "R and s must be non-NULL");
  const int N = p->N;
  DevBuf<double> Rt(9 * static_cast<size_t>(N)), sv(N), Yt(9 * static_cast<size_t>(N));
  hipLaunchKernelGGL(from_rs_kernel, dim3(cdiv(N, kB)), dim3(kB), 0, st, N, R, s, Rt.ptr, sv.ptr, Yt.ptr);
  XM_LAUNCH_CHECK("from_rs_kernel");
  DevBuf<int32_t> mirror = build_mirror(p, st);
  Recovered rec;
  recover(p, Yt.ptr, mirror.ptr, rec, st);
  if (t_out) XM_HIP(hipMemcpyAsync(t_out, rec.t.ptr, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (p_out) XM_HIP(hipMemcpyAsync(p_out, rec.pk.ptr, 3 * static_cast<size_t>(p->M) * sizeof(double),
                                   hipMemcpyDeviceToDevice, st));
  XM_HIP(hipStreamSynchronize(st));
}

void residuals(xm_problem* p, const double* R, const double* s, int frame_units, double* e_out, double* score_out,
               hipStream_t st) {
  require(R && s, XM_EINVAL, "R and s must be non-NULL");
  require(e_out || score_out, XM_EINVAL, "at least one of e and score must be non-NULL");
  const int N = p->N;
  DevBuf<double> Rt(9 * static_cast<size_t>(N)), sv(N), Yt(9 * static_cast<size_t>(N));
  hipLaunchKernelGGL(from_rs_kernel, dim3(cdiv(N, kB)), dim3(kB), 0, st, N, R, s, Rt.ptr, sv.ptr, Yt.ptr);
  XM_LAUNCH_CHECK("from_rs_kernel");
  DevBuf<int32_t> mirror = build_mirror(p, st);
  Recovered rec;
  recover(p, Yt.ptr, mirror.ptr, rec, st);
  if (p->n_in > p->n_obs) {  // observations the build's mask left out
    if (e_out)
      hipLaunchKernelGGL((fill_kernel<double>), dim3(cdiv(3 * p->n_in, kB)), dim3(kB), 0, st, 3 * p->n_in, 0.0,
                         e_out);
    if (score_out)
      hipLaunchKernelGGL((fill_kernel<double>), dim3(cdiv(p->n_in, kB)), dim3(kB), 0, st, p->n_in, 0.0, score_out);
    XM_LAUNCH_CHECK("fill_kernel");
  }
  const int64_t n = p->n_obs;
  hipLaunchKernelGGL(residual_out_kernel, dim3(cdiv(n, kB)), dim3(kB), 0, st, n, p->fr_s.ptr, p->lm_s.ptr,
                     p->u_s.ptr, p->perm.ptr, Yt.ptr, rec.t.ptr, rec.pk.ptr, sv.ptr, frame_units, e_out, score_out);
  XM_LAUNCH_CHECK("residual_out_kernel");
  XM_HIP(hipStreamSynchronize(st));
}

AdjointResult adjoint(xm_problem* p, const double* R, const double* s, const double* gR, const double* gs,
                      double gcost, void* gu, void* gw, xm_dtype gdt, double cg_tol, int cg_max, hipStream_t st) {
  require(R && s && gu && gw, XM_EINVAL, "R, s, gu and gw must be non-NULL");
  require(p->scale_reg == 0.0, XM_EINVAL, "the adjoint is not available with the scale regulariser");
  require(gdt == XM_F64 || gdt == XM_F32, XM_EINVAL, "gradient dtype must be XM_F64 or XM_F32");
  const int N = p->N;
  const int64_t n3 = p->n3;
  if (cg_tol <= 0) cg_tol = 1e-10;
  if (cg_max <= 0) cg_max = 4 * N;
  AdjointResult res;
  const size_t nv = 9 * static_cast<size_t>(N);
  DevBuf<double> Rt(nv), sv(N), Yt(nv), G(nv), gR_(nv), gs_(N), Sc(nv), ec(N);
  DevBuf<double> bR(nv), bs(N), etaR(nv), etas(N), HetaR(nv), Hetas(N), resR(nv), ress(N), dR(nv), ds(N);
  DevBuf<double> HdR(nv), Hds(N), Ydot(nv), Gd(nv), part(static_cast<size_t>(cdiv(N, kFrameBlock)) * 8);
  Manifold<double> mf(N);
  const int nb = static_cast<int>(mf.blocks());
  hipLaunchKernelGGL(from_rs_kernel, dim3(cdiv(N, kB)), dim3(kB), 0, st, N, R, s, Rt.ptr, sv.ptr, Yt.ptr);
  XM_LAUNCH_CHECK("from_rs_kernel");
  DevBuf<int32_t> mirror = build_mirror(p, st);
  Recovered rec, recl;
  recover(p, Yt.ptr, mirror.ptr, rec, st);
  const bool with_rot = (gR != nullptr) || (gs != nullptr);
  if (with_rot) {
    // caches of the Hessian at (R, s): G = Q Yt, S_k, e_k
    spmm_yt<double>(p, XM_F64, Yt.ptr, 3, G.ptr, st);
    mf.grad(3, Rt.ptr, sv.ptr, G.ptr, gR_.ptr, gs_.ptr, Sc.ptr, ec.ptr, part.ptr, st);
    double sums[5];
    read_partials(part.ptr, nb, 5, sums, st);
    res.cost = sums[0];
    // right-hand side and CG (the truncated-CG kernels without a trust region):
    // res_0 = b, d = -res, eta += alpha d, res += alpha H d  =>  eta = -H^{-1} b
    hipLaunchKernelGGL(rgrad_loss_kernel, dim3(cdiv(N, kB)), dim3(kB), 0, st, N, Rt.ptr, sv.ptr, gR, gs, bR.ptr,
                       bs.ptr);
    XM_LAUNCH_CHECK("rgrad_loss_kernel");
    XM_HIP(hipMemsetAsync(etaR.ptr, 0, nv * sizeof(double), st));
    XM_HIP(hipMemsetAsync(etas.ptr, 0, N * sizeof(double), st));
    XM_HIP(hipMemsetAsync(HetaR.ptr, 0, nv * sizeof(double), st));
    XM_HIP(hipMemsetAsync(Hetas.ptr, 0, N * sizeof(double), st));
    XM_HIP(hipMemcpyAsync(resR.ptr, bR.ptr, nv * sizeof(double), hipMemcpyDeviceToDevice, st));
    XM_HIP(hipMemcpyAsync(ress.ptr, bs.ptr, N * sizeof(double), hipMemcpyDeviceToDevice, st));
    double b2 = vec_dot<double>(bR.ptr, bR.ptr, static_cast<int64_t>(nv), part.ptr, 8, st);
    {
      // metric part of |b|^2 for the scale components
      std::vector<double> hb(N), hs(N);
      XM_HIP(hipMemcpyAsync(hb.data(), bs.ptr, N * sizeof(double), hipMemcpyDeviceToHost, st));
      XM_HIP(hipMemcpyAsync(hs.data(), sv.ptr, N * sizeof(double), hipMemcpyDeviceToHost, st));
      XM_HIP(hipStreamSynchronize(st));
      for (int k = 1; k < N; ++k) b2 += hb[k] * hb[k] / (hs[k] * hs[k]);
    }
    double r_r = b2;
    const double stop = cg_tol * std::sqrt(b2);
    int mode = 0, j = 0;
    double beta = 0.0;
    if (b2 > 0.0) {
      for (j = 1; j <= cg_max; ++j) {
        mf.ydot(3, Rt.ptr, sv.ptr, resR.ptr, ress.ptr, dR.ptr, ds.ptr, beta, mode, Ydot.ptr, st);
        spmm_yt<double>(p, XM_F64, Ydot.ptr, 3, Gd.ptr, st, XM_ROLE_CURVATURE);
        mf.hess(3, Rt.ptr, sv.ptr, G.ptr, Sc.ptr, ec.ptr, dR.ptr, ds.ptr, Gd.ptr, etaR.ptr, etas.ptr, HdR.ptr,
                Hds.ptr, part.ptr, st, true);
        read_partials(part.ptr, nb, 4, sums, st);
        // the Hessian of a certified, tight optimum is positive definite in the
        // anchored chart; a direction of non-positive curvature means the point
        // is not one, and CG cannot continue
        if (!(sums[0] > 0.0)) {
          res.negative_curvature = true;
          break;
        }
        const double alpha = r_r / sums[0];
        mf.tcg_update(3, sv.ptr, alpha, 0, dR.ptr, ds.ptr, HdR.ptr, Hds.ptr, etaR.ptr, etas.ptr, HetaR.ptr,
                      Hetas.ptr, resR.ptr, ress.ptr, part.ptr, st);
        double rr[2];
        read_partials(part.ptr, nb, 2, rr, st);
        res.cg_residual = std::sqrt(rr[0]) / std::sqrt(b2);
        if (std::sqrt(rr[0]) <= stop) break;
        beta = rr[0] / r_r;
        r_r = rr[0];
        mode = 1;
      }
    }
    res.cg_iters = std::min(j, cg_max);
    res.converged = !res.negative_curvature && (b2 == 0.0 || res.cg_residual <= cg_tol);
    // lam = -eta; the direction passed on is eta itself: Ueta = eta_s R + s eta_R = -Udot
    mf.ydot(3, Rt.ptr, sv.ptr, resR.ptr, ress.ptr, etaR.ptr, etas.ptr, 0.0, 2, Ydot.ptr, st);
    recover(p, Ydot.ptr, mirror.ptr, recl, st);
  }
  const int64_t n = p->n_obs;
  if (p->n_in > n) {  // observations the build's mask left out get zero gradients
    if (gdt == XM_F64) {
      hipLaunchKernelGGL((fill_kernel<double>), dim3(cdiv(3 * p->n_in, kB)), dim3(kB), 0, st, 3 * p->n_in, 0.0,
                         static_cast<double*>(gu));
      hipLaunchKernelGGL((fill_kernel<double>), dim3(cdiv(p->n_in, kB)), dim3(kB), 0, st, p->n_in, 0.0,
                         static_cast<double*>(gw));
    } else {
      hipLaunchKernelGGL((fill_kernel<float>), dim3(cdiv(3 * p->n_in, kB)), dim3(kB), 0, st, 3 * p->n_in, 0.0f,
                         static_cast<float*>(gu));
      hipLaunchKernelGGL((fill_kernel<float>), dim3(cdiv(p->n_in, kB)), dim3(kB), 0, st, p->n_in, 0.0f,
                         static_cast<float*>(gw));
    }
    XM_LAUNCH_CHECK("fill_kernel");
  }
  const double* Yd = with_rot ? Ydot.ptr : Yt.ptr;
  const double* td = with_rot ? recl.t.ptr : rec.t.ptr;
  const double* pd = with_rot ? recl.pk.ptr : rec.pk.ptr;
  if (gdt == XM_F64)
    hipLaunchKernelGGL((obs_grad_kernel<double>), dim3(cdiv(n, kB)), dim3(kB), 0, st, n, p->fr_s.ptr, p->lm_s.ptr,
                       p->u_s.ptr, p->w_s.ptr, p->perm.ptr, Yt.ptr, rec.t.ptr, rec.pk.ptr, Yd, td, pd, gcost,
                       with_rot ? 1.0 : 0.0, static_cast<double*>(gu), static_cast<double*>(gw));
  else
    hipLaunchKernelGGL((obs_grad_kernel<float>), dim3(cdiv(n, kB)), dim3(kB), 0, st, n, p->fr_s.ptr, p->lm_s.ptr,
                       p->u_s.ptr, p->w_s.ptr, p->perm.ptr, Yt.ptr, rec.t.ptr, rec.pk.ptr, Yd, td, pd, gcost,
                       with_rot ? 1.0 : 0.0, static_cast<float*>(gu), static_cast<float*>(gw));
  XM_LAUNCH_CHECK("obs_grad_kernel");
  XM_HIP(hipStreamSynchronize(st));
  (void)n3;
  return res;
}

}  // namespace xm
