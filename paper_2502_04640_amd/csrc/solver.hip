// Riemannian staircase (Algorithm "Riemannian Staircase") with a trust-region
// / truncated-CG local optimiser (Absil et al. 2008; Boumal 2023), driven from
// the host, all vector work in the kernels of manifold.hip / spmm.hip.
//
// tCG is preconditioned (option, on by default) by the per-frame scalar
// M_k = s_k^2 tr(Q_kk)/3 (normalised to mean 1; 3 M_k on the scale part),
// the diagonal of the Hessian with each 3x3 diagonal block of Q replaced by a
// multiple of I: it equalises the curvature of frames whose scales and
// observation counts differ by orders of magnitude; the trust region is then
// measured in the M-norm (Steihaug-Toint with a preconditioner).
//
// Parameters the paper leaves open (textbook defaults): tCG stops at
// |r| <= |r0| min(|r0|^theta, kappa), kappa = 0.1, theta = 1; steps are
// accepted when rho > 0.1; the radius is quartered when rho < 1/4 and doubled
// (up to sqrt(3N)) when rho > 3/4 on a boundary step; initial radius
// sqrt(3N)/8; rho carries the usual max(1,|f|) 1e3 eps regularisation.
// Stop when |grad| <= grad_tol qbar |Y|, or, at the precision floor of
// reduced-precision products, after 6 rejected steps in a row with |grad|
// within 30 grad_tol qbar |Y|, or after 12 rejected steps in a row at any
// gradient (stagnation).  A reduced-precision solve then continues from
// that point in an FP64 stage: the iterate, the manifold arithmetic and the
// gradient products in FP64, the truncated-CG Hessian-vector products in
// FP32 (an inexact-Newton / iterative-refinement split:
// the model only steers the step, the FP64 gradient decides where it ends),
// down to the FP64 tolerance.  An FP32 iterate cannot get closer to the
// optimum than its own rounding, whose gradient (about |Q| 6e-8 |Y|) is far
// above what the dual certificate needs.  The candidate's cost change is
// evaluated as <Y+ - Y, Q (Y+ + Y)> from the two products already computed,
// which stays accurate where f(Y+) - f(Y) would cancel.  The staircase escape
// follows Theorem "Descent Direction": block k of [Y; alpha v^T] is
// re-orthonormalised (scale kept), alpha halved until the cost drops, at most
// 40 times.  It is taken only when the dual has a negative direction off
// rows(Y): when the certificate's bound fails through its stationarity terms
// alone, the point is instead polished at the same rank with a 10x tighter
// gradient tolerance (up to three times; FP64 Hessian products).
#include <chrono>
#include <cmath>
#include <memory>
#include <cstdio>
#include <type_traits>
#include <vector>

#include "manifold.h"
#include "problem.h"

namespace xm {
namespace {

template <typename T>
struct Vecs {
  int N, rmax;
  size_t nv;
  DevBuf<T> Rt, s, Yt, G, Rt2, s2, Yt2, G2, gR, gs, Sc, ec;
  DevBuf<T> etaR, etas, HetaR, Hetas, resR, ress, dR, ds, HdR, Hds, Ydot, Gd;
  DevBuf<double> part;
  Vecs(int n, int rm) : N(n), rmax(rm), nv(static_cast<size_t>(3) * n * rm) {
    for (DevBuf<T>* b : {&Rt, &Yt, &G, &Rt2, &Yt2, &G2, &gR, &etaR, &HetaR, &resR, &dR, &HdR, &Ydot, &Gd})
      b->alloc(nv);
    for (DevBuf<T>* b : {&s, &s2, &gs, &ec, &etas, &Hetas, &ress, &ds, &Hds}) b->alloc(n);
    Sc.alloc(static_cast<size_t>(9) * n);
    part.alloc(static_cast<size_t>(cdiv(n, kFrameBlock)) * 8 + 8);
  }
};

template <typename T>
__global__ void sub_kernel(int64_t n, const T* __restrict__ a, const T* __restrict__ b, T* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}

// G64 = Gref + G (FP64); G <- G64 rounded (candidate products chained through the step)
template <typename T>
__global__ void combine_kernel(int64_t n, const double* __restrict__ Gref, T* __restrict__ G,
                               double* __restrict__ G64) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const double g = Gref[i] + static_cast<double>(G[i]);
  G64[i] = g;
  G[i] = static_cast<T>(g);
}

// start of a truncated-CG solve: eta = 0, H eta = 0, residual = gradient
// (rotation block of nvr values and scale block of N values, in one launch)
template <typename T>
__global__ void tcg_init_kernel(int64_t nvr, int32_t N, const T* __restrict__ gR, const T* __restrict__ gs,
                                T* __restrict__ etaR, T* __restrict__ etas, T* __restrict__ HetaR,
                                T* __restrict__ Hetas, T* __restrict__ resR, T* __restrict__ ress) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < nvr) {
    etaR[i] = T(0);
    HetaR[i] = T(0);
    resR[i] = gR[i];
  }
  if (i < N) {
    etas[i] = T(0);
    Hetas[i] = T(0);
    ress[i] = gs[i];
  }
}

template <typename T>
__global__ void widen_kernel(int64_t n, const T* __restrict__ a, double* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) out[i] = static_cast<double>(a[i]);
}

struct RtrOut {
  double f = 0, gnorm = 0, ynorm = 0, Delta = 0;
  int outer = 0, inner = 0, spmm = 0, accepted = 0;
  bool converged = false, floor = false;
};

template <typename T>
RtrOut rtr(xm_problem* p, Vecs<T>& V, int r, xm_dtype qg, xm_dtype qh, const xm_solve_opts& o, double grad_tol,
           hipStream_t st) {
  const int N = p->N;
  Manifold<T> mf(N);
  if (o.precondition) mf.qkk = p->qkk.ptr;
  mf.lam = p->scale_reg;
  const int nb = static_cast<int>(mf.blocks());
  const double qbar = p->qbar;
  const double Dbar = std::sqrt(3.0 * N);
  double Delta = (o.delta0 > 0) ? o.delta0 : Dbar / 8.0;
  const int max_outer = (o.max_outer > 0) ? o.max_outer : 1000;
  const int max_inner = (o.max_inner > 0) ? o.max_inner : std::min(3 * N * r, 2000);
  const double kappa = 0.1, theta = 1.0, rho_prime = 0.1;
  // precision floor: in reduced precision the gradient cannot fall below the
  // rounding noise of the products, and there every model step is rejected
  const int floor_rejections = 6;
  const double floor_tol = 30.0 * grad_tol;
  int rejections = 0;
  RtrOut out;
  double sums[5];

  mf.scale(r, V.Rt.ptr, V.s.ptr, V.Yt.ptr, st);
  // Candidate products from the step (when the curvature products are
  // factored): G(Y+) = G(Y) + Q (Y+ - Y), the product of the small difference
  // taken in the curvature role and added in FP64.  Its rounding scales with
  // |Y+ - Y|, so while the steps taken since the last full product sum to at
  // most kChainFrac |Y| the accumulated error stays at the level of one full
  // product; past that, a full product restarts the chain.
  constexpr double kChainFrac = 0.05;
  const size_t nvr0 = static_cast<size_t>(3) * N * r;
  const bool chain = p->spmm_kind[XM_ROLE_CURVATURE][qg] == XM_SPMM_FACTORED;
  DevBuf<T> dY;
  DevBuf<double> C64a, C64b;  // FP64 G at the current point and at the candidate
  double* Gc64 = nullptr;
  double* Gc2_64 = nullptr;
  double chain_dist = 0.0;
  if (chain) {
    dY.alloc(nvr0);
    C64a.alloc(nvr0);
    C64b.alloc(nvr0);
    Gc64 = C64a.ptr;
    Gc2_64 = C64b.ptr;
  }
  auto form_grad = [&]() {
    mf.grad(r, V.Rt.ptr, V.s.ptr, V.G.ptr, V.gR.ptr, V.gs.ptr, V.Sc.ptr, V.ec.ptr, V.part.ptr, st);
  };
  spmm_yt<T>(p, qg, V.Yt.ptr, r, V.G.ptr, st);
  ++out.spmm;
  if (chain) {
    hipLaunchKernelGGL(widen_kernel<T>, dim3(cdiv(nvr0, 256)), dim3(256), 0, st, static_cast<int64_t>(nvr0),
                       V.G.ptr, Gc64);
    XM_LAUNCH_CHECK("widen_kernel");
  }
  form_grad();
  read_partials(V.part.ptr, nb, 5, sums, st);
  double f = sums[0], gg = sums[1], gnorm = std::sqrt(sums[1]), ynorm = std::sqrt(sums[2]);
  // preconditioner scale at the current point and <g, P g>
  double pscale = sums[3] / N, gpg = sums[4] * pscale;
  const size_t nvr = static_cast<size_t>(3) * N * r;
  // the device-side step of each truncated-CG iteration, after the hess
  // kernel's partials in the same buffer (read back with them in one copy)
  double* ctl = V.part.ptr + 4 * static_cast<size_t>(nb);
  int k = 0;
  for (k = 0; k < max_outer; ++k) {
    if (gnorm <= grad_tol * qbar * ynorm) {
      out.converged = true;
      break;
    }
    // ---- truncated CG ----
    hipLaunchKernelGGL(tcg_init_kernel<T>, dim3(cdiv(std::max<size_t>(nvr, N), 256)), dim3(256), 0, st,
                       static_cast<int64_t>(nvr), N, V.gR.ptr, V.gs.ptr, V.etaR.ptr, V.etas.ptr, V.HetaR.ptr,
                       V.Hetas.ptr, V.resR.ptr, V.ress.ptr);
    XM_LAUNCH_CHECK("tcg_init_kernel");
    mf.pscale = pscale;
    double z_r = gpg;  // <res, P res>
    const double norm_r0 = std::sqrt(gg);
    int mode = 0;
    double beta = 0.0;
    bool boundary = false;
    int j = 0;
    for (j = 1; j <= max_inner; ++j) {
      mf.ydot(r, V.Rt.ptr, V.s.ptr, V.resR.ptr, V.ress.ptr, V.dR.ptr, V.ds.ptr, beta, mode, V.Ydot.ptr, st);
      spmm_yt<T>(p, qh, V.Ydot.ptr, r, V.Gd.ptr, st, XM_ROLE_CURVATURE);
      ++out.spmm;
      mf.hess(r, V.Rt.ptr, V.s.ptr, V.G.ptr, V.Sc.ptr, V.ec.ptr, V.dR.ptr, V.ds.ptr, V.Gd.ptr, V.etaR.ptr,
              V.etas.ptr, V.HdR.ptr, V.Hds.ptr, V.part.ptr, st);
      // the step (interior alpha, or the boundary tau on non-positive
      // curvature / leaving the region) is chosen on the device, and the
      // update applied, before the one host round trip of the iteration
      mf.tcg_step_update(r, V.s.ptr, V.part.ptr, z_r, Delta * Delta, ctl, V.dR.ptr, V.ds.ptr, V.HdR.ptr,
                         V.Hds.ptr, V.etaR.ptr, V.etas.ptr, V.HetaR.ptr, V.Hetas.ptr, V.resR.ptr, V.ress.ptr,
                         V.part.ptr, st);
      double hctl[6];
      read_partials2(V.part.ptr, nb, 2, sums, 4 * static_cast<int64_t>(nb), 6, hctl, st);
      if (hctl[1] != 0.0) {
        boundary = true;
        break;
      }
      const double r_r_new = sums[0], z_r_new = sums[1];
      if (std::sqrt(r_r_new) <= norm_r0 * std::min(std::pow(norm_r0, theta), kappa)) break;
      beta = z_r_new / z_r;
      z_r = z_r_new;
      mode = 1;
    }
    out.inner += std::min(j, max_inner);
    // ---- candidate and ratio test ----
    mf.retract(r, V.Rt.ptr, V.s.ptr, V.etaR.ptr, V.etas.ptr, V.Rt2.ptr, V.s2.ptr, V.Yt2.ptr, st);
    bool chained = false;
    double step = 0.0;
    if (chain) {
      const int64_t n = static_cast<int64_t>(nvr0);
      hipLaunchKernelGGL(sub_kernel<T>, dim3(cdiv(n, 256)), dim3(256), 0, st, n, V.Yt2.ptr, V.Yt.ptr, dY.ptr);
      XM_LAUNCH_CHECK("sub_kernel");
      step = std::sqrt(vec_dot<T>(dY.ptr, dY.ptr, n, V.part.ptr, 8, st));
      if (chain_dist + step <= kChainFrac * ynorm) {
        spmm_yt<T>(p, qg, dY.ptr, r, V.G2.ptr, st, XM_ROLE_CURVATURE);
        hipLaunchKernelGGL(combine_kernel<T>, dim3(cdiv(n, 256)), dim3(256), 0, st, n, Gc64, V.G2.ptr, Gc2_64);
        XM_LAUNCH_CHECK("combine_kernel");
        chained = true;
      }
    }
    if (!chained) {
      spmm_yt<T>(p, qg, V.Yt2.ptr, r, V.G2.ptr, st);
      if (chain) {
        hipLaunchKernelGGL(widen_kernel<T>, dim3(cdiv(nvr0, 256)), dim3(256), 0, st, static_cast<int64_t>(nvr0),
                           V.G2.ptr, Gc2_64);
        XM_LAUNCH_CHECK("widen_kernel");
      }
    }
    ++out.spmm;
    mf.model(r, V.s.ptr, V.s2.ptr, V.gR.ptr, V.gs.ptr, V.etaR.ptr, V.etas.ptr, V.HetaR.ptr, V.Hetas.ptr,
             V.Yt.ptr, V.G.ptr, V.Yt2.ptr, V.G2.ptr, V.part.ptr, st);
    read_partials(V.part.ptr, nb, 3, sums, st);
    const double mdec = -(sums[0] + 0.5 * sums[1]);
    const double df = sums[2];
    const double reg = std::max(1.0, std::fabs(f)) * 1e3 * 2.220446049250313e-16;
    const double rho = (-df + reg) / (mdec + reg);
    // a candidate whose cost is not finite (a scale step that overflowed) is
    // rejected and the radius cut, like any poor model agreement
    const bool finite = std::isfinite(rho);
    // a step the (reduced-precision) model misjudges as an increase is still
    // taken when the evaluated cost went down
    const bool accept = finite && ((mdec > 0.0 && rho > rho_prime) || (mdec <= 0.0 && df < -reg));
    // the ratio means nothing when the model predicts no decrease (rounding in
    // <eta, H eta> at a radius far beyond the Newton step, e.g. along the flat
    // directions of a rank-deficient point): such a step, unless the cost went
    // down anyway, cuts the radius and never grows it
    if (!finite || rho < 0.25 || (mdec <= 0.0 && !accept)) Delta *= 0.25;
    else if (mdec > 0.0 && rho > 0.75 && boundary) Delta = std::min(2.0 * Delta, Dbar);
    if (o.verbose)
      std::fprintf(stderr, "[xm] r=%d it=%d f=%.12e |g|=%.3e Delta=%.3e rho=%.3f inner=%d %s%s\n", r, k, f, gnorm,
                   Delta, rho, std::min(j, max_inner), boundary ? "boundary" : "interior", accept ? "" : " rejected");
    if (!accept && ++rejections >= floor_rejections && gnorm <= floor_tol * qbar * ynorm) {
      out.converged = out.floor = true;
      ++k;
      break;
    }
    // stagnation: twice as many rejections in a row (the radius down by 4^12)
    // at any gradient; the products' rounding decides every ratio there
    // (a reduced-precision stage hands its point to the FP64 stage)
    if (!accept && rejections >= 2 * floor_rejections) {
      out.floor = true;
      out.converged = gnorm <= floor_tol * qbar * ynorm;
      ++k;
      break;
    }
    if (accept) {
      rejections = 0;
      ++out.accepted;
      std::swap(V.Rt.ptr, V.Rt2.ptr);
      std::swap(V.s.ptr, V.s2.ptr);
      std::swap(V.Yt.ptr, V.Yt2.ptr);
      std::swap(V.G.ptr, V.G2.ptr);
      if (chain) {
        std::swap(Gc64, Gc2_64);
        chain_dist = chained ? chain_dist + step : 0.0;
      }
      form_grad();
      read_partials(V.part.ptr, nb, 5, sums, st);
      f = sums[0];
      gg = sums[1];
      gnorm = std::sqrt(gg);
      ynorm = std::sqrt(sums[2]);
      pscale = sums[3] / N;
      gpg = sums[4] * pscale;
    }
  }
  if (!out.converged && gnorm <= grad_tol * qbar * ynorm) out.converged = true;
  out.outer = k;
  out.f = f;
  out.gnorm = gnorm;
  out.ynorm = ynorm;
  out.Delta = Delta;
  return out;
}

// cost, gradient norm and |Y|_F of a point from an FP64 product
struct Check {
  double f, gnorm, ynorm;
};

Check fp64_check(xm_problem* p, const double* Yt64, int r, hipStream_t st) {
  const int N = p->N;
  Vecs<double> V(N, r);
  Manifold<double> mf(N);
  mf.lam = p->scale_reg;
  mf.split(r, Yt64, V.Rt.ptr, V.s.ptr, V.Yt.ptr, st);
  spmm_yt<double>(p, XM_F64, V.Yt.ptr, r, V.G.ptr, st);
  mf.grad(r, V.Rt.ptr, V.s.ptr, V.G.ptr, V.gR.ptr, V.gs.ptr, V.Sc.ptr, V.ec.ptr, V.part.ptr, st);
  double sums[5];
  read_partials(V.part.ptr, static_cast<int>(mf.blocks()), 5, sums, st);
  return {sums[0], std::sqrt(sums[1]), std::sqrt(sums[2])};
}

// Escape to rank r + 1 from the FP64 point X (Rt, s at rank r, Yt = s Rt in
// Yt64) along v: the cost before and after each trial step from FP64
// products, since the decrease Theorem "Descent Direction" guarantees is of
// order alpha^2 |lambda_min|.  On success X.Rt holds the rank-(r + 1) point.
bool escape_fp64(xm_problem* p, Vecs<double>& X, const double* Yt64, int r, const double* vmin, int* spmm_count,
                 hipStream_t st) {
  const int64_t n3 = p->n3;
  Manifold<double> mf(p->N);
  const int nblk = static_cast<int>(std::min<unsigned>(mf.blocks(), 8));
  spmm_yt<double>(p, XM_F64, Yt64, r, X.G2.ptr, st);
  ++*spmm_count;
  const double f0 = vec_dot<double>(Yt64, X.G2.ptr, n3 * r, X.part.ptr, nblk, st);
  double alpha = 1.0;
  for (int h = 0; h <= 40; ++h, alpha *= 0.5) {
    mf.escape(r, X.Rt.ptr, X.s.ptr, vmin, alpha, X.Rt2.ptr, X.Yt2.ptr, st);
    spmm_yt<double>(p, XM_F64, X.Yt2.ptr, r + 1, X.G2.ptr, st);
    ++*spmm_count;
    const double fn = vec_dot<double>(X.Yt2.ptr, X.G2.ptr, n3 * (r + 1), X.part.ptr, nblk, st);
    if (fn < f0) {
      std::swap(X.Rt.ptr, X.Rt2.ptr);
      return true;
    }
  }
  return false;
}

template <typename T>
__global__ void narrow_kernel(int64_t n, const double* __restrict__ a, T* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) out[i] = static_cast<T>(a[i]);
}

void add_stats(RtrOut& a, const RtrOut& b) {
  a.outer += b.outer;
  a.inner += b.inner;
  a.spmm += b.spmm;
  a.f = b.f;
  a.gnorm = b.gnorm;
  a.ynorm = b.ynorm;
  a.Delta = b.Delta;
  a.converged = b.converged;
  a.floor = b.floor;
}

template <typename T>
xm_status staircase(xm_problem* p, const xm_solve_opts& o, const double* Y0, int r_in, double* Y_out,
                    xm_solve_info* info, hipStream_t st) {
  const int N = p->N;
  const int64_t n3 = p->n3;
  constexpr bool f64 = std::is_same<T, double>::value;
  const xm_dtype qg = f64 ? XM_F64 : XM_F32;
  const xm_dtype qh = f64 ? XM_F64 : (o.compute == XM_BF16 ? XM_BF16 : XM_F32);
  // the reduced-precision stage stops well above its rounding floor: the
  // FP64 stage after it finishes the job, and near the floor the stage's
  // ratios are noise (on the 10155-frame clustered scenes a 3e-7 stage
  // tolerance sometimes took twice the inner iterations)
  const double grad_tol = (o.grad_tol > 0) ? o.grad_tol : (f64 ? 1e-9 : 1e-6);
  // tolerance of the FP64 stage of a reduced-precision solve: that of an FP64 solve
  const double grad_tol64 = f64 ? grad_tol : grad_tol / 1000.0;
  const double cert_tol = (o.cert_tol > 0) ? o.cert_tol : (f64 ? 1e-7 : 1e-5);
  const int rmax = o.r_max;
  Vecs<T> V(N, rmax + 1);
  Manifold<T> mf(N);
  Manifold<double> mf64(N);
  DevBuf<double> Yt64(static_cast<size_t>(n3) * (rmax + 1)), vmin(n3);
  // the FP64 stage's vectors (reduced precision only; an FP64 solve works in V)
  std::unique_ptr<Vecs<double>> W;
  if (!f64) W.reset(new Vecs<double>(N, rmax + 1));

  int r;
  if (Y0) {
    require(r_in >= 3 && r_in <= rmax, XM_EINVAL, "r_in must be in [3, r_max]");
    r = r_in;
    transpose_rows<double, double>(Y0, r, static_cast<int>(n3), Yt64.ptr, st);
    mf.split(r, Yt64.ptr, V.Rt.ptr, V.s.ptr, V.Yt.ptr, st);
  } else {
    r = o.r0;
    mf.init(r, o.lift, V.Rt.ptr, V.s.ptr, st);
  }
  *info = xm_solve_info{};
  double solve_ms = 0, cert_ms = 0;
  RtrOut ro;
  CertResult cr;
  // refinements at the current rank: when the certificate fails only through
  // the stationarity terms of its bound (the complement of rows(Y) alone
  // certifies, so no escape direction exists), the point is polished to a
  // tighter gradient tolerance, at most three times per rank (FP64 Hessian
  // products in a reduced-precision solve: near its floor the FP32 model
  // gains little per step).  Those terms shrink like a power |g|^k of the
  // gradient, 1 <= k <= 2 (the deflated block linearly, the coupling through
  // its square); the next target is the reached |g| times
  // (tol qbar / (2 |bound|))^(1/k), k = 2 for the first polish and fitted to
  // the last two (|g|, bound) pairs after that; the new tolerance is that
  // target or 10x the previous tolerance, whichever is lower, and never more
  // than 1e4x below the previous one.
  constexpr int kMaxRefines = 3;
  const double base_tol = grad_tol64;  // the tolerance the polish stages scale
  int refines = 0;
  double tscale = 1.0, g_prev = 0.0, b_prev = 0.0;
  while (true) {
    auto t0 = std::chrono::steady_clock::now();
    Vecs<double>* X = nullptr;
    if constexpr (f64) {
      ro = rtr<T>(p, V, r, qg, qh, o, grad_tol * tscale, st);
      X = &V;
    } else {
      // FP64 stage from the reduced-precision point (re-orthonormalised in
      // FP64), starting with the radius the first stage ended with; its
      // truncated-CG products use the FP32 Q (or factors) also in a BF16
      // solve, whose coarser Hessian would slow the final Newton steps.  A
      // refinement runs the FP64 stage alone, from where it ended.
      X = W.get();
      xm_solve_opts o2 = o;
      if (refines == 0) {
        ro = rtr<T>(p, V, r, qg, qh, o, grad_tol, st);
        transpose_rows<T, double>(V.Yt.ptr, 1, static_cast<int>(n3 * r), Yt64.ptr, st);
        mf64.split(r, Yt64.ptr, X->Rt.ptr, X->s.ptr, X->Yt.ptr, st);
        o2.delta0 = std::max(ro.Delta, std::sqrt(3.0 * N) / 512.0);
      } else {
        ro = RtrOut{};
      }
      const RtrOut r2 = rtr<double>(p, *X, r, XM_F64, refines == 0 ? XM_F32 : XM_F64, o2, grad_tol64 * tscale, st);
      if (o.verbose)
        std::fprintf(stderr, "[xm] rank %d: FP64 stage from |g|=%.3e: %d steps, %d products -> |g|=%.3e\n", r,
                     ro.gnorm, r2.outer, r2.spmm, r2.gnorm);
      add_stats(ro, r2);
    }
    XM_HIP(hipMemcpyAsync(Yt64.ptr, X->Yt.ptr, n3 * r * sizeof(double), hipMemcpyDeviceToDevice, st));
    XM_HIP(hipStreamSynchronize(st));
    auto t1 = std::chrono::steady_clock::now();
    solve_ms += std::chrono::duration<double, std::milli>(t1 - t0).count();
    info->outer_iters += ro.outer;
    info->inner_iters += ro.inner;
    info->spmm_count += ro.spmm;
    cr = certify_yt(p, Yt64.ptr, r, cert_tol, o.lanczos_max, o.lanczos_tol, vmin.ptr, st);
    auto t2 = std::chrono::steady_clock::now();
    cert_ms += std::chrono::duration<double, std::milli>(t2 - t1).count();
    info->lanczos_iters += cr.iters;
    if (o.verbose)
      std::fprintf(stderr, "[xm] rank %d: f=%.12e |g|=%.3e lambda_s=%.6e (res %.2e, %d it) bound %.3e %s\n", r, ro.f,
                   ro.gnorm, cr.lambda_min, cr.ritz_residual, cr.iters, cr.lambda_bound,
                   cr.certified ? "certified" : "not certified");
    if (cr.certified) break;
    if (cr.complement_ok && refines < kMaxRefines) {
      const double b = std::fabs(cr.lambda_bound), need = 0.5 * cert_tol * p->qbar / b;
      double k = 2.0;
      if (refines > 0 && g_prev > ro.gnorm && b_prev > b)
        k = std::fmin(2.0, std::fmax(1.0, std::log(b_prev / b) / std::log(g_prev / ro.gnorm)));
      const double t = std::fmin(1.0, std::fmax(1e-4, std::pow(need, 1.0 / k)));
      const double reached = ro.gnorm / (p->qbar * ro.ynorm);  // relative, as the tolerance
      tscale = std::fmax(1e-4 * tscale, std::fmin(0.1 * tscale, t * reached / base_tol));
      g_prev = ro.gnorm;
      b_prev = b;
      ++refines;
      continue;
    }
    if (r >= rmax) break;
    if (!escape_fp64(p, *X, Yt64.ptr, r, vmin.ptr, &info->spmm_count, st)) break;
    ++r;
    refines = 0;
    tscale = 1.0;
    ++info->stair_steps;
    if constexpr (!f64) {
      // back to the reduced-precision stage at the new rank
      const int64_t nr = n3 * r;
      hipLaunchKernelGGL(narrow_kernel<T>, dim3(cdiv(nr, 256)), dim3(256), 0, st, nr, X->Rt.ptr, V.Rt.ptr);
      hipLaunchKernelGGL(narrow_kernel<T>, dim3(cdiv(N, 256)), dim3(256), 0, st, static_cast<int64_t>(N), X->s.ptr,
                         V.s.ptr);
      XM_LAUNCH_CHECK("narrow_kernel");
    }
  }
  // final FP64 quantities (the certified point is in Yt64)
  const Check ck = fp64_check(p, Yt64.ptr, r, st);
  XM_HIP(hipMemsetAsync(Y_out, 0, static_cast<size_t>(rmax) * n3 * sizeof(double), st));
  transpose_rows<double, double>(Yt64.ptr, static_cast<int>(n3), r, Y_out, st);
  XM_HIP(hipStreamSynchronize(st));
  info->r = r;
  info->certified = cr.certified ? 1 : 0;
  info->converged = ro.converged ? (ro.floor ? 2 : 1) : 0;
  info->cost = ck.f;
  info->grad_norm = ck.gnorm;
  info->lambda_min = cr.lambda_bound;
  info->primal = cr.primal;
  info->dual = cr.dual;
  info->solve_ms = solve_ms;
  info->cert_ms = cert_ms;
  // a certified point is a global optimum whatever stopped the last stage
  // (a polish that ended on stagnation above its tighter tolerance)
  return (ro.converged || cr.certified) ? XM_OK : XM_ENOCONV;
}

}  // namespace

xm_status bm_solve(xm_problem* p, const xm_solve_opts& o, const double* Y0, int r_in, double* Y_out,
                   xm_solve_info* info, hipStream_t s) {
  require(o.r0 >= 3 && o.r_max >= o.r0 && o.r_max <= 7, XM_EINVAL, "need 3 <= r0 <= r_max <= 7");
  require(Y_out != nullptr && info != nullptr, XM_EINVAL, "Y_out and info must be non-NULL");
  if (o.compute == XM_F64) return staircase<double>(p, o, Y0, r_in, Y_out, info, s);
  require(o.compute == XM_F32 || o.compute == XM_BF16, XM_EINVAL, "unknown compute dtype");
  require(p->Q32.ptr != nullptr, XM_EINVAL, "reduced-precision solve needs the FP32 copy (XM_KEEP_F32)");
  if (o.compute == XM_BF16) require(p->Q16.ptr != nullptr, XM_EINVAL, "BF16 solve needs XM_KEEP_BF16");
  return staircase<float>(p, o, Y0, r_in, Y_out, info, s);
}

}  // namespace xm
