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
// within 30 grad_tol qbar |Y|.  A reduced-precision solve then checks the
// gradient with FP64 products and, if it is above grad_tol / 30, runs one
// short trust-region pass (at most 8 steps toward that tolerance; truncated-CG
// steps of at most 100 products, enough to resolve the flat scale modes of
// weakly linked frames) whose gradient products
// are taken relative to the current point, with the FP64 product at that point
// as reference (see Rebase).  The
// cost decrease is evaluated as <Y+ - Y, Q (Y+ + Y)> from the two products
// already computed, which stays accurate in FP32 where f(Y+) - f(Y) would
// cancel.  The staircase escape follows Theorem "Descent Direction": block k of
// [Y; alpha v^T] is re-orthonormalised (scale kept), alpha halved until the
// cost drops, at most 40 times.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <type_traits>
#include <vector>

#include "manifold.h"
#include "problem.h"

// Refinement pass of reduced-precision solves (compile-time constants):
// passes, trust-region steps per pass, products per truncated-CG solve.
#ifndef XM_REFINE_PASSES
#define XM_REFINE_PASSES 1
#endif
#ifndef XM_REFINE_STEPS
#define XM_REFINE_STEPS 8
#endif
#ifndef XM_REFINE_INNER
#define XM_REFINE_INNER 100
#endif

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
    part.alloc(static_cast<size_t>(cdiv(n, 256)) * 8);
  }
};

// Gradient products relative to a reference point (reduced precision only):
// G(Y) = Gref + Q (Y - Yref) with Gref = Q Yref from the FP64 Q, kept in FP64.
// The reduced-precision product then only carries the rounding error of the
// small difference Y - Yref, not of Q Y itself, whose entries cancel heavily
// near the optimum (Y is close to the null space of the dual matrix).  G is
// kept in FP64 (G64), and the Riemannian gradient and the cost change are
// formed from it in FP64, so that the cancellation in the projection
// E - R sym(R^T E) loses nothing either; the Hessian products use the rounded
// copy.  This is what lets an FP32 solve converge below the rounding noise
// of its own products.
template <typename T>
struct Rebase {
  const T* Yref = nullptr;
  const double* Gref = nullptr;  // Q Yref, FP64
  T* tmp = nullptr;
  double* G64 = nullptr;         // G(Y) at the current point, FP64
  double* G2_64 = nullptr;       // G(Y) at the candidate, FP64
  bool on() const { return Yref != nullptr; }
};

template <typename T>
__global__ void sub_kernel(int64_t n, const T* __restrict__ a, const T* __restrict__ b, T* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}

// G64 = Gref + G (FP64); G <- G64 rounded
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

template <typename T>
void grad_product(xm_problem* p, xm_dtype qg, const T* Yt, int r, T* G, double* G64, const Rebase<T>& rb,
                  hipStream_t st) {
  const int64_t n = p->n3 * static_cast<int64_t>(r);
  if (!rb.on()) {
    spmm_yt<T>(p, qg, Yt, r, G, st);
    return;
  }
  hipLaunchKernelGGL(sub_kernel<T>, dim3(cdiv(n, 256)), dim3(256), 0, st, n, Yt, rb.Yref, rb.tmp);
  XM_LAUNCH_CHECK("sub_kernel");
  // the product of the small difference Y - Yref: no cancellation at the scale
  // of Q Y, so the curvature-role product (the factored form on large
  // problems) is accurate enough
  spmm_yt<T>(p, qg, rb.tmp, r, G, st, XM_ROLE_CURVATURE);
  hipLaunchKernelGGL(combine_kernel<T>, dim3(cdiv(n, 256)), dim3(256), 0, st, n, rb.Gref, G, G64);
  XM_LAUNCH_CHECK("combine_kernel");
}

struct RtrOut {
  double f = 0, gnorm = 0, ynorm = 0;
  int outer = 0, inner = 0, spmm = 0, accepted = 0;
  bool converged = false, floor = false;
};

template <typename T>
RtrOut rtr(xm_problem* p, Vecs<T>& V, int r, xm_dtype qg, xm_dtype qh, const xm_solve_opts& o, double grad_tol,
           const Rebase<T>& rb, hipStream_t st) {
  const int N = p->N;
  Manifold<T> mf(N);
  if (o.precondition) mf.qkk = p->qkk.ptr;
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
  double* G64 = rb.G64;
  double* G2_64 = rb.G2_64;
  // Candidate products from the step (when the curvature products are
  // factored): G(Y+) = G(Y) + Q (Y+ - Y), the product of the small difference
  // taken in the curvature role and added in FP64.  Its rounding scales with
  // |Y+ - Y|, so while the steps taken since the last full product sum to at
  // most kChainFrac |Y| the accumulated error stays at the level of one full
  // product; past that, a full product restarts the chain.
  constexpr double kChainFrac = 0.05;
  const size_t nvr0 = static_cast<size_t>(3) * N * r;
  const bool chain = !rb.on() && p->spmm_kind[XM_ROLE_CURVATURE][qg] == XM_SPMM_FACTORED;
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
    if (rb.on()) mf.grad(r, V.Rt.ptr, V.s.ptr, static_cast<const double*>(G64), V.gR.ptr, V.gs.ptr, V.Sc.ptr,
                         V.ec.ptr, V.part.ptr, st);
    else mf.grad(r, V.Rt.ptr, V.s.ptr, static_cast<const T*>(V.G.ptr), V.gR.ptr, V.gs.ptr, V.Sc.ptr, V.ec.ptr,
                 V.part.ptr, st);
  };
  grad_product<T>(p, qg, V.Yt.ptr, r, V.G.ptr, G64, rb, st);
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
      read_partials(V.part.ptr, nb, 4, sums, st);
      const double d_Hd = sums[0], d_Pd = sums[1], e_Pd = sums[2], e_Pe = sums[3];
      const double alpha = z_r / d_Hd;
      const double e_Pe_new = e_Pe + 2.0 * alpha * e_Pd + alpha * alpha * d_Pd;
      if (d_Hd <= 0.0 || e_Pe_new >= Delta * Delta) {
        const double tau = (-e_Pd + std::sqrt(e_Pd * e_Pd + d_Pd * (Delta * Delta - e_Pe))) / d_Pd;
        mf.tcg_update(r, V.s.ptr, tau, 1, V.dR.ptr, V.ds.ptr, V.HdR.ptr, V.Hds.ptr, V.etaR.ptr, V.etas.ptr,
                      V.HetaR.ptr, V.Hetas.ptr, V.resR.ptr, V.ress.ptr, V.part.ptr, st);
        boundary = true;
        break;
      }
      mf.tcg_update(r, V.s.ptr, alpha, 0, V.dR.ptr, V.ds.ptr, V.HdR.ptr, V.Hds.ptr, V.etaR.ptr, V.etas.ptr,
                    V.HetaR.ptr, V.Hetas.ptr, V.resR.ptr, V.ress.ptr, V.part.ptr, st);
      read_partials(V.part.ptr, nb, 2, sums, st);
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
      grad_product<T>(p, qg, V.Yt2.ptr, r, V.G2.ptr, G2_64, rb, st);
      if (chain) {
        hipLaunchKernelGGL(widen_kernel<T>, dim3(cdiv(nvr0, 256)), dim3(256), 0, st, static_cast<int64_t>(nvr0),
                           V.G2.ptr, Gc2_64);
        XM_LAUNCH_CHECK("widen_kernel");
      }
    }
    ++out.spmm;
    if (rb.on())
      mf.model(r, V.s.ptr, V.gR.ptr, V.gs.ptr, V.etaR.ptr, V.etas.ptr, V.HetaR.ptr, V.Hetas.ptr, V.Yt.ptr,
               static_cast<const double*>(G64), V.Yt2.ptr, static_cast<const double*>(G2_64), true, V.part.ptr, st);
    else
      mf.model(r, V.s.ptr, V.gR.ptr, V.gs.ptr, V.etaR.ptr, V.etas.ptr, V.HetaR.ptr, V.Hetas.ptr, V.Yt.ptr,
               static_cast<const T*>(V.G.ptr), V.Yt2.ptr, static_cast<const T*>(V.G2.ptr), false, V.part.ptr, st);
    read_partials(V.part.ptr, nb, 3, sums, st);
    const double mdec = -(sums[0] + 0.5 * sums[1]);
    const double df = sums[2];
    const double reg = std::max(1.0, std::fabs(f)) * 1e3 * 2.220446049250313e-16;
    const double rho = (-df + reg) / (mdec + reg);
    // a candidate whose cost is not finite (a scale step that overflowed) is
    // rejected and the radius cut, like any poor model agreement
    const bool finite = std::isfinite(rho);
    if (!finite || rho < 0.25) Delta *= 0.25;
    else if (rho > 0.75 && boundary) Delta = std::min(2.0 * Delta, Dbar);
    // a step the (reduced-precision) model misjudges as an increase is still
    // taken when the evaluated cost went down
    const bool accept = finite && ((mdec > 0.0 && rho > rho_prime) || (mdec <= 0.0 && df < -reg));
    if (o.verbose)
      std::fprintf(stderr, "[xm] r=%d it=%d f=%.12e |g|=%.3e Delta=%.3e rho=%.3f inner=%d %s%s\n", r, k, f, gnorm,
                   Delta, rho, std::min(j, max_inner), boundary ? "boundary" : "interior", accept ? "" : " rejected");
    if (!accept && ++rejections >= floor_rejections && gnorm <= floor_tol * qbar * ynorm) {
      out.converged = out.floor = true;
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
      std::swap(G64, G2_64);
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
  return out;
}

// cost, gradient norm and |Y|_F of the current point from FP64 products (for
// reduced-precision solves); optionally the FP64 product Q Y, rounded to T
struct Check {
  double f, gnorm, ynorm;
};

Check fp64_check(xm_problem* p, const double* Yt64, int r, hipStream_t st, double* G_out = nullptr) {
  const int N = p->N;
  Vecs<double> V(N, r);
  Manifold<double> mf(N);
  mf.split(r, Yt64, V.Rt.ptr, V.s.ptr, V.Yt.ptr, st);
  spmm_yt<double>(p, XM_F64, V.Yt.ptr, r, V.G.ptr, st);
  mf.grad(r, V.Rt.ptr, V.s.ptr, V.G.ptr, V.gR.ptr, V.gs.ptr, V.Sc.ptr, V.ec.ptr, V.part.ptr, st);
  double sums[5];
  read_partials(V.part.ptr, static_cast<int>(mf.blocks()), 5, sums, st);
  if (G_out) XM_HIP(hipMemcpyAsync(G_out, V.G.ptr, p->n3 * r * sizeof(double), hipMemcpyDeviceToDevice, st));
  return {sums[0], std::sqrt(sums[1]), std::sqrt(sums[2])};
}

template <typename T>
xm_status staircase(xm_problem* p, const xm_solve_opts& o, const double* Y0, int r_in, double* Y_out,
                    xm_solve_info* info, hipStream_t st) {
  const int N = p->N;
  const int64_t n3 = p->n3;
  const bool f64 = std::is_same<T, double>::value;
  const xm_dtype qg = f64 ? XM_F64 : XM_F32;
  const xm_dtype qh = f64 ? XM_F64 : (o.compute == XM_BF16 ? XM_BF16 : XM_F32);
  const double grad_tol = (o.grad_tol > 0) ? o.grad_tol : (f64 ? 1e-9 : 3e-7);
  const double cert_tol = (o.cert_tol > 0) ? o.cert_tol : (f64 ? 1e-7 : 1e-5);
  const int rmax = o.r_max;
  Vecs<T> V(N, rmax + 1);
  Manifold<T> mf(N);
  DevBuf<double> Yt64(static_cast<size_t>(n3) * (rmax + 1)), vmin(n3);
  // reduced precision: reference point and FP64 products for the refinement passes
  DevBuf<T> Yref, Rtmp;
  DevBuf<double> Gref, G64a, G64b;
  if (!f64) {
    Yref.alloc(static_cast<size_t>(n3) * rmax);
    Rtmp.alloc(static_cast<size_t>(n3) * rmax);
    Gref.alloc(static_cast<size_t>(n3) * rmax);
    G64a.alloc(static_cast<size_t>(n3) * rmax);
    G64b.alloc(static_cast<size_t>(n3) * rmax);
  }
  // refinement target: the FP32 stage stops at grad_tol (its products' own
  // rounding allows little more), the FP64-referenced passes go 30x further
  const int max_refine = XM_REFINE_PASSES;
  const double refine_tol = grad_tol / 30.0;

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
  while (true) {
    auto t0 = std::chrono::steady_clock::now();
    ro = rtr<T>(p, V, r, qg, qh, o, grad_tol, Rebase<T>{}, st);
    // Reduced precision: check the gradient with FP64 products; while it is
    // above the tolerance, continue from the current point with gradient
    // products taken relative to it (Rebase), the FP64 product as reference.
    for (int pass = 0; !f64 && pass < max_refine; ++pass) {
      transpose_rows<T, double>(V.Yt.ptr, 1, static_cast<int>(n3 * r), Yt64.ptr, st);
      const Check ck = fp64_check(p, Yt64.ptr, r, st, Gref.ptr);
      ++info->spmm_count;
      if (o.verbose)
        std::fprintf(stderr, "[xm] rank %d: FP64 check |g|=%.3e (tol %.3e)%s\n", r, ck.gnorm,
                     refine_tol * p->qbar * ck.ynorm, ck.gnorm <= refine_tol * p->qbar * ck.ynorm ? "" : ", refining");
      if (ck.gnorm <= refine_tol * p->qbar * ck.ynorm) break;
      XM_HIP(hipMemcpyAsync(Yref.ptr, V.Yt.ptr, n3 * r * sizeof(T), hipMemcpyDeviceToDevice, st));
      // a refinement pass is a short polish from a converged point: at most 8
      // steps, starting from a radius 64x below the default
      xm_solve_opts oref = o;
      oref.max_outer = (o.max_outer > 0) ? std::min(o.max_outer, XM_REFINE_STEPS) : XM_REFINE_STEPS;
      if (oref.delta0 <= 0) oref.delta0 = std::sqrt(3.0 * N) / 8.0 / 64.0;
      oref.max_inner = (o.max_inner > 0) ? std::min(o.max_inner, XM_REFINE_INNER) : XM_REFINE_INNER;
      const RtrOut r2 = rtr<T>(p, V, r, qg, qh, oref, refine_tol,
                               Rebase<T>{Yref.ptr, Gref.ptr, Rtmp.ptr, G64a.ptr, G64b.ptr}, st);
      ro.outer += r2.outer;
      ro.inner += r2.inner;
      ro.spmm += r2.spmm;
      ro.f = r2.f;
      ro.gnorm = r2.gnorm;
      ro.ynorm = r2.ynorm;
      // convergence is judged at grad_tol: the refinement target is a bonus
      if (r2.converged && !r2.floor) ro.floor = false;
      ro.converged = ro.converged || r2.converged;
      if (r2.accepted == 0) break;  // the iterate's own rounding is the floor: no further progress
    }
    XM_HIP(hipStreamSynchronize(st));
    auto t1 = std::chrono::steady_clock::now();
    solve_ms += std::chrono::duration<double, std::milli>(t1 - t0).count();
    info->outer_iters += ro.outer;
    info->inner_iters += ro.inner;
    info->spmm_count += ro.spmm;
    // FP64 copy of the factor for the certificate
    if (f64) XM_HIP(hipMemcpyAsync(Yt64.ptr, V.Yt.ptr, n3 * r * sizeof(double), hipMemcpyDeviceToDevice, st));
    else transpose_rows<T, double>(V.Yt.ptr, 1, static_cast<int>(n3 * r), Yt64.ptr, st);
    cr = certify_yt(p, Yt64.ptr, r, cert_tol, o.lanczos_max, o.lanczos_tol, vmin.ptr, st);
    auto t2 = std::chrono::steady_clock::now();
    cert_ms += std::chrono::duration<double, std::milli>(t2 - t1).count();
    info->lanczos_iters += cr.iters;
    if (o.verbose)
      std::fprintf(stderr, "[xm] rank %d: f=%.12e |g|=%.3e lambda_s=%.6e (res %.2e, %d it) %s\n", r, ro.f,
                   ro.gnorm, cr.lambda_min, cr.ritz_residual, cr.iters, cr.certified ? "certified" : "not certified");
    if (cr.certified || r >= rmax) break;
    // escape to rank r + 1 with step halving.  The costs before and after are
    // both taken with FP64 products at the FP64 copies of the points: the
    // decrease of Theorem "Descent Direction" is of order alpha^2 |lambda_min|,
    // which a reduced-precision product's rounding near the optimum can exceed.
    const int nblk = static_cast<int>(std::min<unsigned>(mf.blocks(), 8));
    DevBuf<double> Y2_64(static_cast<size_t>(n3) * (r + 1)), G2_64(static_cast<size_t>(n3) * (r + 1));
    spmm_yt<double>(p, XM_F64, Yt64.ptr, r, G2_64.ptr, st);
    ++info->spmm_count;
    const double f0 = vec_dot<double>(Yt64.ptr, G2_64.ptr, static_cast<int64_t>(n3) * r, V.part.ptr, nblk, st);
    bool moved = false;
    double alpha = 1.0;
    for (int h = 0; h <= 40; ++h, alpha *= 0.5) {
      mf.escape(r, V.Rt.ptr, V.s.ptr, vmin.ptr, alpha, V.Rt2.ptr, V.Yt2.ptr, st);
      const double* y2 = Y2_64.ptr;
      if constexpr (std::is_same<T, double>::value) y2 = V.Yt2.ptr;
      else transpose_rows<T, double>(V.Yt2.ptr, 1, static_cast<int>(n3 * (r + 1)), Y2_64.ptr, st);
      spmm_yt<double>(p, XM_F64, y2, r + 1, G2_64.ptr, st);
      ++info->spmm_count;
      // f(Y+) = <Yt2, Q Yt2>
      const double fn = vec_dot<double>(y2, G2_64.ptr, static_cast<int64_t>(n3) * (r + 1), V.part.ptr, nblk, st);
      if (fn < f0) {
        moved = true;
        break;
      }
    }
    if (!moved) break;
    std::swap(V.Rt.ptr, V.Rt2.ptr);
    ++r;
    ++info->stair_steps;
  }
  // final FP64 quantities
  if (f64) XM_HIP(hipMemcpyAsync(Yt64.ptr, V.Yt.ptr, n3 * r * sizeof(double), hipMemcpyDeviceToDevice, st));
  else transpose_rows<T, double>(V.Yt.ptr, 1, static_cast<int>(n3 * r), Yt64.ptr, st);
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
  return ro.converged ? XM_OK : XM_ENOCONV;
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
