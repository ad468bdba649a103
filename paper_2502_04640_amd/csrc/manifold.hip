// Per-frame kernels of the Riemannian trust-region solver on
//   St(r,3) x (R_+ x St(r,3))^{N-1}   (Prop. "BM Riemannian Optimization").
//
// Layout ("Yt", frame-major): an r x 3 block X_k of frame k is stored as
// X[(3k + c) * r + a] = X_k[a][c], so the product kernel sees rows of Y^T.
// One thread owns one frame (3r <= 24 values); every kernel that needs inner
// products writes per-block partial sums [block][q] that the host adds in a
// fixed order.  All partial sums accumulate in FP64, whatever T is.
//
// Formulas (f = tr(Q Y^T Y), G = Q Y^T, Gamma_k = 2 G_k):
//   E_k = s_k Gamma_k, e_k = <R_k, Gamma_k>, S_k = sym(R_k^T E_k)
//   grad_R = E_k - R_k S_k,                grad_s = s_k^2 e_k   (k >= 1)
//   Hess:  Ydot_k = sdot_k R_k + s_k Rdot_k,  Gd = Q Ydot^T,
//          Edot = sdot Gamma + s 2 Gd,  edot = <Rdot, Gamma> + <R, 2 Gd>,
//          H_R = P_R(Edot - Rdot S_k),  H_s = s^2 edot + s e sdot,
//          P_R(Z) = Z - R sym(R^T Z)
//   metric: <a, b> = sum <aR, bR> + sum_{k>=1} a_s b_s / s_k^2
//   retraction: R <- Gram-Schmidt(R + Rdot), s <- s exp(sdot / s)
#include <cmath>

#include "manifold.h"
#include "problem.h"

namespace xm {
namespace {

constexpr int kB = kFrameBlock;   // per-frame kernels
constexpr int kVB = 256;          // vec_dot

template <typename T, int R>
struct Blk {
  T v[3][R];  // v[c][a] = X_k[a][c]
  __device__ void load(const T* p, int k) {
    const T* q = p + static_cast<int64_t>(k) * 3 * R;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < R; ++a) v[c][a] = q[c * R + a];
  }
  __device__ void store(T* p, int k) const {
    T* q = p + static_cast<int64_t>(k) * 3 * R;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < R; ++a) q[c * R + a] = v[c][a];
  }
};

template <typename T, int R>
__device__ __forceinline__ double dotb(const Blk<T, R>& x, const Blk<T, R>& y) {
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < R; ++a) s += static_cast<double>(x.v[c][a]) * static_cast<double>(y.v[c][a]);
  return s;
}

// M[c][d] = sum_a X[a][c] Y[a][d] = (X^T Y)[c][d]
template <typename T, int R>
__device__ __forceinline__ void xty(const Blk<T, R>& x, const Blk<T, R>& y, T (&M)[3][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T s = T(0);
#pragma unroll
      for (int a = 0; a < R; ++a) s += x.v[c][a] * y.v[d][a];
      M[c][d] = s;
    }
}

template <typename T>
__device__ __forceinline__ void symm(T (&M)[3][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = c + 1; d < 3; ++d) {
      const T m = T(0.5) * (M[c][d] + M[d][c]);
      M[c][d] = m;
      M[d][c] = m;
    }
}

// out[a][c] -= sum_d X[a][d] S[d][c]
template <typename T, int R>
__device__ __forceinline__ void sub_xs(Blk<T, R>& out, const Blk<T, R>& x, const T (&S)[3][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < R; ++a) {
      T s = T(0);
#pragma unroll
      for (int d = 0; d < 3; ++d) s += x.v[d][a] * S[d][c];
      out.v[c][a] -= s;
    }
}

// Per-frame preconditioner weight c_k = s_k^2 q_kk / pscale (q_kk = tr(Q_kk)/3;
// pscale = mean over frames of s_k^2 q_kk), or 1 when qkk is NULL.  The
// preconditioner M acts as c_k on the rotation part and 3 c_k on the scale
// part of a tangent vector (the diagonal of the Hessian with Q_kk replaced by
// q_kk I); P = M^{-1}.
__device__ __forceinline__ double prec_weight(const double* qkk, double pscale, double s) {
  return qkk ? s * s * qkk[0] / pscale : 1.0;
}
// factor of the scale part relative to the rotation part (1 without a preconditioner)
__device__ __forceinline__ double prec_sfac(const double* qkk) { return qkk ? 3.0 : 1.0; }

// per-workgroup partial sums (workgroups of at most 256 threads: 4 waves)
template <int NQ>
__device__ __forceinline__ void write_partials(double (&v)[NQ], double* part) {
  __shared__ double lds[NQ * 4];
  block_sum<NQ>(v, lds);
  if (threadIdx.x == 0)
    for (int q = 0; q < NQ; ++q) part[blockIdx.x * NQ + q] = v[q];
}

// ---------------------------------------------------------------------------
// Riemannian gradient: E_k = s_k Gamma_k projected on the tangent space of
// the Stiefel factor, e_k = <R_k, Gamma_k> for the scale (Gamma = 2 Q Y).
template <typename T, int R>
__global__ __launch_bounds__(kB) void grad_kernel(int32_t N, const T* __restrict__ Rt, const T* __restrict__ s,
                                                  const T* __restrict__ G, T* __restrict__ gR, T* __restrict__ gs,
                                                  T* __restrict__ Sc, T* __restrict__ ec, const double* qkk,
                                                  double lam, double* part) {
  const int k = blockIdx.x * kB + threadIdx.x;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (k < N) {
    Blk<T, R> Rk, Gam;
    Rk.load(Rt, k);
    Gam.load(G, k);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < R; ++a) Gam.v[c][a] *= T(2);
    const T sk = s[k];
    // df/ds_k: the quadratic part <R_k, Gamma_k> plus F'(s_k) = 4 lam s (s^2 - 1)
    const double sdk = static_cast<double>(sk);
    const double e = dotb(Rk, Gam) + ((k == 0) ? 0.0 : 4.0 * lam * sdk * (sdk * sdk - 1.0));
    const double Fk = (k == 0) ? 0.0 : lam * (sdk * sdk - 1.0) * (sdk * sdk - 1.0);
    T M[3][3];
    xty(Rk, Gam, M);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d) M[c][d] *= sk;
    symm(M);
    Blk<T, R> g;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < R; ++a) g.v[c][a] = sk * Gam.v[c][a];
    sub_xs(g, Rk, M);
    const Blk<T, R>& gt = g;
    gt.store(gR, k);
    const T gsk = (k == 0) ? T(0) : static_cast<T>(static_cast<double>(sk) * sk * e);
    gs[k] = gsk;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d) Sc[k * 9 + c * 3 + d] = static_cast<T>(M[c][d]);
    ec[k] = static_cast<T>(e);
    v[0] = 0.5 * sdk * (e - ((k == 0) ? 0.0 : 4.0 * lam * sdk * (sdk * sdk - 1.0))) + Fk;
    v[1] = dotb(gt, gt) + ((k == 0) ? 0.0 : static_cast<double>(gsk) * gsk / (static_cast<double>(sk) * sk));
    v[2] = 3.0 * static_cast<double>(sk) * sk;
    // unnormalised preconditioner sums: s^2 q_kk and <g, M^{-1} g> * pscale
    const double w = prec_weight(qkk ? qkk + k : nullptr, 1.0, static_cast<double>(sk));
    v[3] = w;
    v[4] = dotb(gt, gt) / w +
           ((k == 0) ? 0.0 : static_cast<double>(gsk) * gsk / (prec_sfac(qkk) * w * static_cast<double>(sk) * sk));
  }
  write_partials<5>(v, part);
}

// mode 0: delta = -res;  mode 1: delta = -res + beta * delta;  mode 2: delta as is.
// Ydot = sdot R + s Rdot (for delta).
template <typename T, int R>
__global__ __launch_bounds__(kB) void ydot_kernel(int32_t N, const T* __restrict__ Rt, const T* __restrict__ s,
                                                  const T* __restrict__ resR, const T* __restrict__ ress,
                                                  T* __restrict__ dR, T* __restrict__ ds, double beta, int mode,
                                                  const double* qkk, double pscale, T* __restrict__ Ydot) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  Blk<T, R> Rk, d;
  Rk.load(Rt, k);
  T dsk;
  if (mode == 2) {
    d.load(dR, k);
    dsk = ds[k];
  } else {
    // preconditioned residual z = P res
    Blk<T, R> r;
    r.load(resR, k);
    const double c = prec_weight(qkk ? qkk + k : nullptr, pscale, static_cast<double>(s[k]));
    const T ic = static_cast<T>(1.0 / c), ic3 = static_cast<T>(1.0 / (prec_sfac(qkk) * c));
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
      for (int a = 0; a < R; ++a) r.v[cc][a] *= ic;
    const T rs = ress[k] * ic3;
    if (mode == 1) {
      d.load(dR, k);
      const T b = static_cast<T>(beta);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < R; ++a) d.v[c][a] = -r.v[c][a] + b * d.v[c][a];
      dsk = -rs + b * ds[k];
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < R; ++a) d.v[c][a] = -r.v[c][a];
      dsk = -rs;
    }
    d.store(dR, k);
    ds[k] = dsk;
  }
  const T sk = s[k];
  Blk<T, R> y;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < R; ++a) y.v[c][a] = dsk * Rk.v[c][a] + sk * d.v[c][a];
  y.store(Ydot, k);
}

template <typename T, int R>
__global__ __launch_bounds__(kB) void hess_kernel(int32_t N, const T* __restrict__ Rt, const T* __restrict__ s,
                                                  const T* __restrict__ G, const T* __restrict__ Sc,
                                                  const T* __restrict__ ec, const T* __restrict__ dR,
                                                  const T* __restrict__ ds, const T* __restrict__ Gd,
                                                  const T* __restrict__ etaR, const T* __restrict__ etas,
                                                  T* __restrict__ HR, T* __restrict__ Hs, const double* qkk,
                                                  double pscale, double lam, double* part, int anchor0) {
  const int k = blockIdx.x * kB + threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (k == 0 && anchor0) {
    // frame 0 held fixed (anchored chart): the Hessian is projected onto the other frames
    for (int e = 0; e < 3 * R; ++e) HR[e] = T(0);
    Hs[0] = T(0);
  } else if (k < N) {
    Blk<T, R> Rk, Gam, Gdd, Rd, Z;
    Rk.load(Rt, k);
    Gam.load(G, k);
    Gdd.load(Gd, k);
    Rd.load(dR, k);
    const T sk = s[k], dsk = ds[k], ek = ec[k];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < R; ++a) {
        Gam.v[c][a] *= T(2);
        Gdd.v[c][a] *= T(2);
        Z.v[c][a] = dsk * Gam.v[c][a] + sk * Gdd.v[c][a];  // Edot
      }
    const double edot = dotb(Rd, Gam) + dotb(Rk, Gdd);
    T S[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d) S[c][d] = Sc[k * 9 + c * 3 + d];
    sub_xs(Z, Rd, S);  // Z = Edot - Rdot S
    T W[3][3];
    xty(Rk, Z, W);
    symm(W);
    sub_xs(Z, Rk, W);  // H_R = Z - R sym(R^T Z)
    Z.store(HR, k);
    const double sd = static_cast<double>(sk);
    // s^2 d(df/ds)[sdot] + s (df/ds) sdot, with ek = df/ds (regulariser
    // included) and the regulariser's second derivative 4 lam (3 s^2 - 1)
    const double hs = (k == 0) ? 0.0
                               : sd * sd * (edot + 4.0 * lam * (3.0 * sd * sd - 1.0) * static_cast<double>(dsk)) +
                                     sd * static_cast<double>(ek) * static_cast<double>(dsk);
    Hs[k] = static_cast<T>(hs);
    const double is2 = (k == 0) ? 0.0 : 1.0 / (sd * sd);
    Blk<T, R> eta;
    eta.load(etaR, k);
    const double es = etas[k];
    // the trust region is measured in the preconditioner norm <a, M b>
    const double c = prec_weight(qkk ? qkk + k : nullptr, pscale, sd), c3 = prec_sfac(qkk) * c * is2;
    v[0] = dotb(Rd, Z) + static_cast<double>(dsk) * hs * is2;                               // <d, Hd>
    v[1] = c * dotb(Rd, Rd) + c3 * static_cast<double>(dsk) * static_cast<double>(dsk);     // <d, M d>
    v[2] = c * dotb(eta, Rd) + c3 * es * static_cast<double>(dsk);                          // <eta, M d>
    v[3] = c * dotb(eta, eta) + c3 * es * es;                                               // <eta, M eta>
  }
  write_partials<4>(v, part);
}

// mode 0 (interior): eta += a d, Heta += a Hd, res += a Hd, partial <res, res>
// mode 1 (boundary): eta += a d, Heta += a Hd
template <typename T, int R>
__global__ __launch_bounds__(kB) void tcg_update_kernel(int32_t N, const T* __restrict__ s, double alpha, int mode,
                                                        const double* __restrict__ ctl,
                                                        const T* __restrict__ dR, const T* __restrict__ ds,
                                                        const T* __restrict__ HdR, const T* __restrict__ Hds,
                                                        T* __restrict__ etaR, T* __restrict__ etas,
                                                        T* __restrict__ HetaR, T* __restrict__ Hetas,
                                                        T* __restrict__ resR, T* __restrict__ ress, const double* qkk,
                                                        double pscale, double* part) {
  const int k = blockIdx.x * kB + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (ctl) {  // step and mode decided on the device (tcg_step_kernel)
    alpha = ctl[0];
    mode = static_cast<int>(ctl[1]);
  }
  if (k < N) {
    const T a = static_cast<T>(alpha);
    Blk<T, R> d, hd, e, he;
    d.load(dR, k);
    hd.load(HdR, k);
    e.load(etaR, k);
    he.load(HetaR, k);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int q = 0; q < R; ++q) {
        e.v[c][q] += a * d.v[c][q];
        he.v[c][q] += a * hd.v[c][q];
      }
    e.store(etaR, k);
    he.store(HetaR, k);
    etas[k] += a * ds[k];
    Hetas[k] += a * Hds[k];
    if (mode == 0) {
      Blk<T, R> r;
      r.load(resR, k);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int q = 0; q < R; ++q) r.v[c][q] += a * hd.v[c][q];
      r.store(resR, k);
      const T rs = ress[k] + a * Hds[k];
      ress[k] = rs;
      const double sd = static_cast<double>(s[k]);
      const double rr = dotb(r, r), ss = (k == 0) ? 0.0 : static_cast<double>(rs) * rs / (sd * sd);
      const double c = prec_weight(qkk ? qkk + k : nullptr, pscale, sd);
      v[0] = rr + ss;                      // <res, res>
      v[1] = rr / c + ss / (prec_sfac(qkk) * c);  // <res, P res>
    }
  }
  write_partials<2>(v, part);
}

// The scalar step of a truncated-CG iteration, on the device so that the
// update needs no host round trip: one wavefront adds the partials of
// hess_kernel (lane l takes blocks l, l + 64, ..., then a fixed xor tree:
// deterministic), then alpha = z_r / <d, Hd>; if the curvature is not positive
// or the step leaves the trust region, the boundary step tau
// (|eta + tau d|_M = Delta) instead.  ctl = {step, mode (0 interior,
// 1 boundary), <d,Hd>, <d,Md>, <eta,Md>, <eta,M eta>}.
__global__ __launch_bounds__(64) void tcg_step_kernel(const double* __restrict__ part, int nb, double z_r,
                                                      double delta2, double* __restrict__ ctl) {
  const int lane = threadIdx.x;
  double q[4];
  for (int j = 0; j < 4; ++j) {
    double acc = 0.0;
    for (int b = lane; b < nb; b += 64) acc += part[b * 4 + j];
    q[j] = wave_sum(acc);
  }
  if (lane != 0) return;
  const double d_Hd = q[0], d_Pd = q[1], e_Pd = q[2], e_Pe = q[3];
  const double alpha = z_r / d_Hd;
  const double e_Pe_new = e_Pe + 2.0 * alpha * e_Pd + alpha * alpha * d_Pd;
  const bool boundary = !(d_Hd > 0.0) || e_Pe_new >= delta2;
  ctl[0] = boundary ? (-e_Pd + sqrt(e_Pd * e_Pd + d_Pd * (delta2 - e_Pe))) / d_Pd : alpha;
  ctl[1] = boundary ? 1.0 : 0.0;
  for (int j = 0; j < 4; ++j) ctl[2 + j] = q[j];
}

// Gram-Schmidt of the three columns of an r x 3 block (positive-diagonal QR).
template <typename T, int R>
__device__ __forceinline__ void gram_schmidt(Blk<T, R>& m) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int d = 0; d < c; ++d) {
      T p = T(0);
#pragma unroll
      for (int a = 0; a < R; ++a) p += m.v[d][a] * m.v[c][a];
#pragma unroll
      for (int a = 0; a < R; ++a) m.v[c][a] -= p * m.v[d][a];
    }
    T nn = T(0);
#pragma unroll
    for (int a = 0; a < R; ++a) nn += m.v[c][a] * m.v[c][a];
    const T inv = T(1) / sqrt(nn);
#pragma unroll
    for (int a = 0; a < R; ++a) m.v[c][a] *= inv;
  }
}

template <typename T, int R>
__global__ __launch_bounds__(kB) void retract_kernel(int32_t N, const T* __restrict__ Rt, const T* __restrict__ s,
                                                     const T* __restrict__ etaR, const T* __restrict__ etas,
                                                     T* __restrict__ Rt2, T* __restrict__ s2, T* __restrict__ Yt2) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  Blk<T, R> m, e;
  m.load(Rt, k);
  e.load(etaR, k);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < R; ++a) m.v[c][a] += e.v[c][a];
  gram_schmidt(m);
  m.store(Rt2, k);
  const T sk = s[k];
  // log-scale step, clamped so that an oversized trial step cannot overflow
  const T x = fmin(fmax(etas[k] / sk, T(-30)), T(30));
  const T sn = (k == 0) ? T(1) : sk * exp(x);
  s2[k] = sn;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < R; ++a) m.v[c][a] *= sn;
  m.store(Yt2, k);
}

// partials: <g, eta>, <eta, Heta>, <Y2 - Y, G2 + G>
template <typename T, int R>
__global__ __launch_bounds__(kB) void model_kernel(int32_t N, const T* __restrict__ s, const T* __restrict__ s2,
                                                   double lam, const T* __restrict__ gR,
                                                   const T* __restrict__ gs, const T* __restrict__ etaR,
                                                   const T* __restrict__ etas, const T* __restrict__ HetaR,
                                                   const T* __restrict__ Hetas, const T* __restrict__ Yt,
                                                   const T* __restrict__ G, const T* __restrict__ Yt2,
                                                   const T* __restrict__ G2, double* part) {
  const int k = blockIdx.x * kB + threadIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  if (k < N) {
    Blk<T, R> g, e, he, y, y2, gg, g2;
    g.load(gR, k);
    e.load(etaR, k);
    he.load(HetaR, k);
    y.load(Yt, k);
    gg.load(G, k);
    y2.load(Yt2, k);
    g2.load(G2, k);
    const double sd = static_cast<double>(s[k]);
    const double is2 = (k == 0) ? 0.0 : 1.0 / (sd * sd);
    v[0] = dotb(g, e) + static_cast<double>(gs[k]) * static_cast<double>(etas[k]) * is2;
    v[1] = dotb(e, he) + static_cast<double>(etas[k]) * static_cast<double>(Hetas[k]) * is2;
    double df = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < R; ++a)
        df += (static_cast<double>(y2.v[c][a]) - static_cast<double>(y.v[c][a])) *
              (static_cast<double>(g2.v[c][a]) + static_cast<double>(gg.v[c][a]));
    if (k > 0 && lam != 0.0) {
      const double a2 = static_cast<double>(s2[k]) * static_cast<double>(s2[k]) - 1.0, a1 = sd * sd - 1.0;
      df += lam * (a2 - a1) * (a2 + a1);
    }
    v[2] = df;
  }
  write_partials<3>(v, part);
}

// Staircase escape (Theorem "Descent Direction"): block k of [Y; alpha v^T]
// retracted onto s_k St(r+1, 3):  R' = GS([R_k; alpha v_k^T / s_k]), s' = s.
template <typename T, int R>
__global__ __launch_bounds__(kB) void escape_kernel(int32_t N, const T* __restrict__ Rt, const T* __restrict__ s,
                                                    const double* __restrict__ v, double alpha, T* __restrict__ Rt2,
                                                    T* __restrict__ Yt2) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  Blk<T, R + 1> m;
  const T sk = s[k];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int a = 0; a < R; ++a) m.v[c][a] = Rt[static_cast<int64_t>(k) * 3 * R + c * R + a];
    m.v[c][R] = static_cast<T>(alpha * v[3 * k + c] / static_cast<double>(sk));
  }
  gram_schmidt(m);
  m.store(Rt2, k);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a <= R; ++a) m.v[c][a] *= sk;
  m.store(Yt2, k);
}

// Split a factor Yt (FP64, rank r) into (Rt, s) of precision T:
// s_k = sqrt(|Y_k|^2 / 3) (s_0 forced to 1), R_k = Gram-Schmidt(Y_k / s_k),
// and Ytc = s R in precision T.
template <typename T, int R>
__global__ void split_kernel(int32_t N, const double* __restrict__ Yt, T* __restrict__ Rt, T* __restrict__ s,
                             T* __restrict__ Ytc) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  const double* y = Yt + static_cast<int64_t>(k) * 3 * R;
  double nn = 0.0;
  for (int e = 0; e < 3 * R; ++e) nn += y[e] * y[e];
  const double sk = sqrt(nn / 3.0);
  Blk<double, R> m;
  for (int c = 0; c < 3; ++c)
    for (int a = 0; a < R; ++a) m.v[c][a] = y[c * R + a] / sk;
  gram_schmidt(m);
  const double sn = (k == 0) ? 1.0 : sk;
  for (int c = 0; c < 3; ++c)
    for (int a = 0; a < R; ++a) {
      Rt[static_cast<int64_t>(k) * 3 * R + c * R + a] = static_cast<T>(m.v[c][a]);
      Ytc[static_cast<int64_t>(k) * 3 * R + c * R + a] = static_cast<T>(sn * m.v[c][a]);
    }
  s[k] = static_cast<T>(sn);
}

// Yt = s Rt
template <typename T, int R>
__global__ void scale_kernel(int32_t N, const T* __restrict__ Rt, const T* __restrict__ s, T* __restrict__ Yt) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  const T sk = s[k];
  for (int e = 0; e < 3 * R; ++e) Yt[static_cast<int64_t>(k) * 3 * R + e] = sk * Rt[static_cast<int64_t>(k) * 3 * R + e];
}

// U^0 = [I, ..., I] (Algorithm "Riemannian Staircase", initialisation), padded
// with zero rows for r > 3; with lift > 0 every block is first perturbed by
// lift * u, u uniform in [-1, 1] from a counter-based hash (splitmix64) of the
// entry index, then re-orthonormalised, so rows beyond the third are not
// stuck at zero.  s = 1.
template <typename T, int R>
__global__ void init_kernel(int32_t N, double lift, uint64_t seed, T* Rt, T* s) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  Blk<double, R> m;
  for (int c = 0; c < 3; ++c)
    for (int a = 0; a < R; ++a) {
      double v = (a == c) ? 1.0 : 0.0;
      if (lift > 0.0) {
        uint64_t z = (static_cast<uint64_t>(k) * 3 * R + c * R + a) + seed * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        v += lift * (static_cast<double>(z >> 11) * (2.0 / 9007199254740992.0) - 1.0);
      }
      m.v[c][a] = v;
    }
  gram_schmidt(m);
  for (int c = 0; c < 3; ++c)
    for (int a = 0; a < R; ++a) Rt[static_cast<int64_t>(k) * 3 * R + c * R + a] = static_cast<T>(m.v[c][a]);
  s[k] = T(1);
}

template <typename T>
__global__ __launch_bounds__(kVB) void vec_dot_kernel(const T* __restrict__ a, const T* __restrict__ b, int64_t n,
                                                     double* part) {
  double v[1] = {0.0};
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kVB + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kVB)
    v[0] += static_cast<double>(a[i]) * static_cast<double>(b[i]);
  write_partials<1>(v, part);
}

}  // namespace

template <typename T>
double vec_dot(const T* a, const T* b, int64_t n, double* part, int blocks, hipStream_t st) {
  hipLaunchKernelGGL((vec_dot_kernel<T>), dim3(blocks), dim3(kVB), 0, st, a, b, n, part);
  XM_LAUNCH_CHECK("vec_dot_kernel");
  double out = 0.0;
  read_partials(part, blocks, 1, &out, st);
  return out;
}
template double vec_dot<float>(const float*, const float*, int64_t, double*, int, hipStream_t);
template double vec_dot<double>(const double*, const double*, int64_t, double*, int, hipStream_t);

// ---------------------------------------------------------------------------
// Host launchers.  `part` must hold cdiv(N, 256) * NQ doubles.
#define XM_DISPATCH_R(r, CALL)                                            \
  switch (r) {                                                            \
    case 3: { constexpr int R = 3; CALL; } break;                          \
    case 4: { constexpr int R = 4; CALL; } break;                          \
    case 5: { constexpr int R = 5; CALL; } break;                          \
    case 6: { constexpr int R = 6; CALL; } break;                          \
    case 7: { constexpr int R = 7; CALL; } break;                          \
    case 8: { constexpr int R = 8; CALL; } break;                          \
    default: throw Error(XM_EINVAL, "rank must be in [3, 8]");            \
  }

template <typename T>
void Manifold<T>::grad(int r, const T* Rt, const T* s, const T* G, T* gR, T* gs, T* Sc, T* ec, double* part,
                       hipStream_t st) const {
  XM_DISPATCH_R(r, hipLaunchKernelGGL((grad_kernel<T, R>), dim3(blocks()), dim3(kB), 0, st, N, Rt, s, G, gR,
                                      gs, Sc, ec, qkk, lam, part));
  XM_LAUNCH_CHECK("grad_kernel");
}

template <typename T>
void Manifold<T>::ydot(int r, const T* Rt, const T* s, const T* resR, const T* ress, T* dR, T* ds, double beta,
                       int mode, T* Ydot, hipStream_t st) const {
  XM_DISPATCH_R(r, hipLaunchKernelGGL((ydot_kernel<T, R>), dim3(blocks()), dim3(kB), 0, st, N, Rt, s, resR, ress,
                                      dR, ds, beta, mode, qkk, pscale, Ydot));
  XM_LAUNCH_CHECK("ydot_kernel");
}

template <typename T>
void Manifold<T>::hess(int r, const T* Rt, const T* s, const T* G, const T* Sc, const T* ec, const T* dR,
                       const T* ds, const T* Gd, const T* etaR, const T* etas, T* HR, T* Hs, double* part,
                       hipStream_t st, bool anchor0) const {
  XM_DISPATCH_R(r, hipLaunchKernelGGL((hess_kernel<T, R>), dim3(blocks()), dim3(kB), 0, st, N, Rt, s, G, Sc, ec,
                                      dR, ds, Gd, etaR, etas, HR, Hs, qkk, pscale, lam, part, anchor0 ? 1 : 0));
  XM_LAUNCH_CHECK("hess_kernel");
}

template <typename T>
void Manifold<T>::tcg_update(int r, const T* s, double alpha, int mode, const T* dR, const T* ds, const T* HdR,
                             const T* Hds, T* etaR, T* etas, T* HetaR, T* Hetas, T* resR, T* ress, double* part,
                             hipStream_t st) const {
  XM_DISPATCH_R(r, hipLaunchKernelGGL((tcg_update_kernel<T, R>), dim3(blocks()), dim3(kB), 0, st, N, s, alpha,
                                      mode, static_cast<const double*>(nullptr), dR, ds, HdR, Hds, etaR, etas, HetaR,
                                      Hetas, resR, ress, qkk, pscale, part));
  XM_LAUNCH_CHECK("tcg_update_kernel");
}

template <typename T>
void Manifold<T>::tcg_step_update(int r, const T* s, const double* hess_part, double z_r, double delta2,
                                  double* ctl, const T* dR, const T* ds, const T* HdR, const T* Hds, T* etaR,
                                  T* etas, T* HetaR, T* Hetas, T* resR, T* ress, double* part,
                                  hipStream_t st) const {
  hipLaunchKernelGGL(tcg_step_kernel, dim3(1), dim3(64), 0, st, hess_part, static_cast<int>(blocks()), z_r, delta2,
                     ctl);
  XM_LAUNCH_CHECK("tcg_step_kernel");
  XM_DISPATCH_R(r, hipLaunchKernelGGL((tcg_update_kernel<T, R>), dim3(blocks()), dim3(kB), 0, st, N, s, 0.0, 0,
                                      static_cast<const double*>(ctl), dR, ds, HdR, Hds, etaR, etas, HetaR, Hetas,
                                      resR, ress, qkk, pscale, part));
  XM_LAUNCH_CHECK("tcg_update_kernel");
}

template <typename T>
void Manifold<T>::retract(int r, const T* Rt, const T* s, const T* etaR, const T* etas, T* Rt2, T* s2, T* Yt2,
                          hipStream_t st) const {
  XM_DISPATCH_R(r, hipLaunchKernelGGL((retract_kernel<T, R>), dim3(blocks()), dim3(kB), 0, st, N, Rt, s, etaR,
                                      etas, Rt2, s2, Yt2));
  XM_LAUNCH_CHECK("retract_kernel");
}

template <typename T>
void Manifold<T>::model(int r, const T* s, const T* s2, const T* gR, const T* gs, const T* etaR, const T* etas,
                        const T* HetaR, const T* Hetas, const T* Yt, const T* G, const T* Yt2, const T* G2,
                        double* part, hipStream_t st) const {
  XM_DISPATCH_R(r, hipLaunchKernelGGL((model_kernel<T, R>), dim3(blocks()), dim3(kB), 0, st, N, s, s2, lam, gR, gs,
                                      etaR, etas, HetaR, Hetas, Yt, G, Yt2, G2, part));
  XM_LAUNCH_CHECK("model_kernel");
}

template <typename T>
void Manifold<T>::escape(int r, const T* Rt, const T* s, const double* v, double alpha, T* Rt2, T* Yt2,
                         hipStream_t st) const {
  switch (r) {
    case 3: hipLaunchKernelGGL((escape_kernel<T, 3>), dim3(blocks()), dim3(kB), 0, st, N, Rt, s, v, alpha, Rt2, Yt2); break;
    case 4: hipLaunchKernelGGL((escape_kernel<T, 4>), dim3(blocks()), dim3(kB), 0, st, N, Rt, s, v, alpha, Rt2, Yt2); break;
    case 5: hipLaunchKernelGGL((escape_kernel<T, 5>), dim3(blocks()), dim3(kB), 0, st, N, Rt, s, v, alpha, Rt2, Yt2); break;
    case 6: hipLaunchKernelGGL((escape_kernel<T, 6>), dim3(blocks()), dim3(kB), 0, st, N, Rt, s, v, alpha, Rt2, Yt2); break;
    case 7: hipLaunchKernelGGL((escape_kernel<T, 7>), dim3(blocks()), dim3(kB), 0, st, N, Rt, s, v, alpha, Rt2, Yt2); break;
    default: throw Error(XM_EINVAL, "escape: rank must be in [3, 7]");
  }
  XM_LAUNCH_CHECK("escape_kernel");
}

template <typename T>
void Manifold<T>::split(int r, const double* Yt, T* Rt, T* s, T* Ytc, hipStream_t st) const {
  XM_DISPATCH_R(r, hipLaunchKernelGGL((split_kernel<T, R>), dim3(blocks()), dim3(kB), 0, st, N, Yt, Rt, s, Ytc));
  XM_LAUNCH_CHECK("split_kernel");
}

template <typename T>
void Manifold<T>::scale(int r, const T* Rt, const T* s, T* Yt, hipStream_t st) const {
  XM_DISPATCH_R(r, hipLaunchKernelGGL((scale_kernel<T, R>), dim3(blocks()), dim3(kB), 0, st, N, Rt, s, Yt));
  XM_LAUNCH_CHECK("scale_kernel");
}

template <typename T>
void Manifold<T>::init(int r, double lift, T* Rt, T* s, hipStream_t st) const {
  XM_DISPATCH_R(r, hipLaunchKernelGGL((init_kernel<T, R>), dim3(blocks()), dim3(kB), 0, st, N, lift,
                                      static_cast<uint64_t>(2025), Rt, s));
  XM_LAUNCH_CHECK("init_kernel");
}

template struct Manifold<float>;
template struct Manifold<double>;

}  // namespace xm
