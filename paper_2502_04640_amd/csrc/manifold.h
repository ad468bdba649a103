// Host launchers of the per-frame manifold kernels (manifold.hip).
#pragma once

#include "common.h"

namespace xm {

// threads per workgroup of the per-frame kernels (one thread per frame)
constexpr int kFrameBlock = 256;

// <a, b> over n entries, FP64 accumulation; `part` holds `blocks` doubles
// (blocks <= 256).  Synchronises the stream.
template <typename T>
double vec_dot(const T* a, const T* b, int64_t n, double* part, int blocks, hipStream_t st);

template <typename T>
struct Manifold {
  int32_t N;
  // optional per-frame preconditioner: qkk[k] = tr(Q_kk)/3 (NULL: none) and
  // pscale = mean_k s_k^2 q_kk at the current point
  const double* qkk = nullptr;
  double pscale = 1.0;
  // scale regulariser lam sum_{k>=1} (s_k^2 - 1)^2 of App. "Scale
  // Regularization" (0: the plain objective); it enters the cost, the scale
  // part of the gradient and Hessian and the model's cost change
  double lam = 0.0;
  explicit Manifold(int32_t n) : N(n) {}
  // workgroups of the per-frame kernels (one thread per frame)
  unsigned blocks() const { return cdiv(N, kFrameBlock); }

  // G = Q Yt.  part: [blocks][5] = {cost, |grad|^2 (metric), |Y|_F^2, sum s^2 q_kk,
  //                                 pscale * <grad, P grad>}
  void grad(int r, const T* Rt, const T* s, const T* G, T* gR, T* gs, T* Sc, T* ec, double* part,
            hipStream_t st) const;
  // mode 0: d = -res; 1: d = -res + beta d; 2: d unchanged.  Ydot = ds R + s dR.
  void ydot(int r, const T* Rt, const T* s, const T* resR, const T* ress, T* dR, T* ds, double beta, int mode,
            T* Ydot, hipStream_t st) const;
  // part: [blocks][4] = {<d,Hd>, <d,Md>, <eta,Md>, <eta,M eta>} (M: preconditioner, identity if none)
  // anchor0: frame 0 held fixed (its rows of the output are zero)
  void hess(int r, const T* Rt, const T* s, const T* G, const T* Sc, const T* ec, const T* dR, const T* ds,
            const T* Gd, const T* etaR, const T* etas, T* HR, T* Hs, double* part, hipStream_t st,
            bool anchor0 = false) const;
  // part: [blocks][2] = {<res,res>, <res, P res>} (mode 0)
  void tcg_update(int r, const T* s, double alpha, int mode, const T* dR, const T* ds, const T* HdR, const T* Hds,
                  T* etaR, T* etas, T* HetaR, T* Hetas, T* resR, T* ress, double* part, hipStream_t st) const;
  // the same update with its step chosen on the device from hess_kernel's
  // partials (hess_part): interior alpha = z_r / <d,Hd>, or the boundary step
  // when the curvature is not positive or |eta|_M would pass sqrt(delta2);
  // ctl (device, 6 doubles) receives {step, mode, <d,Hd>, <d,Md>, <eta,Md>,
  // <eta,M eta>}; part as tcg_update (mode 0)
  void tcg_step_update(int r, const T* s, const double* hess_part, double z_r, double delta2, double* ctl,
                       const T* dR, const T* ds, const T* HdR, const T* Hds, T* etaR, T* etas, T* HetaR,
                       T* Hetas, T* resR, T* ress, double* part, hipStream_t st) const;
  void retract(int r, const T* Rt, const T* s, const T* etaR, const T* etas, T* Rt2, T* s2, T* Yt2,
               hipStream_t st) const;
  // part: [blocks][3] = {<g,eta>, <eta,Heta>, <Y2-Y, G2+G> + F(s2) - F(s) (the cost change)}
  void model(int r, const T* s, const T* s2, const T* gR, const T* gs, const T* etaR, const T* etas,
             const T* HetaR, const T* Hetas, const T* Yt, const T* G, const T* Yt2, const T* G2, double* part,
             hipStream_t st) const;
  // rank r -> r + 1 along [0; v^T] with step alpha; Rt2 / Yt2 have rank r + 1
  void escape(int r, const T* Rt, const T* s, const double* v, double alpha, T* Rt2, T* Yt2, hipStream_t st) const;
  void split(int r, const double* Yt, T* Rt, T* s, T* Ytc, hipStream_t st) const;
  void scale(int r, const T* Rt, const T* s, T* Yt, hipStream_t st) const;
  // U^0 = [I; 0] per block, optionally lifted by a seeded perturbation of size `lift`
  void init(int r, double lift, T* Rt, T* s, hipStream_t st) const;
};

}  // namespace xm
