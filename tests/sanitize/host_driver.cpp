// Host-code sanitizer run of the library (AddressSanitizer + UndefinedBehavior
// Sanitizer on the host side only; device code is built as usual).  Drives
// every entry point of include/xm.h through the C ABI on a small seeded scene
// and through its error paths, and checks the returned statuses and a few
// invariants.  Built by paper_2502_04640_amd/build.py (build_hostsan) against
// libxm_hostsan.so; run by tests/test_gpu_hostsan.py.  Exit status 0 when every
// check passes; the sanitizers abort the process on the first finding.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "xm.h"

namespace {

int g_fail = 0;

void check(bool ok, const char* what) {
  std::printf("%s %s\n", ok ? "ok  " : "FAIL", what);
  if (!ok) {
    std::printf("     last error: %s\n", xm_last_error());
    ++g_fail;
  }
}

void status(xm_status got, xm_status want, const char* what) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s (status %d, expected %d)", what, static_cast<int>(got),
                static_cast<int>(want));
  check(got == want, buf);
}

// xorshift64* and a uniform double in [0, 1)
struct Rng {
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed * 2685821657736338717ull + 1) {}
  uint64_t next() {
    s ^= s >> 12;
    s ^= s << 25;
    s ^= s >> 27;
    return s * 2685821657736338717ull;
  }
  double uni() { return static_cast<double>(next() >> 11) * (1.0 / 9007199254740992.0); }
  double normal() {
    const double a = uni() + 1e-300, b = uni();
    return std::sqrt(-2.0 * std::log(a)) * std::cos(6.283185307179586 * b);
  }
};

// rotation from a normalised Gaussian quaternion
void rotation(Rng& g, double R[9]) {
  double q[4], n = 0.0;
  for (double& x : q) {
    x = g.normal();
    n += x * x;
  }
  n = std::sqrt(n);
  for (double& x : q) x /= n;
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  const double M[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z),     2 * (x * z + w * y),
                       2 * (x * y + w * z),     1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                       2 * (x * z - w * y),     2 * (y * z + w * x),     1 - 2 * (x * x + y * y)};
  std::memcpy(R, M, sizeof(M));
}

template <typename T>
T* dev(const std::vector<T>& h) {
  T* d = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&d), h.size() * sizeof(T)) != hipSuccess) std::abort();
  if (hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) std::abort();
  return d;
}

template <typename T>
T* dev_zero(size_t n) {
  T* d = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&d), n * sizeof(T)) != hipSuccess) std::abort();
  if (hipMemset(d, 0, n * sizeof(T)) != hipSuccess) std::abort();
  return d;
}

template <typename T>
std::vector<T> host(const T* d, size_t n) {
  std::vector<T> h(n);
  if (hipMemcpy(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess) std::abort();
  return h;
}

}  // namespace

int main() {
  // ---- scene: N frames on a ring, M landmarks seen by 3..5 frames, the first
  // two observations of landmark k by frames k % N and (k + 1) % N (connected
  // view graph); u = d_i (R_i (x - c_i) + noise), weights in [0.5, 1.5]
  const int32_t N = 40, M = 1500;
  Rng g(7);
  std::vector<double> R(9 * N), c(3 * N), d(N), x(3 * M);
  for (int i = 0; i < N; ++i) {
    rotation(g, &R[9 * i]);
    for (int a = 0; a < 3; ++a) c[3 * i + a] = 4.0 * g.normal();
    d[i] = 0.5 + 1.5 * g.uni();
  }
  for (double& v : x) v = 6.0 * g.normal();
  std::vector<int32_t> fr, lm;
  std::vector<double> u, w;
  for (int k = 0; k < M; ++k) {
    const int L = 3 + static_cast<int>(g.next() % 3);
    std::vector<int> seen;
    for (int l = 0; l < L; ++l) {
      int i = (l == 0) ? k % N : (l == 1) ? (k + 1) % N : static_cast<int>(g.next() % N);
      bool dup = false;
      for (int s : seen) dup = dup || (s == i);
      if (dup) continue;
      seen.push_back(i);
      fr.push_back(i);
      lm.push_back(k);
      for (int a = 0; a < 3; ++a) {
        double v = 0.0;
        for (int b = 0; b < 3; ++b) v += R[9 * i + 3 * a + b] * (x[3 * k + b] - c[3 * i + b]);
        u.push_back(d[i] * (v + 0.01 * g.normal()));
      }
      w.push_back(0.5 + g.uni());
    }
  }
  const int64_t n = static_cast<int64_t>(fr.size());
  std::printf("scene: N=%d M=%d n_obs=%lld\n", N, M, static_cast<long long>(n));
  int32_t *dfr = dev(fr), *dlm = dev(lm);
  double *du = dev(u), *dw = dev(w);

  // ---- build, info, products
  xm_problem* P = nullptr;
  status(xm_build_Q(N, M, n, dfr, dlm, du, XM_F64, dw, XM_F64, XM_KEEP_F32 | XM_KEEP_BF16, nullptr, &P), XM_OK,
         "xm_build_Q");
  if (!P) return 1;
  xm_problem_info info{};
  status(xm_get_info(P, &info), XM_OK, "xm_get_info");
  check(info.N == N && info.n_obs == n && info.n_in == n, "info sizes");
  const int32_t n3 = 3 * N;
  std::vector<double> Yh(5 * static_cast<size_t>(n3));
  for (double& v : Yh) v = g.normal();
  double* dY = dev(Yh);
  double* dO = dev_zero<double>(5 * static_cast<size_t>(n3));
  double* dO2 = dev_zero<double>(5 * static_cast<size_t>(n3));
  for (xm_dtype t : {XM_F64, XM_F32, XM_BF16}) status(xm_spmm(P, t, dY, 5, dO, nullptr), XM_OK, "xm_spmm");
  status(xm_spmm(P, XM_F64, dY, 5, dO, nullptr), XM_OK, "xm_spmm f64");
  status(xm_spmm_noalloc(P, XM_F64, dY, 5, dO2, nullptr), XM_OK, "xm_spmm_noalloc f64");
  {
    const auto a = host(dO, 5 * static_cast<size_t>(n3)), b = host(dO2, 5 * static_cast<size_t>(n3));
    check(std::memcmp(a.data(), b.data(), a.size() * sizeof(double)) == 0, "noalloc product bitwise equal");
  }
  int64_t need = 0;
  status(xm_spmm_noalloc_bytes(P, XM_F32, 5, &need), XM_OK, "xm_spmm_noalloc_bytes");
  std::vector<double> rows(3 * static_cast<size_t>(n3));
  double* dRows = dev_zero<double>(rows.size());
  status(xm_get_Q_rows(P, 0, 3, dRows, nullptr), XM_OK, "xm_get_Q_rows");
  xm_kernel_stat ks[8];
  int32_t nks = 0;
  status(xm_build_stats(P, ks, 8, &nks), XM_OK, "xm_build_stats");
  status(xm_spmm_timing(P, 1), XM_OK, "xm_spmm_timing on");
  status(xm_spmm(P, XM_F32, dY, 5, dO, nullptr), XM_OK, "timed xm_spmm");
  xm_spmm_counters ctr{};
  status(xm_spmm_stats(P, &ctr, 1), XM_OK, "xm_spmm_stats");
  status(xm_spmm_timing(P, 0), XM_OK, "xm_spmm_timing off");
  xm_spmm_kind kind;
  status(xm_get_product_kind(P, XM_ROLE_CURVATURE, XM_F32, &kind), XM_OK, "xm_get_product_kind");
  status(xm_set_product_kind(P, XM_ROLE_CURVATURE, XM_F32, XM_SPMM_FACTORED), XM_OK, "xm_set_product_kind");

  // ---- solves (FP64, FP32, BF16-stored Q), certificate, rounding, recovery
  xm_solve_opts o;
  xm_default_opts(&o);
  double* dYs = dev_zero<double>(static_cast<size_t>(o.r_max) * n3);
  xm_solve_info si{};
  for (xm_dtype t : {XM_F32, XM_BF16, XM_F64}) {
    o.compute = t;
    status(xm_bm_solve(P, &o, nullptr, 0, dYs, &si, nullptr), XM_OK, "xm_bm_solve");
    check(si.certified == 1, "solve certified");
  }
  xm_cert cert{};
  double* dv = dev_zero<double>(n3);
  status(xm_certify(P, dYs, si.r, 0.0, 0, dv, &cert, nullptr), XM_OK, "xm_certify");
  check(cert.certified == 1 && std::isfinite(cert.eta), "certificate and eta");
  double *dR = dev_zero<double>(9 * static_cast<size_t>(N)), *ds = dev_zero<double>(N);
  double rho = 0.0;
  status(xm_round(P, dYs, si.r, dR, ds, &rho, nullptr), XM_OK, "xm_round");
  check(std::fabs(rho - si.cost) <= 1e-6 * (1.0 + std::fabs(si.cost)), "rho_hat at a rank-3 optimum equals the cost");
  double *dt = dev_zero<double>(3 * static_cast<size_t>(N)), *dp = dev_zero<double>(3 * static_cast<size_t>(M));
  status(xm_recover_tp(P, dR, ds, dt, dp, nullptr), XM_OK, "xm_recover_tp");

  // ---- adjoint
  double *dgu = dev_zero<double>(3 * static_cast<size_t>(n)), *dgw = dev_zero<double>(n);
  std::vector<double> gs(N, 0.0);
  gs[1] = 1.0;
  double* dgs = dev(gs);
  xm_adjoint_info ai{};
  status(xm_adjoint(P, dR, ds, nullptr, dgs, 1.0, dgu, dgw, XM_F64, 0.0, 0, &ai, nullptr), XM_OK, "xm_adjoint");

  // ---- XM^2 pieces: residuals, deletion, masked build, warm-started solve
  double *de = dev_zero<double>(3 * static_cast<size_t>(n)), *dscore = dev_zero<double>(n);
  status(xm_residuals(P, dR, ds, 1, de, dscore, nullptr), XM_OK, "xm_residuals");
  uint8_t* dkeep = dev_zero<uint8_t>(n);
  int64_t nd = 0;
  status(xm_drop_largest(dscore, n, 0.1, dkeep, &nd, nullptr), XM_OK, "xm_drop_largest");
  check(nd == static_cast<int64_t>(0.1 * static_cast<double>(n)), "dropped count");
  xm_problem* P2 = nullptr;
  status(xm_build_Q_masked(N, M, n, dfr, dlm, du, XM_F64, dw, XM_F64, dkeep, XM_KEEP_F32, nullptr, &P2), XM_OK,
         "xm_build_Q_masked");
  double* dYs2 = dev_zero<double>(static_cast<size_t>(o.r_max) * n3);
  if (P2) {
    o.compute = XM_F32;
    status(xm_bm_solve(P2, &o, dYs, si.r, dYs2, &si, nullptr), XM_OK, "warm-started solve on the masked build");
    status(xm_set_scale_reg(P2, 0.1), XM_OK, "xm_set_scale_reg");
    status(xm_bm_solve(P2, &o, nullptr, 0, dYs2, &si, nullptr), XM_OK, "regularised solve");
    status(xm_adjoint(P2, dR, ds, nullptr, dgs, 1.0, dgu, dgw, XM_F64, 0.0, 0, &ai, nullptr), XM_EINVAL,
           "adjoint refuses a regularised handle");
  }

  // ---- similarity alignment of the recovered positions to the true centres
  double* dc = dev(c);
  double al[14];
  status(xm_align_similarity(N, dt, dc, nullptr, al, nullptr), XM_OK, "xm_align_similarity");
  check(std::isfinite(al[13]) && al[0] > 0.0, "alignment scale and residual");

  // ---- error paths (no device work reaches the kernels)
  xm_problem* bad = nullptr;
  status(xm_build_Q(1, M, n, dfr, dlm, du, XM_F64, dw, XM_F64, 0, nullptr, &bad), XM_EINVAL, "N < 2");
  status(xm_build_Q(N, M, n, nullptr, dlm, du, XM_F64, dw, XM_F64, 0, nullptr, &bad), XM_EINVAL, "NULL frame");
  std::vector<int32_t> fr_bad = fr;
  fr_bad[3] = N + 7;
  int32_t* dfr_bad = dev(fr_bad);
  status(xm_build_Q(N, M, n, dfr_bad, dlm, du, XM_F64, dw, XM_F64, 0, nullptr, &bad), XM_EINVAL,
         "frame index out of range");
  std::vector<double> u_bad = u;
  u_bad[5] = std::nan("");
  double* du_bad = dev(u_bad);
  status(xm_build_Q(N, M, n, dfr, dlm, du_bad, XM_F64, dw, XM_F64, 0, nullptr, &bad), XM_EINVAL, "NaN keypoint");
  status(xm_spmm(P, XM_F64, dY, 9, dO, nullptr), XM_EINVAL, "rank 9 product");
  status(xm_drop_largest(dscore, n, 1.5, dkeep, &nd, nullptr), XM_EINVAL, "fraction above 1");
  status(xm_align_similarity(1, dt, dc, nullptr, al, nullptr), XM_EINVAL, "alignment of one point");
  status(xm_get_info(nullptr, &info), XM_EINVAL, "NULL handle");
  int64_t live = 0, cached = 0;
  status(xm_memory_info(&live, &cached), XM_OK, "xm_memory_info");

  xm_free(P2);
  xm_free(P);
  xm_free(nullptr);
  xm_memory_trim();
  for (void* p : {static_cast<void*>(dfr), static_cast<void*>(dlm), static_cast<void*>(du), static_cast<void*>(dw),
                  static_cast<void*>(dY), static_cast<void*>(dO), static_cast<void*>(dO2), static_cast<void*>(dRows),
                  static_cast<void*>(dYs), static_cast<void*>(dv), static_cast<void*>(dR), static_cast<void*>(ds),
                  static_cast<void*>(dt), static_cast<void*>(dp), static_cast<void*>(dgu), static_cast<void*>(dgw),
                  static_cast<void*>(dgs), static_cast<void*>(de), static_cast<void*>(dscore),
                  static_cast<void*>(dkeep), static_cast<void*>(dc), static_cast<void*>(dfr_bad),
                  static_cast<void*>(du_bad), static_cast<void*>(dYs2)})
    (void)hipFree(p);
  std::printf("%s: %d failed check(s)\n", g_fail ? "FAILED" : "all checks passed", g_fail);
  return g_fail ? 1 : 0;
}
