// C ABI of libxm (declared and documented in include/xm.h).
#include <cmath>
#include <cstdio>
#include <string>

#include "problem.h"

xm_problem::~xm_problem() {
  for (auto& e : events) {
    (void)hipEventDestroy(e.start);
    (void)hipEventDestroy(e.stop);
  }
}

namespace {
thread_local std::string g_err;

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

xm_status fail(xm_status code, const char* msg) {
  g_err = msg;
  return code;
}
}  // namespace

#define XM_API_TRY \
  try {            \
    g_err.clear();
#define XM_API_CATCH                                    \
  }                                                     \
  catch (const xm::Error& e) {                          \
    return fail(e.code, e.what());                      \
  }                                                     \
  catch (const std::bad_alloc&) {                       \
    return fail(XM_ENOMEM, "host allocation failed");   \
  }                                                     \
  catch (const std::exception& e) {                     \
    return fail(XM_EHIP, e.what());                     \
  }

extern "C" {

xm_status xm_build_Q(int32_t N, int32_t M, int64_t n_obs, const int32_t* frame, const int32_t* landmark,
                     const void* u, xm_dtype u_dtype, const void* w, xm_dtype w_dtype, uint32_t copies,
                     void* stream, xm_problem** out) {
  XM_API_TRY
  if (!out) return fail(XM_EINVAL, "out must be non-NULL");
  *out = nullptr;
  auto P = xm::build_problem(N, M, n_obs, frame, landmark, u, u_dtype, w, w_dtype, nullptr, copies,
                             as_stream(stream));
  *out = P.release();
  return XM_OK;
  XM_API_CATCH
}

xm_status xm_build_Q_masked(int32_t N, int32_t M, int64_t n_obs, const int32_t* frame, const int32_t* landmark,
                            const void* u, xm_dtype u_dtype, const void* w, xm_dtype w_dtype, const uint8_t* mask,
                            uint32_t copies, void* stream, xm_problem** out) {
  XM_API_TRY
  if (!out) return fail(XM_EINVAL, "out must be non-NULL");
  *out = nullptr;
  auto P = xm::build_problem(N, M, n_obs, frame, landmark, u, u_dtype, w, w_dtype, mask, copies,
                             as_stream(stream));
  *out = P.release();
  return XM_OK;
  XM_API_CATCH
}

xm_status xm_residuals(xm_problem* p, const double* R, const double* s, int32_t frame_units, double* e,
                       double* score, void* stream) {
  XM_API_TRY
  if (!p || !R || !s || (!e && !score)) return fail(XM_EINVAL, "NULL argument");
  if (frame_units != 0 && frame_units != 1) return fail(XM_EINVAL, "frame_units must be 0 or 1");
  xm::residuals(p, R, s, frame_units, e, score, as_stream(stream));
  return XM_OK;
  XM_API_CATCH
}

xm_status xm_drop_largest(const double* score, int64_t n, double frac, uint8_t* keep, int64_t* n_dropped,
                          void* stream) {
  XM_API_TRY
  if (!score || !keep) return fail(XM_EINVAL, "NULL argument");
  const int64_t k = xm::drop_largest(score, n, frac, keep, as_stream(stream));
  if (n_dropped) *n_dropped = k;
  return XM_OK;
  XM_API_CATCH
}

xm_status xm_guard_frames(int32_t N, int32_t M, int64_t n, const int32_t* frame, const int32_t* landmark,
                          int32_t min_links, uint8_t* keep, int64_t* n_restored, void* stream) {
  XM_API_TRY
  if (!frame || !landmark || !keep) return fail(XM_EINVAL, "NULL argument");
  const int64_t r = xm::guard_frames(N, M, n, frame, landmark, min_links, keep, as_stream(stream));
  if (n_restored) *n_restored = r;
  return XM_OK;
  XM_API_CATCH
}

void xm_free(xm_problem* p) { delete p; }

xm_status xm_memory_info(int64_t* live_bytes, int64_t* cached_bytes) {
  if (!live_bytes && !cached_bytes) return fail(XM_EINVAL, "NULL argument");
  size_t live = 0, cached = 0;
  xm::pool_usage(&live, &cached);
  if (live_bytes) *live_bytes = static_cast<int64_t>(live);
  if (cached_bytes) *cached_bytes = static_cast<int64_t>(cached);
  g_err.clear();
  return XM_OK;
}

int64_t xm_memory_trim(void) { return static_cast<int64_t>(xm::pool_trim()); }

xm_status xm_get_info(const xm_problem* p, xm_problem_info* info) {
  if (!p || !info) return fail(XM_EINVAL, "NULL argument");
  info->N = p->N;
  info->M = p->M;
  info->n_obs = p->n_obs;
  info->n_in = p->n_in;
  info->nnz_blocks = p->nnzb;
  info->n_pairs = p->n_pairs;
  info->ld = p->ld;
  info->copies = static_cast<int32_t>(p->copies);
  info->qbar = p->qbar;
  info->build_ms = p->build_ms;
  info->scale_reg = p->scale_reg;
  g_err.clear();
  return XM_OK;
}

xm_status xm_set_scale_reg(xm_problem* p, double lambda) {
  if (!p) return fail(XM_EINVAL, "NULL argument");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(XM_EINVAL, "lambda must be finite and >= 0");
  p->scale_reg = lambda;
  g_err.clear();
  return XM_OK;
}

xm_status xm_build_stats(const xm_problem* p, xm_kernel_stat* out, int32_t cap, int32_t* count) {
  if (!p || !count || (cap > 0 && !out)) return fail(XM_EINVAL, "NULL argument");
  const int n = static_cast<int>(p->build_stats.size());
  *count = n;
  for (int k = 0; k < n && k < cap; ++k) {
    const auto& st = p->build_stats[k];
    xm_kernel_stat& o = out[k];
    std::snprintf(o.name, sizeof(o.name), "%s", st.name);
    o.launches = st.launches;
    o.total_ms = st.ms;
    o.bytes = st.bytes;
    o.flops = st.flops;
  }
  g_err.clear();
  return XM_OK;
}

xm_status xm_get_Q_rows(const xm_problem* p, int32_t row0, int32_t nrows, double* out, void* stream) {
  XM_API_TRY
  if (!p || !out) return fail(XM_EINVAL, "NULL argument");
  if (row0 < 0 || nrows < 0 || row0 + static_cast<int64_t>(nrows) > p->n3) return fail(XM_EINVAL, "row range out of bounds");
  if (nrows == 0) return XM_OK;
  hipStream_t s = as_stream(stream);
  xm::get_q_rows(p, row0, nrows, out, s);
  XM_HIP(hipStreamSynchronize(s));
  return XM_OK;
  XM_API_CATCH
}

xm_status xm_spmm(xm_problem* p, xm_dtype dtype, const double* Y, int32_t r, double* out, void* stream) {
  XM_API_TRY
  if (!p || !Y || !out) return fail(XM_EINVAL, "NULL argument");
  if (r < 1 || r > 8) return fail(XM_EINVAL, "r must be in [1, 8]");
  hipStream_t s = as_stream(stream);
  const int n = p->n3;
  if (dtype == XM_F64) {
    xm::DevBuf<double> Yt(static_cast<size_t>(n) * r), G(static_cast<size_t>(n) * r);
    xm::transpose_rows<double, double>(Y, r, n, Yt.ptr, s);
    xm::spmm_yt<double>(p, XM_F64, Yt.ptr, r, G.ptr, s);
    xm::transpose_rows<double, double>(G.ptr, n, r, out, s);
    XM_HIP(hipStreamSynchronize(s));
  } else if (dtype == XM_F32 || dtype == XM_BF16) {
    xm::DevBuf<float> Yt(static_cast<size_t>(n) * r), G(static_cast<size_t>(n) * r);
    xm::transpose_rows<double, float>(Y, r, n, Yt.ptr, s);
    xm::spmm_yt<float>(p, dtype, Yt.ptr, r, G.ptr, s);
    xm::transpose_rows<float, double>(G.ptr, n, r, out, s);
    XM_HIP(hipStreamSynchronize(s));
  } else {
    return fail(XM_EINVAL, "unknown dtype");
  }
  return XM_OK;
  XM_API_CATCH
}

}  // extern "C"

namespace {
// temporaries of xm_spmm_noalloc: Y and the product in the kernels' layout,
// then those of the product itself
size_t noalloc_need(const xm_problem* p, xm_dtype dtype, int r) {
  const size_t vb = (dtype == XM_F64) ? sizeof(double) : sizeof(float);
  return 2 * (static_cast<size_t>(p->n3) * r * vb + 256) +
         xm::product_scratch_bytes(p, dtype, r, XM_ROLE_RESIDUAL, false);
}

template <typename T>
void noalloc_product(xm_problem* p, xm_dtype dtype, const double* Y, int r, double* out, hipStream_t s) {
  xm::Scratch sc{xm::noalloc_scratch_base(), xm::kNoallocScratchBytes, 0};
  xm::DevBuf<T> unused;  // the fixed region serves every take(): never allocated
  const int n = p->n3;
  T* Yt = xm::take<T>(&sc, unused, static_cast<size_t>(n) * r, s);
  T* G = xm::take<T>(&sc, unused, static_cast<size_t>(n) * r, s);
  xm::transpose_rows<double, T>(Y, r, n, Yt, s);
  xm::spmm_yt<T>(p, dtype, Yt, r, G, s, XM_ROLE_RESIDUAL, &sc);
  xm::transpose_rows<T, double>(G, n, r, out, s);
}
}  // namespace

extern "C" {

xm_status xm_spmm_noalloc_bytes(const xm_problem* p, xm_dtype dtype, int32_t r, int64_t* bytes) {
  XM_API_TRY
  if (!p || !bytes) return fail(XM_EINVAL, "NULL argument");
  if (r < 1 || r > 8) return fail(XM_EINVAL, "r must be in [1, 8]");
  if (dtype != XM_F64 && dtype != XM_F32 && dtype != XM_BF16) return fail(XM_EINVAL, "unknown dtype");
  *bytes = static_cast<int64_t>(noalloc_need(p, dtype, r));
  return XM_OK;
  XM_API_CATCH
}

xm_status xm_spmm_noalloc(xm_problem* p, xm_dtype dtype, const double* Y, int32_t r, double* out,
                          void* stream) {
  XM_API_TRY
  if (!p || !Y || !out) return fail(XM_EINVAL, "NULL argument");
  if (r < 1 || r > 8) return fail(XM_EINVAL, "r must be in [1, 8]");
  if (dtype != XM_F64 && dtype != XM_F32 && dtype != XM_BF16) return fail(XM_EINVAL, "unknown dtype");
  const int kind = p->spmm_kind[XM_ROLE_RESIDUAL][dtype];
  if (dtype == XM_F64 && kind != XM_SPMM_FACTORED && !p->Q64.ptr) return fail(XM_EINVAL, "the dense FP64 Q was not kept");
  if (dtype == XM_F32 && kind != XM_SPMM_FACTORED && !p->Q32.ptr)
    return fail(XM_EINVAL, "the FP32 copy of Q was not kept (XM_KEEP_F32)");
  if (dtype == XM_F32 && kind == XM_SPMM_FACTORED && !p->fac32.ptr)
    return fail(XM_EINVAL, "the FP32 factors were not kept (XM_KEEP_F32)");
  if (dtype == XM_BF16 && !p->Q16.ptr) return fail(XM_EINVAL, "the BF16 copy of Q was not kept (XM_KEEP_BF16)");
  const size_t need = noalloc_need(p, dtype, r);
  if (need > xm::kNoallocScratchBytes) {
    char msg[200];
    std::snprintf(msg, sizeof(msg), "xm_spmm_noalloc: this product needs %zu bytes of scratch, the fixed array holds %zu",
                  need, xm::kNoallocScratchBytes);
    return fail(XM_EINVAL, msg);
  }
  hipStream_t s = as_stream(stream);
  if (dtype == XM_F64) noalloc_product<double>(p, dtype, Y, r, out, s);
  else noalloc_product<float>(p, dtype, Y, r, out, s);
  return XM_OK;
  XM_API_CATCH
}

void xm_default_opts(xm_solve_opts* o) {
  if (!o) return;
  *o = xm_solve_opts{};
  o->r0 = 5;
  o->r_max = 7;
  o->lift = 1.0;
  o->compute = XM_F64;
  o->grad_tol = 0.0;
  o->cert_tol = 0.0;
  o->max_outer = 0;
  o->max_inner = 0;
  o->delta0 = 0.0;
  o->lanczos_max = 0;
  o->lanczos_tol = 0.0;
  o->precondition = 1;
  o->verbose = 0;
}

xm_status xm_bm_solve(xm_problem* p, const xm_solve_opts* opts, const double* Y0, int32_t r_in, double* Y_out,
                      xm_solve_info* info, void* stream) {
  XM_API_TRY
  if (!p || !opts) return fail(XM_EINVAL, "NULL argument");
  const xm_status st = xm::bm_solve(p, *opts, Y0, r_in, Y_out, info, as_stream(stream));
  if (st == XM_ENOCONV) g_err = "iteration cap reached before the gradient tolerance";
  return st;
  XM_API_CATCH
}

xm_status xm_certify(xm_problem* p, const double* Y, int32_t r, double tol, int32_t max_iter, double* v_min,
                     xm_cert* cert, void* stream) {
  XM_API_TRY
  if (!p || !Y || !cert) return fail(XM_EINVAL, "NULL argument");
  if (r < 1 || r > 8) return fail(XM_EINVAL, "r must be in [1, 8]");
  hipStream_t s = as_stream(stream);
  const int n = p->n3;
  xm::DevBuf<double> Yt(static_cast<size_t>(n) * r);
  xm::transpose_rows<double, double>(Y, r, n, Yt.ptr, s);
  const double t = (tol > 0) ? tol : 1e-7;
  const xm::CertResult c = xm::certify_yt(p, Yt.ptr, r, t, max_iter, 0.0, v_min, s);
  cert->lambda_min = c.lambda_min;
  cert->ritz_residual = c.ritz_residual;
  cert->lambda_bound = c.lambda_bound;
  cert->primal = c.primal;
  cert->dual = c.dual;
  cert->qbar = p->qbar;
  cert->grad_norm = c.stat_res;
  cert->defl_min = c.defl_min;
  cert->defl_cross = c.defl_cross;
  cert->certified = c.certified ? 1 : 0;
  cert->iters = c.iters;
  // eq. suboptimality: the rounded point's cost against the relaxation's value at Y
  cert->rho_hat = cert->eta = std::nan("");
  if (r >= 3) {
    xm::DevBuf<double> R(9 * static_cast<size_t>(p->N)), sc(p->N);
    double rho = 0.0;
    xm::round_yt(p, Y, r, R.ptr, sc.ptr, &rho, s);
    cert->rho_hat = rho;
    cert->eta = (rho - c.primal) / (1.0 + std::fabs(rho) + std::fabs(c.primal));
  }
  return XM_OK;
  XM_API_CATCH
}

xm_status xm_round(xm_problem* p, const double* Y, int32_t r, double* R_out, double* s_out, double* rho_hat,
                   void* stream) {
  XM_API_TRY
  if (!p) return fail(XM_EINVAL, "NULL argument");
  xm::round_yt(p, Y, r, R_out, s_out, rho_hat, as_stream(stream));
  return XM_OK;
  XM_API_CATCH
}

xm_status xm_align_similarity(int64_t n, const double* P, const double* Q, const double* w, double* out,
                              void* stream) {
  XM_API_TRY
  xm::align_similarity(n, P, Q, w, out, as_stream(stream));
  return XM_OK;
  XM_API_CATCH
}

namespace {
xm_status set_kind(xm_problem* p, int role, xm_dtype dtype, xm_spmm_kind kind) {
  if (!p) return fail(XM_EINVAL, "NULL argument");
  if (dtype < XM_F64 || dtype > XM_BF16) return fail(XM_EINVAL, "unknown dtype");
  if (kind != XM_SPMM_FULL && kind != XM_SPMM_UPPER && kind != XM_SPMM_FACTORED)
    return fail(XM_EINVAL, "unknown product kernel");
  if (kind == XM_SPMM_FACTORED && dtype == XM_BF16) return fail(XM_EINVAL, "no BF16 factored product");
  if (role < 0) {
    p->spmm_kind[XM_ROLE_RESIDUAL][dtype] = kind;
    p->spmm_kind[XM_ROLE_CURVATURE][dtype] = kind;
  } else {
    p->spmm_kind[role][dtype] = kind;
  }
  return XM_OK;
}
}  // namespace

xm_status xm_set_spmm_kind(xm_problem* p, xm_dtype dtype, xm_spmm_kind kind) {
  XM_API_TRY
  return set_kind(p, -1, dtype, kind);
  XM_API_CATCH
}

xm_status xm_set_product_kind(xm_problem* p, xm_product_role role, xm_dtype dtype, xm_spmm_kind kind) {
  XM_API_TRY
  if (role != XM_ROLE_RESIDUAL && role != XM_ROLE_CURVATURE) return fail(XM_EINVAL, "unknown product role");
  return set_kind(p, role, dtype, kind);
  XM_API_CATCH
}

xm_status xm_get_product_kind(const xm_problem* p, xm_product_role role, xm_dtype dtype, xm_spmm_kind* kind) {
  XM_API_TRY
  if (!p || !kind) return fail(XM_EINVAL, "NULL argument");
  if (role != XM_ROLE_RESIDUAL && role != XM_ROLE_CURVATURE) return fail(XM_EINVAL, "unknown product role");
  if (dtype < XM_F64 || dtype > XM_BF16) return fail(XM_EINVAL, "unknown dtype");
  *kind = static_cast<xm_spmm_kind>(p->spmm_kind[role][dtype]);
  return XM_OK;
  XM_API_CATCH
}

xm_status xm_spmm_timing(xm_problem* p, int32_t enable) {
  XM_API_TRY
  if (!p) return fail(XM_EINVAL, "NULL argument");
  p->timing = enable != 0;
  return XM_OK;
  XM_API_CATCH
}

xm_status xm_spmm_stats(xm_problem* p, xm_spmm_counters* out, int32_t reset) {
  XM_API_TRY
  if (!p || !out) return fail(XM_EINVAL, "NULL argument");
  *out = xm_spmm_counters{};
  for (size_t i = 0; i < p->events_used; ++i) {
    auto& e = p->events[i];
    XM_HIP(hipEventSynchronize(e.stop));
    float ms = 0.f;
    XM_HIP(hipEventElapsedTime(&ms, e.start, e.stop));
    out->launches[e.dtype] += 1;
    out->total_ms[e.dtype] += ms;
    out->bytes_per_launch[e.dtype] += e.bytes;
  }
  for (int d = 0; d < XM_STATS_SLOTS; ++d)
    if (out->launches[d] > 0) out->bytes_per_launch[d] /= static_cast<double>(out->launches[d]);
  if (reset) p->events_used = 0;
  return XM_OK;
  XM_API_CATCH
}

xm_status xm_recover_tp(xm_problem* p, const double* R, const double* s, double* t, double* pts, void* stream) {
  XM_API_TRY
  if (!p) return fail(XM_EINVAL, "NULL argument");
  xm::recover_tp(p, R, s, t, pts, as_stream(stream));
  return XM_OK;
  XM_API_CATCH
}

xm_status xm_adjoint(xm_problem* p, const double* R, const double* s, const double* gR, const double* gs,
                     double gcost, void* gu, void* gw, xm_dtype g_dtype, double cg_tol, int32_t cg_max,
                     xm_adjoint_info* info, void* stream) {
  XM_API_TRY
  if (!p) return fail(XM_EINVAL, "NULL argument");
  const xm::AdjointResult r =
      xm::adjoint(p, R, s, gR, gs, gcost, gu, gw, g_dtype, cg_tol, cg_max, as_stream(stream));
  if (info) {
    info->cg_iters = r.cg_iters;
    info->cg_residual = r.cg_residual;
    info->cost = r.cost;
  }
  if (r.negative_curvature) {
    g_err = "adjoint: the Hessian has a direction of non-positive curvature (not a tight certified optimum)";
    return XM_ENOCONV;
  }
  if (!r.converged) {
    g_err = "adjoint: CG stopped above its tolerance (cg_residual > cg_tol)";
    return XM_ENOCONV;
  }
  return XM_OK;
  XM_API_CATCH
}

const char* xm_last_error(void) { return g_err.c_str(); }

}  // extern "C"
