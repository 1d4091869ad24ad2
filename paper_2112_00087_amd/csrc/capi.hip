// extern "C" entry points of the library (declared and documented in hz.h).
// No C++ exception crosses this boundary.
#include <chrono>
#include <new>

#include <complex>

#include "ops.h"
#include "solve.h"

const char* hz_last_error_str();
int schwarz_solve(hz_ctx ctx, const hz_solve_opts& o, const z_t* f, z_t* p, hz_solve_info* info);
void dd_optimised_alpha(double k, double Hsub, double h, int sides, std::complex<double>* out);
int sweep_solve(hz_ctx ctx, int nfreq, const double* freqs, const z_t* F, z_t* P, const hz_solve_opts& o,
                hz_solve_info* infos);
int adjoint_solve(hz_ctx ctx, const hz_solve_opts& o, const z_t* p, const z_t* g, z_t* lam, double* dJ_dbeta,
                  double* dJ_deta, hz_solve_info* info);
int receiver_objective(hz_ctx ctx, int nrec, const int* rec_host, const z_t* p, double* J_host, z_t* g);
int sweep_time_spmm(hz_ctx ctx, int nfreq, const double* freqs, int precision, int reps, double* avg_ms,
                    int32_t* variant, int64_t* bytes);
int sweep_apply(hz_ctx ctx, int nfreq, const double* freqs, int precision, const z_t* X, z_t* Y,
                int32_t* variant);

#define HZ_GUARD_BEGIN try {
#define HZ_GUARD_END                                                          \
  }                                                                           \
  catch (const std::bad_alloc&) {                                             \
    return hz_fail(HZ_ERR_OOM, "host allocation failed");                     \
  }                                                                           \
  catch (...) {                                                               \
    return hz_fail(HZ_ERR_INVALID, "unexpected exception in the library");    \
  }

int noalloc_setup(int device);

int validate_opts(const hz_solve_opts* o) {
  if (!o) return hz_fail(HZ_ERR_INVALID, "opts is NULL");
  if (o->method < HZ_GMRES || o->method > HZ_TFQMR) return hz_fail(HZ_ERR_INVALID, "unknown method %d", o->method);
  if (o->precision != HZ_FP64 && o->precision != HZ_MIXED)
    return hz_fail(HZ_ERR_INVALID, "unknown precision %d", o->precision);
  if (o->precond != HZ_JACOBI && o->precond != HZ_NONE) return hz_fail(HZ_ERR_INVALID, "unknown precond %d", o->precond);
  if (o->method == HZ_GMRES && (o->restart < 1 || o->restart > 128))
    return hz_fail(HZ_ERR_INVALID, "restart %d not in 1..128", o->restart);
  if (o->method == HZ_BICGSTABL && (o->restart < 1 || o->restart > 8))
    return hz_fail(HZ_ERR_INVALID, "BiCGStab(l): l = restart %d not in 1..8", o->restart);
  if (o->method == HZ_SCHWARZ && (o->restart < 1 || o->restart > 1000))
    return hz_fail(HZ_ERR_INVALID, "interface restart %d not in 1..1000", o->restart);
  if (o->max_matvec < 1) return hz_fail(HZ_ERR_INVALID, "max_matvec must be >= 1");
  if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return hz_fail(HZ_ERR_INVALID, "tol must be finite and > 0");
  if (!(o->inner_tol >= 0.0) || !std::isfinite(o->inner_tol)) return hz_fail(HZ_ERR_INVALID, "bad inner_tol");
  if (o->inner_restart < 0 || o->inner_restart > 128) return hz_fail(HZ_ERR_INVALID, "inner_restart not in 0..128");
  if (o->dd_richardson < 0) return hz_fail(HZ_ERR_INVALID, "dd_richardson must be >= 0");
  if (o->method == HZ_SCHWARZ && o->dd_inner != HZ_GMRES && o->dd_inner != HZ_BICGSTAB &&
      o->dd_inner != HZ_BICGSTABL && o->dd_inner != HZ_TFQMR)
    return hz_fail(HZ_ERR_INVALID, "dd_inner must be HZ_GMRES, HZ_BICGSTAB, HZ_BICGSTABL or HZ_TFQMR");
  if (o->method == HZ_SCHWARZ && o->dd_inner == HZ_BICGSTABL && o->inner_restart > 8)
    return hz_fail(HZ_ERR_INVALID, "local BiCGStab(l): l = inner_restart %d not in 0..8", o->inner_restart);
  return HZ_OK;
}

static int check_ctx(hz_ctx ctx) {
  if (!ctx) return hz_fail(HZ_ERR_INVALID, "ctx is NULL");
  int dev = -1;
  HZ_HIP(hipGetDevice(&dev));
  if (dev != ctx->device) HZ_HIP(hipSetDevice(ctx->device));
  return HZ_OK;
}

extern "C" {

const char* hz_last_error(void) { return hz_last_error_str(); }

int hz_assemble(const hz_mesh* mesh, const hz_c128* beta, const double* eta, void* hip_stream, hz_ctx* out) {
  HZ_GUARD_BEGIN
  if (!out) return hz_fail(HZ_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!mesh || !beta) return hz_fail(HZ_ERR_INVALID, "mesh or beta is NULL");
  if (!(mesh->c > 0.0) || !std::isfinite(mesh->c)) return hz_fail(HZ_ERR_INVALID, "speed of sound must be > 0");
  if (mesh->order != HZ_ORDER_GIVEN && mesh->order != HZ_ORDER_RCM)
    return hz_fail(HZ_ERR_INVALID, "unknown node order %d", mesh->order);
  if (mesh->sigma < 0 || mesh->sigma % kWave != 0 || mesh->sigma > (1 << 20))
    return hz_fail(HZ_ERR_INVALID, "sigma %d is not a multiple of 64 in 0..2^20", mesh->sigma);
  if ((mesh->order != HZ_ORDER_GIVEN || mesh->sigma > 0) &&
      (mesh->parts[0] > 0 || mesh->parts[1] > 0 || mesh->parts[2] > 0))
    return hz_fail(HZ_ERR_INVALID, "the Schwarz partition needs the mesh's own numbering (order 0, sigma 0)");
  for (int w = 0; w < 6; ++w)
    if (!std::isfinite(beta[w].re) || !std::isfinite(beta[w].im)) return hz_fail(HZ_ERR_INVALID, "beta not finite");
  std::unique_ptr<hz_ctx_s> ctx(new hz_ctx_s());
  // host-side validation and assembly first: bad input never touches the GPU
  HZ_TRY(host_assemble(mesh, eta, &ctx->h, 6, &ctx->perm));
  HZ_HIP(hipGetDevice(&ctx->device));
  HZ_TRY(noalloc_setup(ctx->device));   // static scratch of hz_dotc_noalloc on this device
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  ctx->c = mesh->c;
  ctx->rho = mesh->rho;
  for (int d = 0; d < 3; ++d) {
    ctx->elems[d] = mesh->elems[d];
    ctx->parts[d] = mesh->parts[d];
  }
  ctx->beta.resize(6);
  for (int w = 0; w < 6; ++w) ctx->beta[w] = std::complex<double>(beta[w].re, beta[w].im);
  ctx->have_eta = eta != nullptr;
  if (eta) ctx->eta_field.assign(eta, eta + ctx->h.ne);
  HZ_TRY(ctx_upload(ctx.get()));
  HZ_HIP(hipStreamSynchronize(ctx->stream));
  *out = ctx.release();
  return HZ_OK;
  HZ_GUARD_END
}

int hz_set_params(hz_ctx ctx, const hz_c128* beta, const double* eta) {
  HZ_GUARD_BEGIN
  HZ_TRY(check_ctx(ctx));
  if (beta) {
    for (int w = 0; w < 6; ++w)
      if (!std::isfinite(beta[w].re) || !std::isfinite(beta[w].im)) return hz_fail(HZ_ERR_INVALID, "beta not finite");
    for (int w = 0; w < 6; ++w) ctx->beta[w] = std::complex<double>(beta[w].re, beta[w].im);
  }
  if (eta) {
    HZ_TRY(host_assemble_meta(&ctx->h, eta));
    ctx->have_eta = true;
    ctx->eta_field.assign(eta, eta + ctx->h.ne);
  }
  HZ_HIP(hipStreamSynchronize(ctx->stream));
  HZ_TRY(ctx_upload_params(ctx));
  ctx->params_version += 1;
  ctx->have_freq = false;
  ctx->scaled = -1;
  ctx->have_A32 = false;
  ctx->have_split = ctx->have_split32 = false;
  ctx->have_stencil = ctx->have_stencil32 = false;
  return HZ_OK;
  HZ_GUARD_END
}

int hz_set_frequency(hz_ctx ctx, double freq_hz) {
  HZ_GUARD_BEGIN
  HZ_TRY(check_ctx(ctx));
  if (!std::isfinite(freq_hz) || freq_hz < 0.0) return hz_fail(HZ_ERR_INVALID, "frequency must be finite and >= 0");
  ctx->freq = freq_hz;
  ctx->k = 2.0 * M_PI * freq_hz / ctx->c;
  HZ_TRY(op_set_frequency(ctx, op_parts(ctx), ctx->k, 1, false));
  ctx->scaled = HZ_JACOBI;
  ctx->have_A32 = false;
  ctx->have_freq = true;
  return HZ_OK;
  HZ_GUARD_END
}

int hz_apply(hz_ctx ctx, const hz_c128* x_dev, hz_c128* y_dev) {
  HZ_GUARD_BEGIN
  HZ_TRY(check_ctx(ctx));
  if (!x_dev || !y_dev) return hz_fail(HZ_ERR_INVALID, "null vector");
  if (!ctx->have_freq) return hz_fail(HZ_ERR_STATE, "no frequency set");
  int rc = 0;
  const int64_t n = ctx->h.n, nr = ctx->sell.n_rows;
  DevBuf* t = ctx->buf("apply.x", sizeof(z_t) * nr, &rc);
  if (rc) return rc;
  const z_t* x = reinterpret_cast<const z_t*>(x_dev);
  // a column-scaled operator A D^-1 is applied to D x
  HZ_TRY(pad_in(ctx, n, nr, x, ctx->scaled == HZ_JACOBI ? ctx->d_d.as<z_t>() : nullptr, t->as<z_t>()));
  if (ctx->perm.empty()) {
    HZ_TRY(op_spmv<double>(ctx->stream, nr, n, op_A(ctx), t->as<z_t>(), reinterpret_cast<z_t*>(y_dev)));
    return HZ_OK;
  }
  DevBuf* yt = ctx->buf("apply.y", sizeof(z_t) * nr, &rc);
  if (rc) return rc;
  HZ_TRY(op_spmv<double>(ctx->stream, nr, n, op_A(ctx), t->as<z_t>(), yt->as<z_t>()));
  HZ_TRY(unpad_out(ctx, n, yt->as<z_t>(), nullptr, reinterpret_cast<z_t*>(y_dev)));
  return HZ_OK;
  HZ_GUARD_END
}

int hz_get_diag(hz_ctx ctx, hz_c128* d_dev) {
  HZ_GUARD_BEGIN
  HZ_TRY(check_ctx(ctx));
  if (!d_dev) return hz_fail(HZ_ERR_INVALID, "null vector");
  if (!ctx->have_freq) return hz_fail(HZ_ERR_STATE, "no frequency set");
  return unpad_out(ctx, ctx->h.n, ctx->d_d.as<z_t>(), nullptr, reinterpret_cast<z_t*>(d_dev));
  HZ_GUARD_END
}

int hz_load(hz_ctx ctx, const hz_c128* g_dev, hz_c128* f_dev) {
  HZ_GUARD_BEGIN
  HZ_TRY(check_ctx(ctx));
  if (!g_dev || !f_dev) return hz_fail(HZ_ERR_INVALID, "null vector");
  if (ctx->dirichlet) {
    // the lifting -A_FD g_D depends on the frequency
    if (!ctx->have_freq) return hz_fail(HZ_ERR_STATE, "a Dirichlet load needs a frequency (call hz_set_frequency)");
    int rc = 0;
    const int64_t n = ctx->h.n, nr = ctx->sell.n_rows;
    DevBuf* gi = ctx->buf("lift.g", sizeof(z_t) * nr, &rc);
    if (rc) return rc;
    DevBuf* fi = ctx->buf("lift.f", sizeof(z_t) * nr, &rc);
    if (rc) return rc;
    HZ_TRY(pad_in(ctx, n, nr, reinterpret_cast<const z_t*>(g_dev), nullptr, gi->as<z_t>()));
    HZ_TRY(op_lift(ctx, gi->as<z_t>(), fi->as<z_t>()));
    return unpad_out(ctx, n, fi->as<z_t>(), nullptr, reinterpret_cast<z_t*>(f_dev));
  }
  return op_load(ctx, reinterpret_cast<const z_t*>(g_dev), reinterpret_cast<z_t*>(f_dev));
  HZ_GUARD_END
}

int hz_dotc(hz_ctx ctx, int64_t n, const hz_c128* a_dev, const hz_c128* b_dev, hz_c128* out) {
  HZ_GUARD_BEGIN
  HZ_TRY(check_ctx(ctx));
  if (!a_dev || !b_dev || !out || n < 0) return hz_fail(HZ_ERR_INVALID, "bad arguments");
  int rc = 0;
  DevBuf* r = ctx->buf("dot.out", sizeof(double) * 2, &rc);
  if (rc) return rc;
  HZ_TRY(op_dotc(ctx, n, reinterpret_cast<const z_t*>(a_dev), reinterpret_cast<const z_t*>(b_dev), r->as<double>()));
  void* hp = nullptr;
  HZ_TRY(ctx_pinned(ctx, 16, &hp));
  HZ_HIP(hipMemcpyAsync(hp, r->p, 16, hipMemcpyDeviceToHost, ctx->stream));
  HZ_HIP(hipStreamSynchronize(ctx->stream));
  out->re = static_cast<double*>(hp)[0];
  out->im = static_cast<double*>(hp)[1];
  return HZ_OK;
  HZ_GUARD_END
}

int hz_solve(hz_ctx ctx, const hz_solve_opts* opts, const hz_c128* f_dev, hz_c128* p_dev, hz_solve_info* info) {
  HZ_GUARD_BEGIN
  HZ_TRY(check_ctx(ctx));
  HZ_TRY(validate_opts(opts));
  if (!f_dev || !p_dev) return hz_fail(HZ_ERR_INVALID, "null vector");
  if (!ctx->have_freq) return hz_fail(HZ_ERR_STATE, "no frequency set (call hz_set_frequency first)");
  const z_t* f = reinterpret_cast<const z_t*>(f_dev);
  z_t* p = reinterpret_cast<z_t*>(p_dev);
  if (opts->method == HZ_SCHWARZ) {
    if (ctx->dirichlet || ctx->h.gls_h > 0.0)
      return hz_fail(HZ_ERR_INVALID, "the Schwarz method takes a Neumann source and the Galerkin scheme");
    return schwarz_solve(ctx, *opts, f, p, info);
  }
  return solve_single(ctx, *opts, f, p, info);
  HZ_GUARD_END
}

int hz_solve_sweep(hz_ctx ctx, int32_t nfreq, const double* freqs_host, const hz_c128* F_dev, hz_c128* P_dev,
                   const hz_solve_opts* opts, hz_solve_info* infos) {
  HZ_GUARD_BEGIN
  HZ_TRY(check_ctx(ctx));
  HZ_TRY(validate_opts(opts));
  if (nfreq < 1 || nfreq > 64) return hz_fail(HZ_ERR_INVALID, "nfreq %d not in 1..64", nfreq);
  if (!freqs_host || !F_dev || !P_dev) return hz_fail(HZ_ERR_INVALID, "null argument");
  if (opts->method == HZ_SCHWARZ) return hz_fail(HZ_ERR_INVALID, "the sweep runs GMRES, BiCGStab, BiCGStab(l) or TFQMR");
  if (ctx->dirichlet) return hz_fail(HZ_ERR_INVALID, "the sweep takes a Neumann source");
  if (ctx->h.gls_h > 0.0 && ctx->have_eta)
    return hz_fail(HZ_ERR_INVALID, "the sweep takes the GLS scheme only without an absorption field");
  for (int j = 0; j < nfreq; ++j)
    if (!std::isfinite(freqs_host[j]) || freqs_host[j] < 0) return hz_fail(HZ_ERR_INVALID, "bad frequency");
  return sweep_solve(ctx, nfreq, freqs_host, reinterpret_cast<const z_t*>(F_dev), reinterpret_cast<z_t*>(P_dev),
                     *opts, infos);
  HZ_GUARD_END
}

int hz_solve_adjoint(hz_ctx ctx, const hz_solve_opts* opts, const hz_c128* p_dev, const hz_c128* g_dev,
                     hz_c128* lambda_dev, double* dJ_dbeta, double* dJ_deta_dev, hz_solve_info* info) {
  HZ_GUARD_BEGIN
  HZ_TRY(check_ctx(ctx));
  HZ_TRY(validate_opts(opts));
  if (!p_dev || !g_dev || !lambda_dev) return hz_fail(HZ_ERR_INVALID, "null vector");
  if (!ctx->have_freq) return hz_fail(HZ_ERR_STATE, "no frequency set (call hz_set_frequency first)");
  return adjoint_solve(ctx, *opts, reinterpret_cast<const z_t*>(p_dev), reinterpret_cast<const z_t*>(g_dev),
                       reinterpret_cast<z_t*>(lambda_dev), dJ_dbeta, dJ_deta_dev, info);
  HZ_GUARD_END
}

int hz_receiver_energy(hz_ctx ctx, int32_t n_rec, const int32_t* receivers, const hz_c128* p_dev, double* J,
                       hz_c128* g_dev) {
  HZ_GUARD_BEGIN
  HZ_TRY(check_ctx(ctx));
  if (n_rec < 0 || (n_rec > 0 && !receivers) || !p_dev || !g_dev || !J)
    return hz_fail(HZ_ERR_INVALID, "bad arguments");
  return receiver_objective(ctx, n_rec, receivers, reinterpret_cast<const z_t*>(p_dev), J,
                            reinterpret_cast<z_t*>(g_dev));
  HZ_GUARD_END
}

namespace {
enum { kKindComplex = 0, kKindSplit = 1, kKindStencil = 2 };
// The product of the given form: the solvers' choice, or a forced form.
int spmv_form(hz_ctx ctx, int32_t precision, int32_t format, int* kind) {
  if (precision != HZ_FP64 && precision != HZ_MIXED) return hz_fail(HZ_ERR_INVALID, "bad precision");
  if (format != HZ_SPMV_SOLVER && format != HZ_SPMV_COMPLEX && format != HZ_SPMV_SPLIT &&
      format != HZ_SPMV_STENCIL)
    return hz_fail(HZ_ERR_INVALID, "bad format");
  const bool mixed = precision == HZ_MIXED;
  HZ_TRY(ensure_operator(ctx, ctx->scaled < 0 ? HZ_JACOBI : ctx->scaled, mixed));
  const bool split = mixed ? ctx->have_split32 : ctx->have_split;
  const bool stencil = mixed ? ctx->have_stencil32 : ctx->have_stencil;
  if (format == HZ_SPMV_SPLIT && !split)
    return hz_fail(HZ_ERR_STATE, "split form not formed (absorption field present or HZ_SPLIT=0)");
  if (format == HZ_SPMV_STENCIL && !stencil)
    return hz_fail(HZ_ERR_STATE, "stencil form not formed (not a box in its own numbering, or HZ_STENCIL=0)");
  if (format == HZ_SPMV_COMPLEX) *kind = kKindComplex;
  else if (format == HZ_SPMV_SPLIT) *kind = kKindSplit;
  else if (format == HZ_SPMV_STENCIL || stencil) *kind = kKindStencil;
  else *kind = split ? kKindSplit : kKindComplex;
  return HZ_OK;
}
}  // namespace

int hz_time_spmv(hz_ctx ctx, int32_t reps, int32_t precision, int32_t format, double* avg_ms) {
  HZ_GUARD_BEGIN
  HZ_TRY(check_ctx(ctx));
  if (!avg_ms || reps < 1 || reps > 100000) return hz_fail(HZ_ERR_INVALID, "bad arguments");
  int kind = 0;
  HZ_TRY(spmv_form(ctx, precision, format, &kind));
  const bool mixed = precision == HZ_MIXED;
  int rc = 0;
  const int64_t nr = ctx->sell.n_rows;
  const size_t es = mixed ? sizeof(c_t) : sizeof(z_t);
  DevBuf* xb = ctx->buf("time.x", es * nr, &rc);
  if (rc) return rc;
  DevBuf* yb = ctx->buf("time.y", es * nr, &rc);
  if (rc) return rc;
  HZ_HIP(hipMemsetAsync(xb->p, 0, es * nr, ctx->stream));
  const SellOp<double> A64 = kind == kKindStencil ? op_stencil<double>(ctx)
                             : kind == kKindSplit  ? op_split<double>(ctx) : op_A_complex(ctx);
  const SellOp<float> A32 = kind == kKindStencil ? op_stencil<float>(ctx)
                            : kind == kKindSplit  ? op_split<float>(ctx) : op_A32_complex(ctx);
  auto one = [&]() -> int {
    if (mixed) return op_spmv<float>(ctx->stream, nr, nr, A32, xb->as<c_t>(), yb->as<c_t>());
    return op_spmv<double>(ctx->stream, nr, nr, A64, xb->as<z_t>(), yb->as<z_t>());
  };
  hipEvent_t e0, e1;
  HZ_HIP(hipEventCreate(&e0));
  HZ_HIP(hipEventCreate(&e1));
  HZ_TRY(one());   // one untimed product first
  HZ_HIP(hipEventRecord(e0, ctx->stream));
  for (int r = 0; r < reps; ++r) HZ_TRY(one());
  HZ_HIP(hipEventRecord(e1, ctx->stream));
  HZ_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  HZ_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = double(ms) / reps;
  return HZ_OK;
  HZ_GUARD_END
}

int hz_time_spmm(hz_ctx ctx, int32_t nfreq, const double* freqs_host, int32_t precision, int32_t reps,
                 double* avg_ms, int64_t* bytes, int32_t* variant) {
  HZ_GUARD_BEGIN
  HZ_TRY(check_ctx(ctx));
  if (!avg_ms || !freqs_host || nfreq < 1 || nfreq > 64 || reps < 1 || reps > 100000)
    return hz_fail(HZ_ERR_INVALID, "bad arguments");
  if (precision != HZ_FP64 && precision != HZ_MIXED) return hz_fail(HZ_ERR_INVALID, "bad precision");
  if (ctx->dirichlet) return hz_fail(HZ_ERR_INVALID, "the sweep takes a Neumann source");
  for (int j = 0; j < nfreq; ++j)
    if (!std::isfinite(freqs_host[j]) || freqs_host[j] < 0) return hz_fail(HZ_ERR_INVALID, "bad frequency");
  ctx->have_freq = false;   // as after a sweep
  HZ_TRY(sweep_time_spmm(ctx, nfreq, freqs_host, precision, reps, avg_ms, variant, bytes));
  return HZ_OK;
  HZ_GUARD_END
}

int hz_apply_sweep(hz_ctx ctx, int32_t nfreq, const double* freqs_host, int32_t precision, const hz_c128* x_dev,
                   hz_c128* y_dev, int32_t* variant) {
  HZ_GUARD_BEGIN
  HZ_TRY(check_ctx(ctx));
  if (!freqs_host || !x_dev || !y_dev || nfreq < 1 || nfreq > 64) return hz_fail(HZ_ERR_INVALID, "bad arguments");
  if (precision != HZ_FP64 && precision != HZ_MIXED) return hz_fail(HZ_ERR_INVALID, "bad precision");
  if (ctx->dirichlet) return hz_fail(HZ_ERR_INVALID, "the sweep takes a Neumann source");
  if (ctx->h.gls_h > 0.0 && ctx->have_eta)
    return hz_fail(HZ_ERR_INVALID, "the sweep takes the GLS scheme only without an absorption field");
  for (int j = 0; j < nfreq; ++j)
    if (!std::isfinite(freqs_host[j]) || freqs_host[j] < 0) return hz_fail(HZ_ERR_INVALID, "bad frequency");
  ctx->have_freq = false;   // as after a sweep
  return sweep_apply(ctx, nfreq, freqs_host, precision, reinterpret_cast<const z_t*>(x_dev),
                     reinterpret_cast<z_t*>(y_dev), variant);
  HZ_GUARD_END
}

int hz_dd_alpha(double k, double H, double h, int32_t sides, hz_c128* alpha) {
  HZ_GUARD_BEGIN
  if (!alpha) return hz_fail(HZ_ERR_INVALID, "alpha is NULL");
  if (!(k > 0.0) || !(h > 0.0) || !(H > h) || !std::isfinite(k) || !std::isfinite(H))
    return hz_fail(HZ_ERR_INVALID, "need k > 0 and H > h > 0");
  if (sides != 1 && sides != 2) return hz_fail(HZ_ERR_INVALID, "sides must be 1 or 2");
  std::complex<double> a[2];
  dd_optimised_alpha(k, H, h, sides, a);
  for (int i = 0; i < 2; ++i) alpha[i] = hz_c128{a[i].real(), a[i].imag()};
  return HZ_OK;
  HZ_GUARD_END
}

int hz_spmv_bytes(hz_ctx ctx, int32_t precision, int32_t format, int64_t* bytes) {
  HZ_GUARD_BEGIN
  HZ_TRY(check_ctx(ctx));
  if (!bytes) return hz_fail(HZ_ERR_INVALID, "bytes is NULL");
  int kind = 0;
  HZ_TRY(spmv_form(ctx, precision, format, &kind));
  const int64_t n = ctx->h.n, nnz = int64_t(ctx->h.col.size());
  const int64_t real = precision == HZ_MIXED ? 4 : 8;   // bytes of one real part
  if (kind == kKindComplex) {
    *bytes = (2 * real + 4) * nnz + 4 * (n + 1) + 4 * real * n;
  } else if (kind == kKindStencil) {
    *bytes = real * nnz + (real + 4) * ctx->n_imag + 4 * (n + 1) + 4 * real * n;
  } else {
    const int64_t idx = ctx->split_dcol ? 2 : 4;
    *bytes = (real + idx) * nnz + (real + 4) * ctx->n_imag + 4 * (n + 1) + 4 * real * n;
  }
  return HZ_OK;
  HZ_GUARD_END
}

int hz_node_order(const hz_mesh* mesh, int32_t* perm) {
  HZ_GUARD_BEGIN
  if (!mesh || !perm || !mesh->hex || mesh->n_nodes <= 0 || mesh->n_elems <= 0)
    return hz_fail(HZ_ERR_INVALID, "null or empty mesh");
  if (mesh->order != HZ_ORDER_GIVEN && mesh->order != HZ_ORDER_RCM)
    return hz_fail(HZ_ERR_INVALID, "unknown node order %d", mesh->order);
  if (mesh->sigma < 0 || mesh->sigma % kWave != 0 || mesh->sigma > (1 << 20))
    return hz_fail(HZ_ERR_INVALID, "sigma %d is not a multiple of 64 in 0..2^20", mesh->sigma);
  if (mesh->elem_type != HZ_HEX8 && mesh->elem_type != HZ_TET4)
    return hz_fail(HZ_ERR_INVALID, "unknown element type %d", mesh->elem_type);
  const int npe = mesh->elem_type == HZ_TET4 ? 4 : 8;
  const int64_t n = mesh->n_nodes, ne = mesh->n_elems;
  for (int64_t q = 0; q < ne * npe; ++q)
    if (mesh->hex[q] < 0 || mesh->hex[q] >= n)
      return hz_fail(HZ_ERR_INVALID, "element node %d out of range", mesh->hex[q]);
  std::vector<int64_t> n2e_ptr, rowptr;
  std::vector<int32_t> n2e, col, P;
  HZ_TRY(mesh_pattern(n, ne, npe, mesh->hex, &n2e_ptr, &n2e, &rowptr, &col));
  node_order(n, rowptr, col, mesh->order, mesh->sigma, &P);
  std::copy(P.begin(), P.end(), perm);
  return HZ_OK;
  HZ_GUARD_END
}

int hz_layout(hz_ctx ctx, int32_t* perm, int64_t* slots, int64_t* bandwidth, int64_t* n_imag) {
  HZ_GUARD_BEGIN
  if (!ctx) return hz_fail(HZ_ERR_INVALID, "ctx is NULL");
  const HostAsm& a = ctx->h;
  if (perm)
    for (int64_t p = 0; p < a.n; ++p) perm[p] = ctx->perm.empty() ? int32_t(p) : ctx->perm[p];
  if (slots) *slots = ctx->sell.n_pad;
  if (bandwidth) {
    int64_t bw = 0;
    for (int64_t i = 0; i < a.n; ++i)
      for (int64_t q = a.rowptr[i]; q < a.rowptr[i + 1]; ++q) bw = std::max<int64_t>(bw, std::abs(a.col[q] - i));
    *bandwidth = bw;
  }
  if (n_imag) *n_imag = ctx->n_imag;
  return HZ_OK;
  HZ_GUARD_END
}

int hz_sizes(hz_ctx ctx, int64_t* n_nodes, int64_t* n_elems, int64_t* nnz, int64_t* device_bytes) {
  if (!ctx) return hz_fail(HZ_ERR_INVALID, "ctx is NULL");
  if (n_nodes) *n_nodes = ctx->h.n;
  if (n_elems) *n_elems = ctx->h.ne;
  if (nnz) *nnz = int64_t(ctx->h.col.size());
  if (device_bytes) *device_bytes = ctx->dev_bytes;
  return HZ_OK;
}

void hz_destroy(hz_ctx ctx) {
  if (!ctx) return;
  int dev = -1;
  if (hipGetDevice(&dev) == hipSuccess && dev != ctx->device) (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
}

}  // extern "C"
