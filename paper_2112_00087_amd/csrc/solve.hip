// Single-frequency solve driver: FP64 Krylov, or mixed precision (complex64
// inner Krylov on a complex64 copy of the operator, FP64 residual and
// iterative refinement).
#include <chrono>

#include "ops.h"
#include "solve.h"

namespace {

// y[i] = s[i] x[perm[i]] for internal rows i < n (perm NULL: identity), 0 on padding
__global__ void k_pad_in(int64_t n, int64_t nrows, const z_t* __restrict__ x, const z_t* __restrict__ s,
                         const int* __restrict__ perm, z_t* __restrict__ y) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= nrows) return;
  z_t v = {0.0, 0.0};
  if (i < n) {
    const z_t xv = x[perm ? int64_t(perm[i]) : i];
    v = s ? s[i] * xv : xv;
  }
  y[i] = v;
}

// p[perm[i]] = s[i] u[i] for internal rows i < n
__global__ void k_unpad_out(int64_t n, const z_t* __restrict__ u, const z_t* __restrict__ s,
                            const int* __restrict__ perm, z_t* __restrict__ p) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  p[perm ? int64_t(perm[i]) : i] = s ? s[i] * u[i] : u[i];
}

// out = r / ||r_seg|| in complex64
__global__ void __launch_bounds__(kBlock) k_to32(Seg L, const z_t* __restrict__ r, const double* __restrict__ inv,
                                                 c_t* __restrict__ out, c_t* __restrict__ zero) {
  Tile t = tile_of(L);
  out[t.row] = ccast<float>(inv[t.seg] * r[t.row]);
  zero[t.row] = c_t{0.0f, 0.0f};
}

// u += ||r_seg|| d (FP64)
__global__ void __launch_bounds__(kBlock) k_ir_add(Seg L, const c_t* __restrict__ d, const double* __restrict__ nrm,
                                                   z_t* __restrict__ u) {
  Tile t = tile_of(L);
  z_t dv = ccast<double>(d[t.row]);
  z_t uv = u[t.row];
  double s = nrm[t.seg];
  u[t.row] = z_t{fma(s, dv.re, uv.re), fma(s, dv.im, uv.im)};
}

}  // namespace

int pad_in(hz_ctx ctx, int64_t n, int64_t nrows, const z_t* x, const z_t* scale, z_t* y) {
  k_pad_in<<<ceil_div(nrows, kBlock), kBlock, 0, ctx->stream>>>(n, nrows, x, scale, ctx_perm(ctx), y);
  HZ_HIP(hipGetLastError());
  return HZ_OK;
}

int unpad_out(hz_ctx ctx, int64_t n, const z_t* u, const z_t* scale, z_t* p) {
  if (n <= 0) return HZ_OK;
  k_unpad_out<<<ceil_div(n, kBlock), kBlock, 0, ctx->stream>>>(n, u, scale, ctx_perm(ctx), p);
  HZ_HIP(hipGetLastError());
  return HZ_OK;
}

int ensure_operator(hz_ctx ctx, int precond, bool want32) {
  if (!ctx->have_freq) return hz_fail(HZ_ERR_STATE, "no frequency set (call hz_set_frequency first)");
  if (want32 && !ctx->d_A32.p) {
    size_t before = ctx->d_A32.bytes;
    HZ_TRY(ctx->d_A32.ensure(sizeof(c_t) * ctx->sell.n_pad));
    ctx->dev_bytes += int64_t(ctx->d_A32.bytes) - int64_t(before);
  }
  if (ctx->scaled != precond || (want32 && !ctx->have_A32)) {
    HZ_TRY(op_set_frequency(ctx, op_parts(ctx), ctx->k, precond == HZ_JACOBI ? 1 : 0, want32));
    ctx->scaled = precond;
    ctx->have_A32 = want32;
  }
  return HZ_OK;
}

// Mixed-precision iterative refinement on a segmented system.  u (FP64) is
// the solution of the (scaled) operator; every outer step forms the FP64
// residual, solves the correction equation in complex64 to inner_tol and adds
// the correction in FP64.
int ir_run(hz_ctx ctx, const SegHost& S, const SellOp<double>& A64, const SellOp<float>& A32,
           const z_t* f, z_t* u, const hz_solve_opts& o, IrOut* out, const std::string& tag) {
  int rc = 0;
  const int64_t nr = S.nrows;
  DevBuf* rb = ctx->buf("ir." + tag + ".r", sizeof(z_t) * nr, &rc);
  if (rc) return rc;
  DevBuf* r32 = ctx->buf("ir." + tag + ".r32", sizeof(c_t) * nr, &rc);
  if (rc) return rc;
  DevBuf* d32 = ctx->buf("ir." + tag + ".d32", sizeof(c_t) * nr, &rc);
  if (rc) return rc;
  DevBuf* sc = ctx->buf("ir." + tag + ".sc", sizeof(double) * 2 * S.nseg, &rc);
  if (rc) return rc;
  std::vector<double> fn2, rr;
  HZ_TRY(seg_norm2_t<double>(ctx, S, f, &fn2));
  out->fnorm.resize(S.nseg);
  for (int i = 0; i < S.nseg; ++i) out->fnorm[i] = std::sqrt(fn2[i]);
  out->outer = 0;
  out->matvecs = 0;
  out->inner_matvecs = 0;
  out->relres.assign(S.nseg, 0.0);
  out->inner_status = HZ_OK;
  KrylovCtl ic;
  ic.tol = o.inner_tol > 0 ? o.inner_tol : 1e-4;
  ic.restart = o.inner_restart > 0 ? o.inner_restart : 30;
  ic.ell = o.restart;                  // BiCGStab(l): l (validated 1..8)
  ic.stall_halfsteps = 4096;           // complex64 TFQMR: end a stalled inner solve
  const int max_outer = 200;
  for (;;) {
    HZ_TRY(true_residual(ctx, S, A64, f, u, rb->as<z_t>(), &rr));
    out->matvecs += 1;
    bool all = true;
    std::vector<double> h(2 * S.nseg);
    for (int i = 0; i < S.nseg; ++i) {
      double rn = std::sqrt(rr[i]);
      double fnv = out->fnorm[i];
      out->relres[i] = fnv > 0 ? rn / fnv : 0.0;
      bool ok = fnv == 0.0 || out->relres[i] <= o.tol;
      all = all && ok;
      // converged segments get a zero correction right-hand side
      h[i] = (ok || rn == 0.0) ? 0.0 : 1.0 / rn;
      h[S.nseg + i] = ok ? 0.0 : rn;
      if (!std::isfinite(rn)) return hz_fail(HZ_ERR_INVALID, "non-finite residual in refinement");
    }
    if (all) return HZ_OK;
    if (out->outer >= max_outer || out->matvecs + out->inner_matvecs >= o.max_matvec) {
      out->inner_status = HZ_NOT_CONVERGED;
      return HZ_OK;
    }
    HZ_HIP(hipMemcpyAsync(sc->p, h.data(), sizeof(double) * 2 * S.nseg, hipMemcpyHostToDevice, ctx->stream));
    k_to32<<<S.nblk, kBlock, 0, ctx->stream>>>(S.dev, rb->as<z_t>(), sc->as<double>(), r32->as<c_t>(),
                                              d32->as<c_t>());
    HZ_HIP(hipGetLastError());
    ic.max_matvec = std::max<int64_t>(1, o.max_matvec - out->matvecs - out->inner_matvecs);
    KrylovOut ko;
    HZ_TRY(krylov_run<float>(ctx, o.method, S, A32, r32->as<c_t>(), d32->as<c_t>(), ic, &ko, tag + ".in"));
    int mx = 0;
    for (int i = 0; i < S.nseg; ++i) mx = std::max(mx, ko.matvecs[i]);
    out->inner_matvecs += mx;
    k_ir_add<<<S.nblk, kBlock, 0, ctx->stream>>>(S.dev, d32->as<c_t>(), sc->as<double>() + S.nseg, u);
    HZ_HIP(hipGetLastError());
    out->outer += 1;
  }
}

int solve_single(hz_ctx ctx, const hz_solve_opts& o, const z_t* f, z_t* p, hz_solve_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  const bool mixed = o.precision == HZ_MIXED;
  HZ_TRY(ensure_operator(ctx, o.precond, mixed));
  SegHost* S = nullptr;
  HZ_TRY(ctx_single_seg(ctx, &S));
  int rc = 0;
  const int64_t n = ctx->h.n, nr = S->nrows;
  DevBuf* fb = ctx->buf("solve.f", sizeof(z_t) * nr, &rc);
  if (rc) return rc;
  DevBuf* ub = ctx->buf("solve.u", sizeof(z_t) * nr, &rc);
  if (rc) return rc;
  z_t* fz = fb->as<z_t>();
  z_t* uz = ub->as<z_t>();
  const bool jac = o.precond == HZ_JACOBI;
  HZ_TRY(pad_in(ctx, n, nr, f, nullptr, fz));
  HZ_TRY(pad_in(ctx, n, nr, p, jac ? ctx->d_d.as<z_t>() : nullptr, uz));
  std::vector<double> fn2;
  HZ_TRY(seg_norm2_t<double>(ctx, *S, fz, &fn2));
  if (!std::isfinite(fn2[0])) return hz_fail(HZ_ERR_INVALID, "right-hand side has NaN/Inf entries");
  const SellOp<double> A = op_A(ctx);
  hz_solve_info inf = {};
  int status = HZ_OK;
  if (fn2[0] == 0.0) {
    HZ_TRY(op_fill(ctx->stream, n, p, z_t{0.0, 0.0}));
    HZ_HIP(hipStreamSynchronize(ctx->stream));
    inf.status = HZ_OK;
    if (info) *info = inf;
    return HZ_OK;
  }
  if (!mixed) {
    KrylovCtl c;
    c.tol = o.tol;
    c.max_matvec = o.max_matvec;
    c.restart = o.restart;
    c.ell = o.restart;
    KrylovOut ko;
    HZ_TRY(krylov_run<double>(ctx, o.method, *S, A, fz, uz, c, &ko, "main"));
    inf.iters = ko.iters[0];
    inf.matvecs = ko.matvecs[0];
    inf.relres_est = ko.relres_est[0];
    status = ko.status[0];
  } else {
    IrOut io;
    HZ_TRY(ir_run(ctx, *S, A, op_A32(ctx), fz, uz, o, &io, "main"));
    inf.iters = io.outer;
    inf.matvecs = int(io.matvecs);
    inf.inner_matvecs = int(io.inner_matvecs);
    inf.relres_est = io.relres[0];
    status = io.inner_status;
  }
  std::vector<double> rr;
  HZ_TRY(true_residual(ctx, *S, A, fz, uz, nullptr, &rr));
  inf.relres_true = std::sqrt(rr[0] / fn2[0]);
  HZ_TRY(unpad_out(ctx, n, uz, jac ? ctx->d_dinv.as<z_t>() : nullptr, p));
  HZ_HIP(hipStreamSynchronize(ctx->stream));
  if (status == HZ_OK && !(inf.relres_true <= o.tol)) status = HZ_NOT_CONVERGED;
  if (!std::isfinite(inf.relres_true)) status = HZ_BREAKDOWN;
  inf.status = status;
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return status;
}
