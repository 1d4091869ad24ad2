// Stabilised bi-conjugate gradient method (the paper's P-BiCGSTAB, Sec. 4)
// on the right-Jacobi operator, for every segment of a segmented system.
//
// One iteration of van der Vorst's method is five vector kernels (two of
// them sparse products with fused inner-product epilogues) and three
// one-block-per-segment finalize kernels that turn block partials into the
// Krylov scalars (the early-exit test on ||s|| rides on the omega step).
// The scalars never leave the device; the host only reads the per-segment
// state every few iterations to decide whether to stop.
// Every kernel first reads its segment's flags and returns if that segment
// has converged, so extra queued iterations cost only empty launches.
#include <chrono>

#include "ops.h"

namespace {

struct BiSt {
  z_t rho, rho_old, alpha, omega;
  z_t beta;                       // (rho / rho_old) (alpha / omega) for the next p update
  double rr, ss, thr2, rhat2;
  int iter, done, early, reset;
  int nan, pad0;
};

template <typename T>
struct BiV {
  const cx<T>* f;
  cx<T>* u;
  cx<T>* r;
  cx<T>* rhat;
  cx<T>* p;
  cx<T>* v;
  cx<T>* s;
  cx<T>* t;
};

template <typename T> __device__ __forceinline__ z_t zd(cx<T> a) { return ccast<double>(a); }
template <typename T> __device__ __forceinline__ cx<T> zt(z_t a) { return ccast<T>(a); }

// r = f - A u; restart: rhat = r, p = v = 0.  Partial ||r||^2.
template <typename T, int F>
__global__ void __launch_bounds__(kBlock) k_resid(Seg L, SellOp<T> A, BiV<T> V, double* part) {
  SumTile t = tile_of_sums(L);
  z_t y = zd(sell_row_form<F>(A, t.row, V.u));
  z_t r = zd(V.f[t.row]) - y;
  cx<T> rs = zt<T>(r);
  V.r[t.row] = rs;
  V.rhat[t.row] = rs;
  V.p[t.row] = cx<T>{T(0), T(0)};
  V.v[t.row] = cx<T>{T(0), T(0)};
  z_t rr = zd(rs);
  double q[1] = {norm2(rr)};
  store_partials<1>(q, part, t);
}

__global__ void k_resid_fin(Seg L, BiSt* st, const double* part) {
  int s = blockIdx.x;
  double o[1];
  seg_sums<1>(L, part, s, o);
  if (threadIdx.x == 0) {
    const double rr = o[0];
    BiSt& S = st[s];
    S.rr = rr;
    S.rho = z_t{rr, 0.0};
    S.rho_old = S.alpha = S.omega = z_t{1.0, 0.0};
    S.beta = z_t{rr, 0.0};
    S.rhat2 = rr;
    S.early = 0;
    S.reset = 0;
    S.nan = !isfinite(rr);
    S.done = (rr <= S.thr2) || S.nan;
  }
}

// p = r + beta (p - omega v), beta = (rho / rho_old) (alpha / omega); on reset rhat = p = r.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_p(Seg L, const BiSt* st, BiV<T> V) {
  Tile t = tile_of(L);
  const BiSt& S = st[t.seg];
  if (S.done) return;
  cx<T> r = V.r[t.row];
  if (S.reset) {
    V.rhat[t.row] = r;
    V.p[t.row] = r;
    return;
  }
  z_t p = zd(V.p[t.row]) - S.omega * zd(V.v[t.row]);
  V.p[t.row] = zt<T>(zd(r) + S.beta * p);
}

// v = A p; partial rhat^H v.  Instantiated per storage form F of A (one
// form per kernel keeps the register count, hence the occupancy, of that form).
template <typename T, int F>
__global__ void HZ_PRODUCT_BOUNDS k_v(Seg L, SellOp<T> A, const BiSt* st, BiV<T> V, double* part) {
  SumTile t = tile_of_sums(L);
  if (st[t.seg].done) return;
  cx<T> y = sell_row_form<F>(A, t.row, V.p);
  V.v[t.row] = y;
  z_t a = zd(V.rhat[t.row]), b = zd(y);
  double q[2] = {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
  store_partials<2>(q, part, t);
}

__global__ void k_alpha_fin(Seg L, BiSt* st, const double* part) {
  int s = blockIdx.x;
  const int done = st[s].done;
  double o[2];
  seg_sums<2>(L, part, s, o);
  if (done) return;
  if (threadIdx.x == 0) {
    const double re = o[0], im = o[1];
    BiSt& S = st[s];
    S.reset = 0;
    z_t rv = {re, im};
    if (norm2(rv) == 0.0 || !isfinite(re) || !isfinite(im)) {
      S.alpha = z_t{0.0, 0.0};   // minimal-residual step this iteration, restart after it
      S.reset = 1;
    } else {
      S.alpha = cdiv(S.rho, rv);
    }
  }
}

// s = r - alpha v.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_s(Seg L, const BiSt* st, BiV<T> V) {
  Tile t = tile_of(L);
  const BiSt& S = st[t.seg];
  if (S.done) return;
  z_t s = zd(V.r[t.row]) - S.alpha * zd(V.v[t.row]);
  V.s[t.row] = zt<T>(s);
}

// t = A s; partials t^H s, t^H t, s^H s (per storage form F, as k_v).
template <typename T, int F>
__global__ void HZ_PRODUCT_BOUNDS k_t(Seg L, SellOp<T> A, const BiSt* st, BiV<T> V, double* part) {
  SumTile t = tile_of_sums(L);
  const BiSt& S = st[t.seg];
  if (S.done) return;
  cx<T> y = sell_row_form<F>(A, t.row, V.s);
  V.t[t.row] = y;
  z_t a = zd(y), b = zd(V.s[t.row]);
  double q[4] = {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re, norm2(a), norm2(b)};
  store_partials<4>(q, part, t);
}

// omega = t^H s / t^H t, or the early exit when ||s|| already meets the target
// (then x += alpha p completes the iteration).
__global__ void k_omega_fin(Seg L, BiSt* st, const double* part) {
  int s = blockIdx.x;
  const int done = st[s].done;
  double o[4];
  seg_sums<4>(L, part, s, o);
  if (done) return;
  if (threadIdx.x == 0) {
    const double re = o[0], im = o[1], tt = o[2], ss = o[3];
    BiSt& S = st[s];
    S.ss = ss;
    S.early = (ss <= S.thr2) ? 1 : 0;
    S.omega = (tt > 0.0 && !S.early) ? z_t{re / tt, im / tt} : z_t{0.0, 0.0};
  }
}

// u += alpha p + omega s; r = s - omega t; partials rhat^H r, ||r||^2.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_xr(Seg L, const BiSt* st, BiV<T> V, double* part) {
  SumTile t = tile_of_sums(L);
  const BiSt& S = st[t.seg];
  if (S.done) return;
  z_t u = zd(V.u[t.row]) + S.alpha * zd(V.p[t.row]);
  if (S.early) {
    V.u[t.row] = zt<T>(u);
    return;
  }
  z_t s = zd(V.s[t.row]);
  V.u[t.row] = zt<T>(u + S.omega * s);
  cx<T> r = zt<T>(s - S.omega * zd(V.t[t.row]));
  V.r[t.row] = r;
  z_t a = zd(V.rhat[t.row]), b = zd(r);
  double q[3] = {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re, norm2(b)};
  store_partials<3>(q, part, t);
}

__global__ void k_rho_fin(Seg L, BiSt* st, const double* part) {
  int s = blockIdx.x;
  BiSt& S = st[s];
  const int done = S.done, early = S.early;
  double o[3];
  // (its barriers also see every thread's flags read before thread 0 rewrites them)
  seg_sums<3>(L, part, s, o);
  if (done) return;
  if (early) {
    if (threadIdx.x == 0) {
      S.iter += 1;
      S.rr = S.ss;
      S.done = 1;
      S.early = 0;
    }
    return;
  }
  if (threadIdx.x == 0) {
    const double re = o[0], im = o[1], rr = o[2];
    S.iter += 1;
    S.rho_old = S.rho;
    S.rho = z_t{re, im};
    S.rr = rr;
    if (!isfinite(rr) || !isfinite(re) || !isfinite(im)) {
      S.nan = 1;
      S.done = 1;
    } else if (rr <= S.thr2) {
      S.done = 1;
    } else if (sqrt(norm2(S.rho)) < 1e-300 * sqrt(S.rhat2 * rr) || norm2(S.omega) == 0.0) {
      // breakdown: restart the shadow residual from the current residual
      S.reset = 1;
      S.rho = z_t{rr, 0.0};
      S.rho_old = S.alpha = S.omega = z_t{1.0, 0.0};
      S.rhat2 = rr;
    }
    S.beta = cdiv(S.rho, S.rho_old) * cdiv(S.alpha, S.omega);
  }
}

__global__ void k_set_thr(int nseg, BiSt* st, const double* fn2, double tol, int reset_iter) {
  int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= nseg) return;
  st[s].thr2 = tol * tol * fn2[s];
  if (reset_iter) st[s].iter = 0;
}

}  // namespace

template <typename T>
int bicgstab_run(hz_ctx ctx, const SegHost& S, const SellOp<T>& A, const cx<T>* f, cx<T>* u,
                 const KrylovCtl& ctl, KrylovOut* out, const std::string& tag) {
  int rc = 0;
  const int64_t nr = S.nrows;
  const size_t vb = sizeof(cx<T>) * nr;
  const std::string p = "bicg." + tag + (sizeof(T) == 8 ? ".z." : ".c.");
  BiV<T> V;
  V.f = f;
  V.u = u;
  cx<T>** vecs[6] = {&V.r, &V.rhat, &V.p, &V.v, &V.s, &V.t};
  const char* names[6] = {"r", "rhat", "p", "v", "s", "t"};
  for (int i = 0; i < 6; ++i) {
    DevBuf* b = ctx->buf(p + names[i], vb, &rc);
    if (rc) return rc;
    *vecs[i] = b->as<cx<T>>();
  }
  DevBuf* stb = ctx->buf(p + "st", sizeof(BiSt) * S.nseg, &rc);
  if (rc) return rc;
  DevBuf* part = ctx->buf(p + "part", sizeof(double) * 4 * S.nblk, &rc);
  if (rc) return rc;
  DevBuf* fnb = ctx->buf(p + "fn2", sizeof(double) * S.nseg, &rc);
  if (rc) return rc;
  BiSt* st = stb->as<BiSt>();
  double* pt = part->as<double>();
  hipStream_t s = ctx->stream;
  const Seg& L = S.dev;

  // ||f||^2 per segment -> thresholds
  std::vector<double> fn2;
  HZ_TRY(seg_norm2_t<T>(ctx, S, f, &fn2));
  out->fnorm.resize(S.nseg);
  for (int i = 0; i < S.nseg; ++i) out->fnorm[i] = std::sqrt(fn2[i]);
  HZ_HIP(hipMemcpyAsync(fnb->p, fn2.data(), sizeof(double) * S.nseg, hipMemcpyHostToDevice, s));
  HZ_HIP(hipMemsetAsync(stb->p, 0, sizeof(BiSt) * S.nseg, s));
  k_set_thr<<<ceil_div(S.nseg, kBlock), kBlock, 0, s>>>(S.nseg, st, fnb->as<double>(), ctl.tol, 1);
  HZ_HIP(hipGetLastError());

  void* hp = nullptr;
  HZ_TRY(ctx_pinned(ctx, sizeof(BiSt) * S.nseg, &hp));
  BiSt* hst = static_cast<BiSt*>(hp);
  const int grid = S.nblk;
  std::vector<int> restarts(S.nseg, 0);
  int64_t resid_calls = 0;
  int chunk = 4;

  auto read_state = [&]() -> int {
    HZ_HIP(hipMemcpyAsync(hst, st, sizeof(BiSt) * S.nseg, hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    return HZ_OK;
  };
  auto enqueue_resid = [&]() -> int {
    if (A.val) k_resid<T, kFormComplex><<<grid, kBlock, 0, s>>>(L, A, V, pt);
    else if (A.st) k_resid<T, kFormStencil><<<grid, kBlock, 0, s>>>(L, A, V, pt);
    else k_resid<T, kFormSplit><<<grid, kBlock, 0, s>>>(L, A, V, pt);
    k_resid_fin<<<S.nseg, kFinBlock, 0, s>>>(L, st, pt);
    HZ_HIP(hipGetLastError());
    ++resid_calls;
    return HZ_OK;
  };
  auto enqueue_iter = [&]() -> int {
    k_p<T><<<grid, kBlock, 0, s>>>(L, st, V);
    if (A.val) k_v<T, kFormComplex><<<grid, kBlock, 0, s>>>(L, A, st, V, pt);
    else if (A.st) k_v<T, kFormStencil><<<grid, kBlock, 0, s>>>(L, A, st, V, pt);
    else k_v<T, kFormSplit><<<grid, kBlock, 0, s>>>(L, A, st, V, pt);
    k_alpha_fin<<<S.nseg, kFinBlock, 0, s>>>(L, st, pt);
    k_s<T><<<grid, kBlock, 0, s>>>(L, st, V);
    if (A.val) k_t<T, kFormComplex><<<grid, kBlock, 0, s>>>(L, A, st, V, pt);
    else if (A.st) k_t<T, kFormStencil><<<grid, kBlock, 0, s>>>(L, A, st, V, pt);
    else k_t<T, kFormSplit><<<grid, kBlock, 0, s>>>(L, A, st, V, pt);
    k_omega_fin<<<S.nseg, kFinBlock, 0, s>>>(L, st, pt);
    k_xr<T><<<grid, kBlock, 0, s>>>(L, st, V, pt);
    k_rho_fin<<<S.nseg, kFinBlock, 0, s>>>(L, st, pt);
    HZ_HIP(hipGetLastError());
    return HZ_OK;
  };

  HZ_TRY(enqueue_resid());
  HZ_TRY(read_state());
  for (;;) {
    bool all_done = true;
    int max_iter = 0;
    for (int i = 0; i < S.nseg; ++i) {
      all_done = all_done && hst[i].done;
      max_iter = std::max(max_iter, hst[i].iter);
    }
    int64_t mv = 2 * int64_t(max_iter) + resid_calls;
    if (all_done) {
      // the recursive residuals say converged: confirm with the true residual
      // (a fresh residual also restarts any segment that drifted)
      HZ_TRY(enqueue_resid());
      HZ_TRY(read_state());
      bool ok = true;
      for (int i = 0; i < S.nseg; ++i) ok = ok && hst[i].done;
      if (ok || mv + 1 >= ctl.max_matvec) break;
      continue;
    }
    if (mv + 2 > ctl.max_matvec) break;
    int n_it = int(std::min<int64_t>(chunk, (ctl.max_matvec - mv) / 2));
    if (n_it < 1) break;
    for (int it = 0; it < n_it; ++it) HZ_TRY(enqueue_iter());
    HZ_TRY(read_state());
    chunk = std::min(chunk * 2, 64);
  }
  out->iters.resize(S.nseg);
  out->matvecs.resize(S.nseg);
  out->status.resize(S.nseg);
  out->relres_est.resize(S.nseg);
  for (int i = 0; i < S.nseg; ++i) {
    out->iters[i] = hst[i].iter;
    out->matvecs[i] = 2 * hst[i].iter + int(resid_calls);
    double fnv = out->fnorm[i];
    out->relres_est[i] = fnv > 0 ? std::sqrt(hst[i].rr) / fnv : 0.0;
    out->status[i] = hst[i].nan ? HZ_BREAKDOWN : (hst[i].done ? HZ_OK : HZ_NOT_CONVERGED);
  }
  return HZ_OK;
}

template int bicgstab_run<double>(hz_ctx, const SegHost&, const SellOp<double>&, const z_t*, z_t*,
                                  const KrylovCtl&, KrylovOut*, const std::string&);
template int bicgstab_run<float>(hz_ctx, const SegHost&, const SellOp<float>&, const c_t*, c_t*,
                                 const KrylovCtl&, KrylovOut*, const std::string&);
