// Transpose-free QMR of Freund (SIAM J. Sci. Comput. 14, 1993), the
// paper's P-tfQMR (Sec. 4, solver comparison table), on the right-Jacobi
// operator B = A D^-1, for every segment of a segmented system.
//
// Half-steps come in pairs (m even, m + 1 odd), one product each:
//   even:  alpha known;  u' = u - alpha v;  w -= alpha uhat;  d = u + (theta^2/alpha) eta d
//          theta = ||w|| / tau, c = 1/sqrt(1 + theta^2), tau *= theta c, eta = c^2 alpha
//          x += eta d;  uhat = B u'
//   odd:   w -= alpha uhat;  d = u' + (theta^2/alpha) eta d;  theta, c, tau, eta as above
//          x += eta d;  rho' = r*^H w, beta = rho'/rho;  u = w + beta u'
//          v = beta uhat + beta^2 v + B u;  uhat = B u;  alpha = rho' / r*^H v
// Kernels: 3 vector, 2 product (with fused dot), 3 one-block-per-segment
// finalize per pair.  u' lives in its own buffer for the odd half-step (it
// is never copied back into u), and the odd product reads B u' from uhat
// and writes B u over it row by row, so v needs no staging buffer: 29
// vector passes per pair.  A segment whose quasi-residual bound tau sqrt(m+1)
// meets the target applies its last x update and stops; the host confirms
// with the true residual (restarting a segment that has not converged), and
// restarts segments that broke down (r*^H v or rho zero).
#include <chrono>

#include "ops.h"

namespace {

struct TqSt {
  z_t alpha, rho, beta, eta;
  double theta, tau, thr, thr2, rr;
  double chk;           // quasi-residual bound at the last stall checkpoint
  int m, iter, done, last, brk, nan, restart, pad;
  int mchk, stall_win;  // half-step of that checkpoint; its spacing (0: off)
  int stalled, pad2;    // the bound stalled: the solve ends unconfirmed
};

template <typename T>
struct TqV {
  const cx<T>* f;
  cx<T>* x;       // iterate of B x = f
  cx<T>* rs;      // shadow vector r*
  cx<T>* w;
  cx<T>* u;
  cx<T>* un;      // u' of the even half-step
  cx<T>* v;
  cx<T>* uh;      // B u, then B u'
  cx<T>* d;
};

template <typename T> __device__ __forceinline__ z_t zd(cx<T> a) { return ccast<double>(a); }
template <typename T> __device__ __forceinline__ cx<T> zt(z_t a) { return ccast<T>(a); }

__device__ __forceinline__ bool tq_off(const TqSt& S) { return S.done || S.brk || S.nan; }

__device__ __forceinline__ void acc_dot(double* q, z_t a, z_t b) {
  q[0] = fma(a.re, b.re, fma(a.im, b.im, q[0]));
  q[1] = fma(a.re, b.im, fma(-a.im, b.re, q[1]));
}

// theta, c, tau, eta after w was updated; the stopping bound
__device__ __forceinline__ void tq_qmr(TqSt& S, double ww) {
  S.theta = sqrt(ww) / S.tau;
  const double c2 = 1.0 / (1.0 + S.theta * S.theta);
  S.tau = S.tau * S.theta * sqrt(c2);
  S.eta = c2 * S.alpha;
  S.iter += 1;
  if (!isfinite(ww)) {
    S.nan = 1;
    return;
  }
  const double bound = S.tau * sqrt(double(S.m + 1));
  if (bound <= S.thr) {
    S.done = 1;       // quasi-residual bound met: the last x update follows
    S.last = 1;
  } else if (S.stall_win > 0 && S.m - S.mchk >= S.stall_win) {
    if (bound > 0.5 * S.chk) {
      S.done = 1;     // stalled: stop with the iterate reached (last x update follows)
      S.last = 1;
      S.stalled = 1;
    }
    S.chk = bound;
    S.mchk = S.m;
  }
  S.m += 1;
}

// ---------------------------------------------------------------- restart
__global__ void k_tq_mark(int nseg, TqSt* st, int all) {
  int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= nseg) return;
  st[s].restart = all ? 1 : st[s].brk;
}

// r0 = f - B x; r* = w = u = r0; d = 0; partial ||r0||^2
template <typename T, int F>
__global__ void __launch_bounds__(kBlock) k_tq_resid(Seg L, SellOp<T> A, const TqSt* st, TqV<T> V, double* part) {
  SumTile t = tile_of_sums(L);
  if (!st[t.seg].restart) return;
  const cx<T> r = zt<T>(zd(V.f[t.row]) - zd(sell_row_form<F>(A, t.row, V.x)));
  V.rs[t.row] = r;
  V.w[t.row] = r;
  V.u[t.row] = r;
  V.d[t.row] = cx<T>{T(0), T(0)};
  double q[1] = {norm2(zd(r))};
  store_partials<1>(q, part, t);
}

__global__ void k_tq_resid_fin(Seg L, TqSt* st, const double* part) {
  const int s = blockIdx.x;
  const int go = st[s].restart;
  __syncthreads();
  if (!go) return;
  double o[1];
  seg_sums<1>(L, part, s, o);
  if (threadIdx.x == 0) {
    TqSt& S = st[s];
    const double rr = o[0];
    S.rr = rr;
    S.nan = !isfinite(rr);
    S.done = (rr <= S.thr2) || S.nan;
    S.last = 0;
    S.brk = 0;
    S.tau = sqrt(rr);
    S.theta = 0.0;
    S.eta = z_t{0.0, 0.0};
    S.rho = z_t{rr, 0.0};
    S.m = 0;
    S.chk = S.tau;
    S.mchk = 0;
    // restart stays set until the first product (v = uhat = B u) is formed
  }
}

// v = uhat = B u for restarting segments; partial r*^H v
template <typename T, int F>
__global__ void HZ_PRODUCT_BOUNDS k_tq_resid_prod(Seg L, SellOp<T> A, const TqSt* st, TqV<T> V,
                                                          double* part) {
  SumTile t = tile_of_sums(L);
  const TqSt& S = st[t.seg];
  if (!S.restart || S.done) return;
  const cx<T> y = sell_row_form<F>(A, t.row, V.u);
  V.v[t.row] = y;
  V.uh[t.row] = y;
  double q[2] = {0.0, 0.0};
  acc_dot(q, zd(V.rs[t.row]), zd(y));
  store_partials<2>(q, part, t);
}

// alpha = rho / r*^H v (after a restart, or after the odd half-step's product)
__global__ void k_tq_alpha_fin(Seg L, TqSt* st, const double* part, int after_restart) {
  const int s = blockIdx.x;
  const TqSt& S0 = st[s];
  const int go = after_restart ? (S0.restart && !S0.done) : !tq_off(S0);
  const int clear = after_restart && S0.restart;
  const int done = S0.done;
  double o[2];
  seg_sums<2>(L, part, s, o);   // its barriers: every thread has read the flags
  if (threadIdx.x == 0 && clear) st[s].restart = 0;
  if (threadIdx.x == 0 && done) st[s].last = 0;
  if (!go) return;
  if (threadIdx.x == 0) {
    TqSt& S = st[s];
    const z_t sg = {o[0], o[1]};
    if (norm2(sg) == 0.0 || !isfinite(o[0]) || !isfinite(o[1])) S.brk = 1;
    else S.alpha = cdiv(S.rho, sg);
  }
}

// ---------------------------------------------------------------- even half-step
// u' = u - alpha v; w -= alpha uhat; d = u + (theta^2/alpha) eta d; partial ||w||^2
template <typename T>
__global__ void __launch_bounds__(kBlock) k_tq_even1(Seg L, const TqSt* st, TqV<T> V, double* part) {
  SumTile t = tile_of_sums(L);
  const TqSt& S = st[t.seg];
  if (tq_off(S)) return;
  const z_t a = S.alpha;
  const z_t u = zd(V.u[t.row]);
  V.un[t.row] = zt<T>(u - a * zd(V.v[t.row]));
  const cx<T> w = zt<T>(zd(V.w[t.row]) - a * zd(V.uh[t.row]));
  V.w[t.row] = w;
  const z_t g = (S.theta * S.theta) * cdiv(S.eta, a);
  V.d[t.row] = zt<T>(u + g * zd(V.d[t.row]));
  double q[1] = {norm2(zd(w))};
  store_partials<1>(q, part, t);
}

__global__ void k_tq_qmr_fin(Seg L, TqSt* st, const double* part) {
  const int s = blockIdx.x;
  const TqSt& S0 = st[s];
  const int off = tq_off(S0), done = S0.done;
  double o[1];
  seg_sums<1>(L, part, s, o);   // its barriers: every thread has read the flags
  if (off) {
    if (threadIdx.x == 0 && done) st[s].last = 0;
    return;
  }
  if (threadIdx.x == 0) tq_qmr(st[s], o[0]);
}

// x += eta d; then (unless stopping) uhat = B u'
template <typename T, int F>
__global__ void HZ_PRODUCT_BOUNDS k_tq_even2(Seg L, SellOp<T> A, const TqSt* st, TqV<T> V) {
  Tile t = tile_of(L);
  const TqSt& S = st[t.seg];
  if (S.brk || S.nan || (S.done && !S.last)) return;
  V.x[t.row] = zt<T>(zd(V.x[t.row]) + S.eta * zd(V.d[t.row]));
  if (S.done) return;
  V.uh[t.row] = sell_row_form<F>(A, t.row, V.un);
}

// ---------------------------------------------------------------- odd half-step
// w -= alpha uhat; d = u' + (theta^2/alpha) eta d; partials ||w||^2, r*^H w
template <typename T>
__global__ void __launch_bounds__(kBlock) k_tq_odd1(Seg L, const TqSt* st, TqV<T> V, double* part) {
  SumTile t = tile_of_sums(L);
  const TqSt& S = st[t.seg];
  if (tq_off(S)) return;
  const z_t a = S.alpha;
  const cx<T> w = zt<T>(zd(V.w[t.row]) - a * zd(V.uh[t.row]));
  V.w[t.row] = w;
  const z_t g = (S.theta * S.theta) * cdiv(S.eta, a);
  V.d[t.row] = zt<T>(zd(V.un[t.row]) + g * zd(V.d[t.row]));
  const z_t wv = zd(w);
  double q[3] = {norm2(wv), 0.0, 0.0};
  acc_dot(q + 1, zd(V.rs[t.row]), wv);
  store_partials<3>(q, part, t);
}

__global__ void k_tq_odd_fin(Seg L, TqSt* st, const double* part) {
  const int s = blockIdx.x;
  const TqSt& S0 = st[s];
  const int off = tq_off(S0), done = S0.done;
  double o[3];
  seg_sums<3>(L, part, s, o);   // its barriers: every thread has read the flags
  if (off) {
    if (threadIdx.x == 0 && done) st[s].last = 0;
    return;
  }
  if (threadIdx.x == 0) {
    TqSt& S = st[s];
    tq_qmr(S, o[0]);
    const z_t rho1 = {o[1], o[2]};
    if (norm2(S.rho) == 0.0 || !isfinite(o[1]) || !isfinite(o[2])) {
      if (!S.done) S.brk = 1;
    } else {
      S.beta = cdiv(rho1, S.rho);
      S.rho = rho1;
    }
  }
}

// x += eta d; then (unless stopping) u = w + beta u'
template <typename T>
__global__ void __launch_bounds__(kBlock) k_tq_odd2(Seg L, const TqSt* st, TqV<T> V) {
  Tile t = tile_of(L);
  const TqSt& S = st[t.seg];
  if (S.brk || S.nan || (S.done && !S.last)) return;
  V.x[t.row] = zt<T>(zd(V.x[t.row]) + S.eta * zd(V.d[t.row]));
  if (S.done) return;
  V.u[t.row] = zt<T>(zd(V.w[t.row]) + S.beta * zd(V.un[t.row]));
}

// uhat = B u over B u' (each row reads its old value first); v = beta B u'
// + beta^2 v + B u, the first two terms rounded to the storage type before
// the product is added; partial r*^H v
template <typename T, int F>
__global__ void HZ_PRODUCT_BOUNDS k_tq_odd3(Seg L, SellOp<T> A, const TqSt* st, TqV<T> V, double* part) {
  SumTile t = tile_of_sums(L);
  const TqSt& S = st[t.seg];
  if (tq_off(S)) return;
  const z_t b = S.beta;
  const cx<T> vt = zt<T>(b * zd(V.uh[t.row]) + (b * b) * zd(V.v[t.row]));
  const cx<T> y = sell_row_form<F>(A, t.row, V.u);
  V.uh[t.row] = y;
  const cx<T> v = zt<T>(zd(vt) + zd(y));
  V.v[t.row] = v;
  double q[2] = {0.0, 0.0};
  acc_dot(q, zd(V.rs[t.row]), zd(v));
  store_partials<2>(q, part, t);
}

__global__ void k_tq_set_thr(int nseg, TqSt* st, const double* fn2, double tol, int stall_win) {
  int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= nseg) return;
  st[s].thr2 = tol * tol * fn2[s];
  st[s].thr = tol * sqrt(fn2[s]);
  st[s].iter = 0;
  st[s].stall_win = stall_win;
  st[s].stalled = 0;
}

}  // namespace

template <typename T>
int tfqmr_run(hz_ctx ctx, const SegHost& S, const SellOp<T>& A, const cx<T>* f, cx<T>* x, const KrylovCtl& ctl,
              KrylovOut* out, const std::string& tag) {
  int rc = 0;
  const int64_t nr = S.nrows;
  const size_t vb = sizeof(cx<T>) * nr;
  const std::string p = "tfqmr." + tag + (sizeof(T) == 8 ? ".z." : ".c.");
  TqV<T> V = {};
  V.f = f;
  V.x = x;
  cx<T>** vecs[7] = {&V.rs, &V.w, &V.u, &V.un, &V.v, &V.uh, &V.d};
  const char* names[7] = {"rs", "w", "u", "un", "v", "uh", "d"};
  for (int i = 0; i < 7; ++i) {
    DevBuf* b = ctx->buf(p + names[i], vb, &rc);
    if (rc) return rc;
    *vecs[i] = b->as<cx<T>>();
  }
  DevBuf* stb = ctx->buf(p + "st", sizeof(TqSt) * S.nseg, &rc);
  if (rc) return rc;
  DevBuf* part = ctx->buf(p + "part", sizeof(double) * 3 * S.nblk, &rc);
  if (rc) return rc;
  DevBuf* fnb = ctx->buf(p + "fn2", sizeof(double) * S.nseg, &rc);
  if (rc) return rc;
  TqSt* st = stb->as<TqSt>();
  double* pt = part->as<double>();
  hipStream_t s = ctx->stream;
  const Seg& L = S.dev;

  std::vector<double> fn2;
  HZ_TRY(seg_norm2_t<T>(ctx, S, f, &fn2));
  out->fnorm.resize(S.nseg);
  for (int i = 0; i < S.nseg; ++i) out->fnorm[i] = std::sqrt(fn2[i]);
  HZ_HIP(hipMemcpyAsync(fnb->p, fn2.data(), sizeof(double) * S.nseg, hipMemcpyHostToDevice, s));
  HZ_HIP(hipMemsetAsync(stb->p, 0, sizeof(TqSt) * S.nseg, s));
  k_tq_set_thr<<<ceil_div(S.nseg, kBlock), kBlock, 0, s>>>(S.nseg, st, fnb->as<double>(), ctl.tol,
                                                            ctl.stall_halfsteps);
  HZ_HIP(hipGetLastError());

  void* hp = nullptr;
  HZ_TRY(ctx_pinned(ctx, sizeof(TqSt) * S.nseg, &hp));
  TqSt* hst = static_cast<TqSt*>(hp);
  const int grid = S.nblk;
  int64_t restarts = 0, pairs = 0;
  int chunk = 4;

  auto read_state = [&]() -> int {
    HZ_HIP(hipMemcpyAsync(hst, st, sizeof(TqSt) * S.nseg, hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    return HZ_OK;
  };
  auto enqueue_restart = [&](int all) -> int {
    k_tq_mark<<<ceil_div(S.nseg, kBlock), kBlock, 0, s>>>(S.nseg, st, all);
    if (A.val) k_tq_resid<T, kFormComplex><<<grid, kBlock, 0, s>>>(L, A, st, V, pt);
    else if (A.st) k_tq_resid<T, kFormStencil><<<grid, kBlock, 0, s>>>(L, A, st, V, pt);
    else k_tq_resid<T, kFormSplit><<<grid, kBlock, 0, s>>>(L, A, st, V, pt);
    k_tq_resid_fin<<<S.nseg, kFinBlock, 0, s>>>(L, st, pt);
    if (A.val) k_tq_resid_prod<T, kFormComplex><<<grid, kBlock, 0, s>>>(L, A, st, V, pt);
    else if (A.st) k_tq_resid_prod<T, kFormStencil><<<grid, kBlock, 0, s>>>(L, A, st, V, pt);
    else k_tq_resid_prod<T, kFormSplit><<<grid, kBlock, 0, s>>>(L, A, st, V, pt);
    k_tq_alpha_fin<<<S.nseg, kFinBlock, 0, s>>>(L, st, pt, 1);
    HZ_HIP(hipGetLastError());
    ++restarts;
    return HZ_OK;
  };
  auto enqueue_pair = [&]() -> int {
    k_tq_even1<T><<<grid, kBlock, 0, s>>>(L, st, V, pt);
    k_tq_qmr_fin<<<S.nseg, kFinBlock, 0, s>>>(L, st, pt);
    if (A.val) k_tq_even2<T, kFormComplex><<<grid, kBlock, 0, s>>>(L, A, st, V);
    else if (A.st) k_tq_even2<T, kFormStencil><<<grid, kBlock, 0, s>>>(L, A, st, V);
    else k_tq_even2<T, kFormSplit><<<grid, kBlock, 0, s>>>(L, A, st, V);
    k_tq_odd1<T><<<grid, kBlock, 0, s>>>(L, st, V, pt);
    k_tq_odd_fin<<<S.nseg, kFinBlock, 0, s>>>(L, st, pt);
    k_tq_odd2<T><<<grid, kBlock, 0, s>>>(L, st, V);
    if (A.val) k_tq_odd3<T, kFormComplex><<<grid, kBlock, 0, s>>>(L, A, st, V, pt);
    else if (A.st) k_tq_odd3<T, kFormStencil><<<grid, kBlock, 0, s>>>(L, A, st, V, pt);
    else k_tq_odd3<T, kFormSplit><<<grid, kBlock, 0, s>>>(L, A, st, V, pt);
    k_tq_alpha_fin<<<S.nseg, kFinBlock, 0, s>>>(L, st, pt, 0);
    HZ_HIP(hipGetLastError());
    ++pairs;
    return HZ_OK;
  };

  HZ_TRY(enqueue_restart(1));
  HZ_TRY(read_state());
  for (;;) {
    bool all_done = true, any_brk = false, any_stalled = false;
    for (int i = 0; i < S.nseg; ++i) {
      all_done = all_done && hst[i].done;
      any_brk = any_brk || (hst[i].brk && !hst[i].done);
      any_stalled = any_stalled || hst[i].stalled;
    }
    // products so far: two per restart, two per queued pair (stopped segments idle)
    const int64_t mv = 2 * restarts + 2 * pairs;
    if (all_done && any_stalled) break;   // hand the iterate reached back to the refinement
    if (all_done) {
      HZ_TRY(enqueue_restart(1));   // confirm with the true residual
      HZ_TRY(read_state());
      bool ok = true;
      for (int i = 0; i < S.nseg; ++i) ok = ok && hst[i].done;
      if (ok || mv + 2 >= ctl.max_matvec) break;
      continue;
    }
    if (mv + 2 > ctl.max_matvec) break;
    if (any_brk) {
      HZ_TRY(enqueue_restart(0));
      HZ_TRY(read_state());
      continue;
    }
    const int n_pair = int(std::min<int64_t>(chunk, (ctl.max_matvec - mv) / 2));
    if (n_pair < 1) break;
    for (int c = 0; c < n_pair; ++c) HZ_TRY(enqueue_pair());
    HZ_TRY(read_state());
    chunk = std::min(chunk * 2, 32);
  }
  out->iters.resize(S.nseg);
  out->matvecs.resize(S.nseg);
  out->status.resize(S.nseg);
  out->relres_est.resize(S.nseg);
  for (int i = 0; i < S.nseg; ++i) {
    out->iters[i] = hst[i].iter;
    out->matvecs[i] = hst[i].iter + 2 * int(restarts);
    const double fnv = out->fnorm[i];
    out->relres_est[i] = fnv > 0 ? std::sqrt(hst[i].rr) / fnv : 0.0;
    out->status[i] = hst[i].nan ? HZ_BREAKDOWN : (hst[i].done && !hst[i].stalled ? HZ_OK : HZ_NOT_CONVERGED);
  }
  return HZ_OK;
}

template int tfqmr_run<double>(hz_ctx, const SegHost&, const SellOp<double>&, const z_t*, z_t*, const KrylovCtl&,
                               KrylovOut*, const std::string&);
template int tfqmr_run<float>(hz_ctx, const SegHost&, const SellOp<float>&, const c_t*, c_t*, const KrylovCtl&,
                              KrylovOut*, const std::string&);
