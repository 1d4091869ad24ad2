// Operator kernels: forming A(k) (set_frequency), the sparse product, the
// patch load and a reproducible dot product.
#include "ops.h"

// ---------------------------------------------------------------- set_frequency
// Value of A(k) = K - m M + i k^2 M_eta + i k B_beta at stored entry p, m the
// mass coefficient (k^2, or the GLS one), before any Dirichlet elimination.
__device__ __forceinline__ z_t raw_entry_value(int64_t p, const OpParts& P, double k, double m) {
  const double k2 = k * k;
  z_t a = {P.K[p] - m * P.M[p], 0.0};
  if (P.Meta) a.im += k2 * P.Meta[p];
  int b = P.bidx[p];
  if (b >= 0) {
    z_t bb = P.Bb[b];
    a.re -= k * bb.im;          // i k (br + i bi) = -k bi + i k br
    a.im += k * bb.re;
  }
  return a;
}
// The same after the elimination of a Dirichlet set: the entries of its rows
// and columns are those of the identity.
__device__ __forceinline__ z_t entry_value(int64_t p, const OpParts& P, double k, double m) {
  if (P.emask) {
    const int e = P.emask[p];
    if (e == 1) return z_t{0.0, 0.0};
    if (e == 2) return z_t{1.0, 0.0};
  }
  return raw_entry_value(p, P, k, m);
}

__global__ void k_diag(int n, int64_t nrows, OpParts P, double k, double m, z_t* __restrict__ d,
                       z_t* __restrict__ dinv) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= nrows) return;
  if (i < n && P.diag[i] >= 0) {
    z_t v = entry_value(P.diag[i], P, k, m);
    d[i] = v;
    dinv[i] = crecip(v);
  } else {
    d[i] = z_t{1.0, 0.0};
    dinv[i] = z_t{1.0, 0.0};
  }
}

// One pass over the stored entries: A (optionally with column j scaled by
// dinv[j], i.e. the right-Jacobi operator A D^-1), its complex64 copy and the
// real parts of the split form.
__global__ void k_combine(int64_t npad, const int* __restrict__ col, OpParts P, double k, double m,
                          const z_t* __restrict__ dinv, int scale, z_t* __restrict__ A,
                          c_t* __restrict__ A32, double* __restrict__ R, float* __restrict__ R32) {
  int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < npad; p += stride) {
    z_t a = entry_value(p, P, k, m);
    if (scale) a = a * dinv[col[p]];
    A[p] = a;
    if (A32) A32[p] = ccast<float>(a);
    if (R) R[p] = a.re;
    if (R32) R32[p] = float(a.re);
  }
}

// Stencil-form values: slot q copies the split value of sliced-ELL position
// src[q] (0 for a missing neighbour).
__global__ void k_stencil_fill(int64_t nslot, const int* __restrict__ src, const double* __restrict__ R,
                               const float* __restrict__ R32, double* __restrict__ S, float* __restrict__ S32) {
  int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= nslot) return;
  const int p = src[q];
  S[q] = p >= 0 ? R[p] : 0.0;
  if (S32) S32[q] = p >= 0 ? R32[p] : 0.0f;
}

// Imaginary parts of the split form's listed entries.
__global__ void k_split_im(int64_t ni, const int* __restrict__ ipos, const z_t* __restrict__ A,
                           double* __restrict__ I, float* __restrict__ I32) {
  int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= ni) return;
  const int at = ipos[q];
  double v = at >= 0 ? A[at].im : 0.0;   // padding slot: 0
  I[q] = v;
  if (I32) I32[q] = float(v);
}

int op_split_im(hipStream_t s, int64_t ni, const int* ipos, const z_t* A, double* I, float* I32) {
  if (ni <= 0) return HZ_OK;
  k_split_im<<<ceil_div(ni, kBlock), kBlock, 0, s>>>(ni, ipos, A, I, I32);
  HZ_HIP(hipGetLastError());
  return HZ_OK;
}

int op_form(hipStream_t s, int64_t n, int64_t nrows, int64_t npad, const int* col, const OpParts& P, double k,
            int scale, z_t* A, c_t* A32, z_t* d, z_t* dinv, double* R, float* R32) {
  const double m = mass_coefficient(k, P.gls_h);
  k_diag<<<ceil_div(nrows, kBlock), kBlock, 0, s>>>(int(n), nrows, P, k, m, d, dinv);
  HZ_HIP(hipGetLastError());
  int grid = int(std::min<int64_t>(ceil_div(npad, kBlock), 16384));
  k_combine<<<grid, kBlock, 0, s>>>(npad, col, P, k, m, dinv, scale, A, A32, R, R32);
  HZ_HIP(hipGetLastError());
  return HZ_OK;
}

namespace {
int grow(hz_ctx ctx, DevBuf& b, size_t bytes) {
  size_t before = b.bytes;
  HZ_TRY(b.ensure(bytes));
  ctx->dev_bytes += int64_t(b.bytes) - int64_t(before);
  return HZ_OK;
}
}  // namespace

int op_set_frequency(hz_ctx ctx, const OpParts& P, double k, int scale, bool want32) {
  const bool split = ctx->split_on && !ctx->have_eta;
  const int64_t npad = ctx->sell.n_pad, ni = ctx->n_islots;
  if (split) {
    HZ_TRY(grow(ctx, ctx->d_R, sizeof(double) * npad));
    HZ_TRY(grow(ctx, ctx->d_I, sizeof(double) * std::max<int64_t>(ni, 1)));
    if (want32) {
      HZ_TRY(grow(ctx, ctx->d_R32, sizeof(float) * npad));
      HZ_TRY(grow(ctx, ctx->d_I32, sizeof(float) * std::max<int64_t>(ni, 1)));
    }
  }
  ctx->have_split = ctx->have_split32 = false;
  ctx->have_stencil = ctx->have_stencil32 = false;
  HZ_TRY(op_form(ctx->stream, ctx->h.n, ctx->sell.n_rows, npad, ctx->d_scol.as<int>(), P, k, scale,
                 ctx->d_A.as<z_t>(), want32 ? ctx->d_A32.as<c_t>() : nullptr, ctx->d_d.as<z_t>(),
                 ctx->d_dinv.as<z_t>(), split ? ctx->d_R.as<double>() : nullptr,
                 split && want32 ? ctx->d_R32.as<float>() : nullptr));
  if (split) {
    if (ni > 0) {
      k_split_im<<<ceil_div(ni, kBlock), kBlock, 0, ctx->stream>>>(
          ni, ctx->d_ipos.as<int>(), ctx->d_A.as<z_t>(), ctx->d_I.as<double>(),
          want32 ? ctx->d_I32.as<float>() : nullptr);
      HZ_HIP(hipGetLastError());
    }
    ctx->have_split = true;
    ctx->have_split32 = want32;
    if (ctx->stencil_ok) {
      const int64_t nslot = int64_t(kStencil) * ctx->sell.n_rows;
      HZ_TRY(grow(ctx, ctx->d_S, sizeof(double) * nslot));
      if (want32) HZ_TRY(grow(ctx, ctx->d_S32, sizeof(float) * nslot));
      k_stencil_fill<<<ceil_div(nslot, kBlock), kBlock, 0, ctx->stream>>>(
          nslot, ctx->d_ssrc.as<int>(), ctx->d_R.as<double>(), want32 ? ctx->d_R32.as<float>() : nullptr,
          ctx->d_S.as<double>(), want32 ? ctx->d_S32.as<float>() : nullptr);
      HZ_HIP(hipGetLastError());
      ctx->have_stencil = true;
      ctx->have_stencil32 = want32;
    }
  }
  return HZ_OK;
}

// ---------------------------------------------------------------- products
// y[row] = (A x)[row] for rows < nout; one kernel per storage form F.
template <typename T, int F>
__global__ void __launch_bounds__(kBlock) k_spmv(int64_t nout, SellOp<T> A, const cx<T>* __restrict__ x,
                                                 cx<T>* __restrict__ y) {
  int64_t row = int64_t(xcd_chunk_tile(blockIdx.x, gridDim.x)) * kBlock + threadIdx.x;
  cx<T> v = sell_row_form<F>(A, row, x);
  if (row < nout) y[row] = v;
}

template <typename T>
int op_spmv(hipStream_t s, int64_t nrows, int64_t nout, const SellOp<T>& A, const cx<T>* x, cx<T>* y) {
  if (A.val) k_spmv<T, kFormComplex><<<int(nrows / kBlock), kBlock, 0, s>>>(nout, A, x, y);
  else if (A.st) k_spmv<T, kFormStencil><<<int(nrows / kBlock), kBlock, 0, s>>>(nout, A, x, y);
  else k_spmv<T, kFormSplit><<<int(nrows / kBlock), kBlock, 0, s>>>(nout, A, x, y);
  HZ_HIP(hipGetLastError());
  return HZ_OK;
}
template int op_spmv<double>(hipStream_t, int64_t, int64_t, const SellOp<double>&, const z_t*, z_t*);
template int op_spmv<float>(hipStream_t, int64_t, int64_t, const SellOp<float>&, const c_t*, c_t*);

__global__ void k_mul(int64_t n, const z_t* __restrict__ a, const z_t* __restrict__ b, z_t* __restrict__ c) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) c[i] = a[i] * b[i];
}

int op_mul(hipStream_t s, int64_t n, const z_t* a, const z_t* b, z_t* c) {
  if (n <= 0) return HZ_OK;
  k_mul<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, a, b, c);
  HZ_HIP(hipGetLastError());
  return HZ_OK;
}

__global__ void k_fill(int64_t n, z_t* __restrict__ y, z_t v) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) y[i] = v;
}

int op_fill(hipStream_t s, int64_t n, z_t* y, z_t v) {
  if (n <= 0) return HZ_OK;
  k_fill<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, y, v);
  HZ_HIP(hipGetLastError());
  return HZ_OK;
}

__global__ void k_copy(int64_t n, const z_t* __restrict__ x, z_t* __restrict__ y) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) y[i] = x[i];
}

int op_copy(hipStream_t s, int64_t n, const z_t* x, z_t* y) {
  if (n <= 0) return HZ_OK;
  k_copy<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, x, y);
  HZ_HIP(hipGetLastError());
  return HZ_OK;
}

// ---------------------------------------------------------------- patch load
__global__ void k_patch(int np, const int* __restrict__ prow, const int* __restrict__ pptr,
                        const int* __restrict__ pcol, const double* __restrict__ pval,
                        const z_t* __restrict__ g, z_t* __restrict__ f) {
  int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= np) return;
  z_t acc = {0.0, 0.0};
  for (int q = pptr[r]; q < pptr[r + 1]; ++q) {
    z_t gv = g[pcol[q]];
    acc.re = fma(pval[q], gv.re, acc.re);
    acc.im = fma(pval[q], gv.im, acc.im);
  }
  f[prow[r]] = acc;
}

int op_load(hz_ctx ctx, const z_t* g, z_t* f) {
  HZ_TRY(op_fill(ctx->stream, ctx->h.n, f, z_t{0.0, 0.0}));
  int np = int(ctx->h.prow.size());
  if (np > 0) {
    k_patch<<<ceil_div(np, kBlock), kBlock, 0, ctx->stream>>>(np, ctx->d_prow.as<int>(), ctx->d_pptr.as<int>(),
                                                            ctx->d_pcol.as<int>(), ctx->d_pval.as<double>(), g, f);
    HZ_HIP(hipGetLastError());
  }
  return HZ_OK;
}

// ---------------------------------------------------------------- Dirichlet load
// One thread per internal row: f_i = g_i on the Dirichlet set, otherwise
// -sum over the row's stored entries in Dirichlet columns of A_ij g_j (the
// entries before the elimination); padding rows get 0.
__global__ void k_lift(int n, int64_t nrows, const int* __restrict__ ptr, const int* __restrict__ col, OpParts P,
                       double k, double m, const uint8_t* __restrict__ dir, const z_t* __restrict__ g,
                       z_t* __restrict__ f) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= nrows) return;
  if (i >= n) {
    f[i] = z_t{0.0, 0.0};
    return;
  }
  if (dir[i]) {
    f[i] = g[i];
    return;
  }
  const int sl = int(i >> 6), lane = int(i & 63);
  const int beg = ptr[sl], w = (ptr[sl + 1] - beg) >> 6;
  z_t acc = {0.0, 0.0};
  for (int q = 0; q < w; ++q) {
    const int64_t p = beg + (q << 6) + lane;
    const int j = col[p];
    if (!dir[j]) continue;
    const z_t a = raw_entry_value(p, P, k, m);
    cfma(acc, a, g[j]);
  }
  f[i] = z_t{-acc.re, -acc.im};
}

int op_lift(hz_ctx ctx, const z_t* g, z_t* f) {
  const OpParts P = op_parts(ctx);
  const int64_t nr = ctx->sell.n_rows;
  k_lift<<<ceil_div(nr, kBlock), kBlock, 0, ctx->stream>>>(int(ctx->h.n), nr, ctx->d_sptr.as<int>(),
                                                          ctx->d_scol.as<int>(), P, ctx->k,
                                                          mass_coefficient(ctx->k, P.gls_h),
                                                          ctx->d_dirrow.as<uint8_t>(), g, f);
  HZ_HIP(hipGetLastError());
  return HZ_OK;
}

// ---------------------------------------------------------------- dot
template <typename T>
__global__ void k_dot_part(int64_t n, const cx<T>* __restrict__ a, const cx<T>* __restrict__ b,
                           double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  double re = 0.0, im = 0.0;
  int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
    z_t x = ccast<double>(a[i]), y = ccast<double>(b[i]);
    re = fma(x.re, y.re, re);
    re = fma(x.im, y.im, re);
    im = fma(x.re, y.im, im);
    im = fma(-x.im, y.re, im);
  }
  double sr = block_sum(re, lds);
  double si = block_sum(im, lds);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sr;
    part[2 * blockIdx.x + 1] = si;
  }
}

__global__ void k_dot_fin(int nb, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double lds[kBlock / kWave];
  double re = block_sum_strided(part, nb, 2, lds);
  double im = block_sum_strided(part + 1, nb, 2, lds);
  if (threadIdx.x == 0) {
    out[0] = re;
    out[1] = im;
  }
}

int op_dotc_into(hipStream_t stream, int64_t n, const z_t* a, const z_t* b, double* part, double* out_dev) {
  const int g = reduce_grid(n);
  k_dot_part<double><<<g, kBlock, 0, stream>>>(n, a, b, part);
  HZ_HIP(hipGetLastError());
  k_dot_fin<<<1, kBlock, 0, stream>>>(g, part, out_dev);
  HZ_HIP(hipGetLastError());
  return HZ_OK;
}

int op_dotc(hz_ctx ctx, int64_t n, const z_t* a, const z_t* b, double* out_dev /*2*/) {
  int rc = 0;
  DevBuf* part = ctx->buf("dot.part", sizeof(double) * 2 * reduce_grid(n), &rc);
  if (rc) return rc;
  return op_dotc_into(ctx->stream, n, a, b, part->as<double>(), out_dev);
}
