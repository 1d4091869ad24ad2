// Adjoint solve and gradients of a receiver objective with respect to the
// wall admittances and the per-element absorption field.
//
// For J(p) real with derivative g = dJ/dconj(p) and A(t) p = f, the
// derivative in a real parameter t is -2 Re(lambda^H (dA/dt) p) with
// A^H lambda = g.  A is complex symmetric, so A^H = conj(A) and
// lambda = conj(A^-1 conj(g)): the adjoint reuses the forward solver.
#include "ops.h"
#include "p1.h"
#include "q1.h"
#include "solve.h"

int schwarz_solve(hz_ctx ctx, const hz_solve_opts& o, const z_t* f, z_t* p, hz_solve_info* info);

namespace {

__global__ void k_conj(int64_t n, const z_t* __restrict__ a, z_t* __restrict__ b) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) b[i] = conj(a[i]);
}

// M_e of a Q1 hexahedron (NPE 8) or P1 tetrahedron (NPE 4).
template <int NPE>
__device__ __forceinline__ void elem_mass(const double X[NPE][3], double Me[NPE][NPE]);
template <>
__device__ __forceinline__ void elem_mass<8>(const double X[8][3], double Me[8][8]) { q1::hex_mass(X, Me); }
template <>
__device__ __forceinline__ void elem_mass<4>(const double X[4][3], double Me[4][4]) { p1::tet_mass(X, Me); }
template <int NPF>
__device__ __forceinline__ void face_mass(const double X[NPF][3], double Fe[NPF][NPF]);
template <>
__device__ __forceinline__ void face_mass<4>(const double X[4][3], double Fe[4][4]) { q1::quad_mass(X, Fe); }
template <>
__device__ __forceinline__ void face_mass<3>(const double X[3][3], double Fe[3][3]) { p1::tri_mass(X, Fe); }

// dJ/deta_e += 2 k^2 Im(lambda_e^H M_e p_e), M_e formed from the node coordinates.
template <int NPE>
__global__ void __launch_bounds__(kBlock) k_grad_eta(int ne, const int* __restrict__ hex, const double* __restrict__ xyz,
                                                     const z_t* __restrict__ p, const z_t* __restrict__ lam,
                                                     double k2x2, double* __restrict__ dJ) {
  int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= ne) return;
  double X[NPE][3];
  int v[NPE];
  for (int a = 0; a < NPE; ++a) {
    v[a] = hex[int64_t(e) * NPE + a];
    for (int d = 0; d < 3; ++d) X[a][d] = xyz[int64_t(v[a]) * 3 + d];
  }
  double Me[NPE][NPE];
  elem_mass<NPE>(X, Me);
  z_t pe[NPE];
  for (int a = 0; a < NPE; ++a) pe[a] = p[v[a]];
  double im = 0.0;
  for (int a = 0; a < NPE; ++a) {
    z_t q = {0.0, 0.0};
    for (int b = 0; b < NPE; ++b) {
      q.re = fma(Me[a][b], pe[b].re, q.re);
      q.im = fma(Me[a][b], pe[b].im, q.im);
    }
    z_t l = lam[v[a]];
    im += l.re * q.im - l.im * q.re;      // Im(conj(l) q)
  }
  dJ[e] += k2x2 * im;
}

// partials of lambda^H B0_w p per wall (12 doubles per block)
template <int NPF>
__global__ void __launch_bounds__(kBlock) k_grad_beta(int nb, const int* __restrict__ bface, const int* __restrict__ btag,
                                                      const double* __restrict__ xyz, const z_t* __restrict__ p,
                                                      const z_t* __restrict__ lam, double* __restrict__ part) {
  int f = blockIdx.x * kBlock + threadIdx.x;
  double q[12];
  for (int i = 0; i < 12; ++i) q[i] = 0.0;
  if (f < nb) {
    double X[NPF][3];
    int v[NPF];
    for (int a = 0; a < NPF; ++a) {
      v[a] = bface[int64_t(f) * NPF + a];
      for (int d = 0; d < 3; ++d) X[a][d] = xyz[int64_t(v[a]) * 3 + d];
    }
    double Fe[NPF][NPF];
    face_mass<NPF>(X, Fe);
    z_t acc = {0.0, 0.0};
    for (int a = 0; a < NPF; ++a) {
      z_t s = {0.0, 0.0};
      for (int b = 0; b < NPF; ++b) {
        z_t pb = p[v[b]];
        s.re = fma(Fe[a][b], pb.re, s.re);
        s.im = fma(Fe[a][b], pb.im, s.im);
      }
      cfma_conj(acc, lam[v[a]], s);
    }
    int w = btag[f];
    for (int i = 0; i < 6; ++i) {
      q[2 * i] = (i == w) ? acc.re : 0.0;
      q[2 * i + 1] = (i == w) ? acc.im : 0.0;
    }
  }
  __shared__ double lds[kBlock / kWave];
  for (int i = 0; i < 12; ++i) {
    double s = block_sum(q[i], lds);
    if (threadIdx.x == 0) part[int64_t(blockIdx.x) * 12 + i] = s;
  }
}

__global__ void k_grad_beta_fin(int nblk, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double lds[kBlock / kWave];
  for (int i = 0; i < 12; ++i) {
    double s = block_sum_strided(part + i, nblk, 12, lds);
    if (threadIdx.x == 0) out[i] = s;
  }
}

// Adjoint state of a system with an eliminated Dirichlet set: the
// parameters act on the free rows only, so lambda is zero on D.
__global__ void k_zero_dir(int64_t n, const uint8_t* __restrict__ dir, z_t* __restrict__ lam) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n && dir[i]) lam[i] = z_t{0.0, 0.0};
}

// Receiver objective J = sum_r |p_r|^2 and its derivative g = dJ/dconj(p):
// g_r = p_r on the (distinct) receiver nodes, 0 elsewhere (g is cleared
// before this kernel).  One block: J in a fixed summation order.
__global__ void __launch_bounds__(kBlock) k_receivers(int nrec, const int* __restrict__ rec,
                                                      const z_t* __restrict__ p, z_t* __restrict__ g,
                                                      double* __restrict__ J) {
  __shared__ double lds[kBlock / kWave];
  double acc = 0.0;
  for (int r = threadIdx.x; r < nrec; r += kBlock) {
    const z_t v = p[rec[r]];
    g[rec[r]] = v;
    acc = fma(v.re, v.re, fma(v.im, v.im, acc));
  }
  const double s = block_sum(acc, lds);
  if (threadIdx.x == 0) J[0] = s;
}

}  // namespace

int receiver_objective(hz_ctx ctx, int nrec, const int* rec_host, const z_t* p, double* J_host, z_t* g) {
  int rc = 0;
  const int64_t n = ctx->h.n;
  std::vector<char> seen(size_t(n), 0);
  for (int r = 0; r < nrec; ++r) {
    if (rec_host[r] < 0 || rec_host[r] >= n) return hz_fail(HZ_ERR_INVALID, "receiver %d out of range", rec_host[r]);
    if (seen[size_t(rec_host[r])]++) return hz_fail(HZ_ERR_INVALID, "receiver %d listed twice", rec_host[r]);
  }
  DevBuf* rb = ctx->buf("rec.ids", sizeof(int) * size_t(std::max(nrec, 1)), &rc);
  if (rc) return rc;
  DevBuf* jb = ctx->buf("rec.J", sizeof(double), &rc);
  if (rc) return rc;
  void* hp = nullptr;
  HZ_TRY(ctx_pinned(ctx, sizeof(double), &hp));
  HZ_HIP(hipMemcpyAsync(rb->p, rec_host, sizeof(int) * size_t(nrec), hipMemcpyHostToDevice, ctx->stream));
  HZ_TRY(op_fill(ctx->stream, n, g, z_t{0.0, 0.0}));
  k_receivers<<<1, kBlock, 0, ctx->stream>>>(nrec, rb->as<int>(), p, g, jb->as<double>());
  HZ_HIP(hipGetLastError());
  HZ_HIP(hipMemcpyAsync(hp, jb->p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HZ_HIP(hipStreamSynchronize(ctx->stream));
  *J_host += *static_cast<double*>(hp);
  return HZ_OK;
}

int adjoint_solve(hz_ctx ctx, const hz_solve_opts& o, const z_t* p, const z_t* g, z_t* lam, double* dJ_dbeta,
                  double* dJ_deta, hz_solve_info* info) {
  int rc = 0;
  const int64_t n = ctx->h.n;
  DevBuf* gc = ctx->buf("adj.gc", sizeof(z_t) * n, &rc);
  if (rc) return rc;
  HZ_TRY(op_fill(ctx->stream, n, lam, z_t{0.0, 0.0}));
  k_conj<<<ceil_div(n, kBlock), kBlock, 0, ctx->stream>>>(n, g, gc->as<z_t>());
  HZ_HIP(hipGetLastError());
  int st = (o.method == HZ_SCHWARZ) ? schwarz_solve(ctx, o, gc->as<z_t>(), lam, info)
                                    : solve_single(ctx, o, gc->as<z_t>(), lam, info);
  if (st < 0) return st;
  k_conj<<<ceil_div(n, kBlock), kBlock, 0, ctx->stream>>>(n, lam, lam);
  HZ_HIP(hipGetLastError());
  if (ctx->dirichlet) {
    k_zero_dir<<<ceil_div(n, kBlock), kBlock, 0, ctx->stream>>>(n, ctx->d_dirmesh.as<uint8_t>(), lam);
    HZ_HIP(hipGetLastError());
  }
  const double k = ctx->k;
  if (dJ_deta) {
    if (ctx->h.npe == 4)
      k_grad_eta<4><<<ceil_div(ctx->h.ne, kBlock), kBlock, 0, ctx->stream>>>(
          ctx->h.ne, ctx->d_hex.as<int>(), ctx->d_xyz.as<double>(), p, lam, 2.0 * k * k, dJ_deta);
    else
      k_grad_eta<8><<<ceil_div(ctx->h.ne, kBlock), kBlock, 0, ctx->stream>>>(
          ctx->h.ne, ctx->d_hex.as<int>(), ctx->d_xyz.as<double>(), p, lam, 2.0 * k * k, dJ_deta);
    HZ_HIP(hipGetLastError());
  }
  if (dJ_dbeta && ctx->h.nb > 0) {
    int nblk = ceil_div(ctx->h.nb, kBlock);
    DevBuf* part = ctx->buf("adj.part", sizeof(double) * 12 * nblk, &rc);
    if (rc) return rc;
    DevBuf* res = ctx->buf("adj.res", sizeof(double) * 12, &rc);
    if (rc) return rc;
    if (ctx->h.npf == 3)
      k_grad_beta<3><<<nblk, kBlock, 0, ctx->stream>>>(ctx->h.nb, ctx->d_bface.as<int>(), ctx->d_btag.as<int>(),
                                                       ctx->d_xyz.as<double>(), p, lam, part->as<double>());
    else
      k_grad_beta<4><<<nblk, kBlock, 0, ctx->stream>>>(ctx->h.nb, ctx->d_bface.as<int>(), ctx->d_btag.as<int>(),
                                                       ctx->d_xyz.as<double>(), p, lam, part->as<double>());
    k_grad_beta_fin<<<1, kBlock, 0, ctx->stream>>>(nblk, part->as<double>(), res->as<double>());
    HZ_HIP(hipGetLastError());
    double h[12];
    HZ_HIP(hipMemcpyAsync(h, res->p, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HZ_HIP(hipStreamSynchronize(ctx->stream));
    for (int w = 0; w < 6; ++w) {
      dJ_dbeta[2 * w] += 2.0 * k * h[2 * w + 1];       // 2k Im(lambda^H B0_w p)
      dJ_dbeta[2 * w + 1] += 2.0 * k * h[2 * w];       // 2k Re(lambda^H B0_w p)
    }
  }
  HZ_HIP(hipStreamSynchronize(ctx->stream));
  return st;
}
