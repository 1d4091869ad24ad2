// Restarted GMRES(m) on the right-Jacobi operator, for every segment of a
// segmented system (added beside the paper's Sec. 4 solvers).
//
// Arnoldi uses classical Gram-Schmidt with one re-orthogonalisation (CGS2),
// h1 = V^H w, w1 = w - V h1, h2 = V^H w1, w2 = w1 - V h2, in three passes
// over the basis per step instead of four:
//   1. the product w = A v_j, and h1's partial sums from the same rows;
//   2. w1 formed in registers from the row's basis entries, which stay in
//      registers for h2's partial sums (no write of w1);
//   3. w2 = w - V (h1 + h2) written as the next basis vector, with the
//      partial sums of ||w2||^2.
// The basis is stored unnormalised: v_i = s_i V_i with s_i = 1 / ||w2|| of
// the step that made it (1 / beta for V_0), applied wherever V is read, so
// no pass rescales it.  Each pass is followed by one small finalize kernel
// (coefficients; then the Hessenberg column, the complex Givens rotations
// and the residual estimate, in FP64 on the device), so a whole restart
// cycle is queued without a host round trip; the host reads the
// per-segment state once per cycle.  With storage type float the basis and
// the operator are complex64 while the Gram-Schmidt coefficients, H and
// the rotations remain FP64.
#include "ops.h"

namespace {

constexpr int kGmMaxM = 128;   // largest restart length

constexpr int NV = 8;    // basis vectors per multi-dot chunk

struct GmSt {
  double beta, thr2, est, inv_next;
  int k, done, cyc, nan;
  int iters, pad0;
};

struct GmArr {         // per-segment small arrays (FP64)
  z_t* H;              // [(m+1) x m] column-major, per segment
  double* cs;          // [m]
  z_t* sn;             // [m]
  z_t* g;              // [m+1]
  z_t* y;              // [m]
  z_t* h1;             // [m+1] first-pass coefficients
  z_t* h2;             // [m+1] second-pass coefficients
  double* vs;          // [m+1] scale of each stored basis vector (v_i = vs_i V_i)
  int m;
};

template <typename T> __device__ __forceinline__ z_t zd(cx<T> a) { return ccast<double>(a); }

// V0 = f - A u; partial ||V0||^2
template <typename T, int F>
__global__ void __launch_bounds__(kBlock) k_resid(Seg L, SellOp<T> A, const cx<T>* __restrict__ f,
                                                  const cx<T>* __restrict__ u, cx<T>* __restrict__ V0,
                                                  double* part) {
  SumTile t = tile_of_sums(L);
  z_t r = zd(f[t.row]) - zd(sell_row_form<F>(A, t.row, u));
  cx<T> rs = ccast<T>(r);
  V0[t.row] = rs;
  double q[1] = {norm2(zd(rs))};
  store_partials<1>(q, part, t);
}

__global__ void k_beta_fin(Seg L, GmSt* st, GmArr G, const double* part) {
  int s = blockIdx.x;
  double o[1];
  seg_sums<1>(L, part, s, o);
  if (threadIdx.x == 0) {
    const double rr = o[0];
    GmSt& S = st[s];
    double b = sqrt(rr);
    S.beta = b;
    S.est = b;
    S.k = 0;
    S.nan = !isfinite(rr);
    S.done = (rr <= S.thr2) || S.nan;
    S.cyc = S.done;
    S.inv_next = b > 0.0 ? 1.0 / b : 0.0;
    G.vs[int64_t(s) * (G.m + 1)] = S.inv_next;
    z_t* g = G.g + int64_t(s) * (G.m + 1);
    g[0] = z_t{b, 0.0};
    for (int i = 1; i <= G.m; ++i) g[i] = z_t{0.0, 0.0};
  }
}

// Partial sums of 2 (j + 1) quantities, 16 per chunk of 8 basis vectors:
// chunk_to_lds reduces one chunk's 16 values within each wave and puts the
// waves' sums in LDS; after all chunks, lds_to_partials (one barrier) adds
// the waves in order and stores quantity u of chunk c at
// part[(16 c + u) nblk + tile]: each quantity's block partials contiguous,
// the layout k_mdot_fin reads.  Fixed summation order.
constexpr int kMaxChunks = (128 + 1 + NV - 1) / NV;
typedef double ChunkLds[kMaxChunks][2 * NV][kBlock / kWave];

// Wave sums of 16 quantities by recursive halving: at each of the first
// four exchanges (lane distance 32, 16, 8, 4) a lane keeps half of its
// quantities, adds its partner's copies of them and hands over the other
// half, so 8 + 4 + 2 + 1 values cross lanes instead of 16 x 6; then lane
// distances 2 and 1 finish the one quantity each lane holds.  Afterwards
// lane l holds the wave sum of quantity 8 b5 + 4 b4 + 2 b3 + b2 (b = the
// bits of l).  A fixed order: the result does not depend on timing.
__device__ __forceinline__ double wave_sum16(const double (&q)[2 * NV], int lane, int* which) {
  double a[8], b[4], c[2], d;
  const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8, h2 = lane & 4;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double keep = h5 ? q[8 + k] : q[k], give = h5 ? q[k] : q[8 + k];
    a[k] = keep + __shfl_xor(give, 32, kWave);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double keep = h4 ? a[4 + k] : a[k], give = h4 ? a[k] : a[4 + k];
    b[k] = keep + __shfl_xor(give, 16, kWave);
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double keep = h3 ? b[2 + k] : b[k], give = h3 ? b[k] : b[2 + k];
    c[k] = keep + __shfl_xor(give, 8, kWave);
  }
  {
    const double keep = h2 ? c[1] : c[0], give = h2 ? c[0] : c[1];
    d = keep + __shfl_xor(give, 4, kWave);
  }
  d += __shfl_xor(d, 2, kWave);
  d += __shfl_xor(d, 1, kWave);
  *which = 8 * h5 + 4 * h4 + 2 * h3 + h2;
  return d;
}

__device__ __forceinline__ void chunk_to_lds(const double (&q)[2 * NV], int c, ChunkLds& lds) {
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  int u = 0;
  const double v = wave_sum16(q, lane, &u);
  if ((lane & 3) == 0) lds[c][u][w] = v;
}

__device__ __forceinline__ void lds_to_partials(const ChunkLds& lds, int nchunk, double* part, int nblk, int tile) {
  __syncthreads();
  for (int e = threadIdx.x; e < nchunk * 2 * NV; e += kBlock) {
    const int c = e / (2 * NV), u = e % (2 * NV);
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) t += lds[c][u][i];
    part[(int64_t(c) * 2 * NV + u) * nblk + tile] = t;
  }
}

// conj(a) b accumulated into q[0] (re), q[1] (im)
__device__ __forceinline__ void dot_acc(double* q, z_t a, z_t b) {
  q[0] = fma(a.re, b.re, fma(a.im, b.im, q[0]));
  q[1] = fma(a.re, b.im, fma(-a.im, b.re, q[1]));
}

// Pass 1: w = A v_j = s_j (A V_j), and the partial sums of h1_i = v_i^H w
// (i <= j) from the same rows.
template <typename T, int F>
__global__ void HZ_PRODUCT_BOUNDS k_gs_prod(Seg L, SellOp<T> A, const GmSt* st, GmArr G,
                                                    const cx<T>* __restrict__ V, int64_t ld, int j,
                                                    cx<T>* __restrict__ w, double* __restrict__ part) {
  __shared__ ChunkLds lds;
  Tile t = tile_of(L);
  if (st[t.seg].cyc) return;
  const double* vs = G.vs + int64_t(t.seg) * (G.m + 1);
  const z_t y = vs[j] * zd(sell_row_form<F>(A, t.row, V + int64_t(j) * ld));
  const cx<T> ys = ccast<T>(y);
  w[t.row] = ys;
  const z_t wv = zd(ys);
  const int nchunk = (j + NV) / NV;
  for (int c = 0; c < nchunk; ++c) {
    double q[2 * NV];
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int i = c * NV + u;
      q[2 * u] = q[2 * u + 1] = 0.0;
      if (i <= j) dot_acc(&q[2 * u], vs[i] * zd(V[int64_t(i) * ld + t.row]), wv);
    }
    chunk_to_lds(q, c, lds);
  }
  lds_to_partials(lds, nchunk, part, L.nblk, t.tile);
}

// Pass 2 with R threads per row (R = 4 or 8), for j + 1 <= R Q: a block of
// 256 threads walks its 256-row tile 256 / R rows at a time; thread (row r,
// part p) holds basis vectors p Qa .. p Qa + Qa - 1 (Qa = ceil((j + 1) / R))
// of its row in registers; the R parts' sums of h1_i v_i meet by lane
// exchanges (the same value in all R lanes), giving w1; each thread
// accumulates its part's dots v_i^H w1 over its rows, and only then are
// they summed over the wave's rows of that part and over the block's waves
// in order (a fixed order), and stored in the chunk layout of k_mdot_fin.
template <typename T, int R, int Q>
__global__ void __launch_bounds__(kBlock) k_gs_second(Seg L, const GmSt* st, GmArr G, const cx<T>* __restrict__ V,
                                                      int64_t ld, int j, const cx<T>* __restrict__ w,
                                                      double* __restrict__ part) {
  constexpr int kW = kBlock / kWave;
  constexpr int kRowsPerWave = kWave / R;
  __shared__ double lds[R * Q][2][kW];
  const int tile = xcd_chunk_tile(blockIdx.x, gridDim.x);
  const int seg = L.blk_seg[tile];
  if (st[seg].cyc) return;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int p = lane / kRowsPerWave, rl = lane % kRowsPerWave;
  const int n = j + 1, qa = (n + R - 1) / R, i0 = p * qa;
  const double* vs = G.vs + int64_t(seg) * (G.m + 1);
  const z_t* h1 = G.h1 + int64_t(seg) * (G.m + 1);
  double d[Q][2];
#pragma unroll
  for (int u = 0; u < Q; ++u) d[u][0] = d[u][1] = 0.0;
#pragma unroll(Q <= 4 ? 2 : 1)
  for (int r0 = 0; r0 < kBlock; r0 += kW * kRowsPerWave) {
    const int64_t row = int64_t(tile) * kBlock + r0 + wave * kRowsPerWave + rl;
    cx<T> v[Q];
#pragma unroll
    for (int u = 0; u < Q; ++u) {
      const int i = i0 + u;
      v[u] = (u < qa && i < n) ? V[int64_t(i) * ld + row] : cx<T>{T(0), T(0)};
    }
    z_t acc = p == 0 ? zd(w[row]) : z_t{0.0, 0.0};
#pragma unroll
    for (int u = 0; u < Q; ++u) {
      const int i = i0 + u;
      if (u < qa && i < n) {
        const z_t h = vs[i] * h1[i], x = zd(v[u]);
        acc.re -= h.re * x.re - h.im * x.im;
        acc.im -= h.re * x.im + h.im * x.re;
      }
    }
#pragma unroll
    for (int o = kRowsPerWave; o < kWave; o <<= 1) {
      acc.re += __shfl_xor(acc.re, o, kWave);
      acc.im += __shfl_xor(acc.im, o, kWave);
    }
    const z_t w1 = zd(ccast<T>(acc));   // the storage precision's w1, as if stored
#pragma unroll
    for (int u = 0; u < Q; ++u) {
      const int i = i0 + u;
      if (u < qa && i < n) dot_acc(d[u], vs[i] * zd(v[u]), w1);
    }
  }
#pragma unroll
  for (int u = 0; u < Q; ++u) {
#pragma unroll
    for (int o = kRowsPerWave / 2; o > 0; o >>= 1) {
      d[u][0] += __shfl_xor(d[u][0], o, kWave);
      d[u][1] += __shfl_xor(d[u][1], o, kWave);
    }
    const int i = i0 + u;
    if (rl == 0 && u < qa && i < n) {
      lds[i][0][wave] = d[u][0];
      lds[i][1][wave] = d[u][1];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 2 * n; e += kBlock) {
    const int i = e >> 1, ri = e & 1;
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < kW; ++k) t += lds[i][ri][k];
    part[(int64_t(i / NV) * 2 * NV + 2 * (i % NV) + ri) * L.nblk + tile] = t;
  }
}

// Pass 3: w2 = w1 - sum_i h2_i v_i with w1 = w - sum_i h1_i v_i, written in
// place of w (the next stored basis vector); partial ||w2||^2.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_gs_third(Seg L, const GmSt* st, GmArr G, const cx<T>* __restrict__ V,
                                                     int64_t ld, int j, cx<T>* __restrict__ w, double* part) {
  SumTile t = tile_of_sums(L);
  if (st[t.seg].cyc) return;
  const double* vs = G.vs + int64_t(t.seg) * (G.m + 1);
  const z_t* h1 = G.h1 + int64_t(t.seg) * (G.m + 1);
  const z_t* h2 = G.h2 + int64_t(t.seg) * (G.m + 1);
  z_t a1 = zd(w[t.row]), a2 = {0.0, 0.0};
  for (int i = 0; i <= j; ++i) {
    const z_t v = vs[i] * zd(V[int64_t(i) * ld + t.row]);
    const z_t p = h1[i], r = h2[i];
    a1.re -= p.re * v.re - p.im * v.im;
    a1.im -= p.re * v.im + p.im * v.re;
    a2.re -= r.re * v.re - r.im * v.im;
    a2.im -= r.re * v.im + r.im * v.re;
  }
  const z_t w1 = zd(ccast<T>(a1));
  const cx<T> ws = ccast<T>(w1 + a2);
  w[t.row] = ws;
  double q[1] = {norm2(zd(ws))};
  store_partials<1>(q, part, t);
}

// partial h_i = V_i^H w for i in chunk blockIdx.y (i <= j)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_mdot(Seg L, const GmSt* st, GmArr G, const cx<T>* __restrict__ V,
                                                 int64_t ld, int j, const cx<T>* __restrict__ w,
                                                 double* part) {
  SumTile t = tile_of_sums(L);
  if (st[t.seg].cyc) return;
  int i0 = blockIdx.y * NV;
  z_t wv = zd(w[t.row]);
  double q[2 * NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    int i = i0 + c;
    z_t a = {0.0, 0.0};
    if (i <= j) a = G.vs[int64_t(t.seg) * (G.m + 1) + i] * zd(V[int64_t(i) * ld + t.row]);
    q[2 * c] = a.re * wv.re + a.im * wv.im;
    q[2 * c + 1] = a.re * wv.im - a.im * wv.re;
  }
  store_partials_qmajor<2 * NV>(q, part + int64_t(blockIdx.y) * L.nblk * 2 * NV, L.nblk, t);
}

// block (s, i): coefficient i of segment s.  pass 1 -> h1; pass 2 -> h2 and H[:, j] = h1 + h2.
// The real and imaginary block partials of a coefficient are two
// contiguous runs: coalesced loads, several in flight per thread, then the
// block's sum in a fixed order.
__global__ void __launch_bounds__(kFinBlock) k_mdot_fin(Seg L, const GmSt* st, GmArr G, const double* part, int j,
                                                        int pass) {
  int s = blockIdx.x, i = blockIdx.y;
  const int cyc = st[s].cyc;
  int c = i / NV, q = i % NV;
  const double* pre = part + (int64_t(c) * 2 * NV + 2 * q) * L.nblk;
  const double* pim = pre + L.nblk;
  const int b0 = L.nseg == 1 ? 0 : L.seg_blk[s], b1 = L.nseg == 1 ? L.nblk : L.seg_blk[s + 1];
  double ar = 0.0, ai = 0.0;
#pragma unroll 4
  for (int b = b0 + int(threadIdx.x); b < b1; b += kFinBlock) {
    ar += pre[b];
    ai += pim[b];
  }
  __shared__ double lds[2][kFinBlock / kWave];
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  ar = wave_sum(ar);
  ai = wave_sum(ai);
  if (lane == 0) {
    lds[0][w] = ar;
    lds[1][w] = ai;
  }
  __syncthreads();
  if (cyc) return;
  if (threadIdx.x == 0) {
    double re = 0.0, im = 0.0;
    for (int k = 0; k < kFinBlock / kWave; ++k) {
      re += lds[0][k];
      im += lds[1][k];
    }
    z_t h = {re, im};
    if (pass == 1) {
      G.h1[int64_t(s) * (G.m + 1) + i] = h;
    } else {
      G.h2[int64_t(s) * (G.m + 1) + i] = h;
      z_t* H = G.H + int64_t(s) * (G.m + 1) * G.m;
      H[int64_t(j) * (G.m + 1) + i] = G.h1[int64_t(s) * (G.m + 1) + i] + h;
    }
  }
}

// w -= sum_{i<=j} h_i V_i (h = h1 or h2); optionally partial ||w||^2
template <typename T, bool NORM>
__global__ void __launch_bounds__(kBlock) k_axpy(Seg L, const GmSt* st, GmArr G, const cx<T>* __restrict__ V,
                                                 int64_t ld, int j, int pass, cx<T>* __restrict__ w,
                                                 double* part) {
  SumTile t = tile_of_sums(L);
  if (st[t.seg].cyc) return;
  const z_t* h = (pass == 1 ? G.h1 : G.h2) + int64_t(t.seg) * (G.m + 1);
  const double* vs = G.vs + int64_t(t.seg) * (G.m + 1);
  z_t acc = zd(w[t.row]);
  for (int i = 0; i <= j; ++i) {
    z_t v = vs[i] * zd(V[int64_t(i) * ld + t.row]);
    z_t hi = h[i];
    acc.re -= hi.re * v.re - hi.im * v.im;
    acc.im -= hi.re * v.im + hi.im * v.re;
  }
  cx<T> ws = ccast<T>(acc);
  w[t.row] = ws;
  if (NORM) {
    double q[1] = {norm2(zd(ws))};
    store_partials<1>(q, part, t);
  }
}

// New Hessenberg column j: subdiagonal, previous rotations, new rotation,
// residual estimate |g_{j+1}|.
// The column and the previous rotations are staged in LDS by the whole
// block, so the sequential rotation loop of thread 0 reads no global memory.
__global__ void __launch_bounds__(kFinBlock) k_givens_fin(Seg L, GmSt* st, GmArr G, const double* part, int j) {
  int s = blockIdx.x;
  const int cyc = st[s].cyc;
  const int m = G.m;
  z_t* H = G.H + int64_t(s) * (m + 1) * m + int64_t(j) * (m + 1);
  double* cs = G.cs + int64_t(s) * m;
  z_t* sn = G.sn + int64_t(s) * m;
  z_t* g = G.g + int64_t(s) * (m + 1);
  __shared__ z_t hS[kGmMaxM + 1], snS[kGmMaxM];
  __shared__ double csS[kGmMaxM];
  if (!cyc)
    for (int i = threadIdx.x; i <= j; i += kFinBlock) {
      hS[i] = H[i];
      if (i < j) {
        csS[i] = cs[i];
        snS[i] = sn[i];
      }
    }
  double o[1];
  seg_sums<1>(L, part, s, o);   // its barriers also order the staging above
  if (cyc || threadIdx.x != 0) return;
  const double ww = o[0];
  GmSt& S = st[s];
  double hn = sqrt(ww);
  hS[j + 1] = z_t{hn, 0.0};
  for (int i = 0; i < j; ++i) {
    z_t a = hS[i], b = hS[i + 1];
    hS[i] = csS[i] * a + snS[i] * b;
    hS[i + 1] = (-1.0 * (conj(snS[i]) * a)) + csS[i] * b;
  }
  for (int i = 0; i < j; ++i) H[i] = hS[i];
  z_t a = hS[j], b = hS[j + 1];
  double rho = sqrt(norm2(a) + norm2(b));
  double c;
  z_t sv;
  if (rho == 0.0) {
    c = 1.0;
    sv = z_t{0.0, 0.0};
  } else if (norm2(a) == 0.0) {
    c = 0.0;
    sv = z_t{1.0, 0.0};
  } else {
    double aa = sqrt(norm2(a));
    c = aa / rho;
    sv = (1.0 / (aa * rho)) * (a * conj(b));
  }
  cs[j] = c;
  sn[j] = sv;
  H[j] = c * a + sv * b;
  H[j + 1] = z_t{0.0, 0.0};
  z_t gj = g[j];
  g[j + 1] = -1.0 * (conj(sv) * gj);
  g[j] = c * gj;
  S.k = j + 1;
  S.iters += 1;
  S.est = sqrt(norm2(g[j + 1]));
  bool bad = !isfinite(hn) || !isfinite(S.est);
  if (bad) S.nan = 1;
  if (bad || hn == 0.0 || S.est * S.est <= S.thr2) S.cyc = 1;
  S.inv_next = hn > 0.0 ? 1.0 / hn : 0.0;
  G.vs[int64_t(s) * (m + 1) + j + 1] = S.inv_next;
}

// y = H(0:k,0:k)^-1 g(0:k)
__global__ void k_solve_fin(const GmSt* st, GmArr G, int nseg) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  const GmSt& S = st[s];
  if (S.done || S.nan) return;
  const int m = G.m, k = S.k;
  const z_t* H = G.H + int64_t(s) * (m + 1) * m;
  const z_t* g = G.g + int64_t(s) * (m + 1);
  z_t* y = G.y + int64_t(s) * m;
  for (int i = k - 1; i >= 0; --i) {
    z_t acc = g[i];
    for (int l = i + 1; l < k; ++l) acc = acc - H[int64_t(l) * (m + 1) + i] * y[l];
    y[i] = cdiv(acc, H[int64_t(i) * (m + 1) + i]);
  }
}

// u += sum_{i<k} y_i V_i
template <typename T>
__global__ void __launch_bounds__(kBlock) k_update(Seg L, const GmSt* st, GmArr G, const cx<T>* __restrict__ V,
                                                   int64_t ld, cx<T>* __restrict__ u) {
  Tile t = tile_of(L);
  const GmSt& S = st[t.seg];
  if (S.done || S.nan || S.k == 0) return;
  const z_t* y = G.y + int64_t(t.seg) * G.m;
  const double* vs = G.vs + int64_t(t.seg) * (G.m + 1);
  z_t acc = zd(u[t.row]);
  for (int i = 0; i < S.k; ++i) {
    z_t v = vs[i] * zd(V[int64_t(i) * ld + t.row]);
    z_t yi = y[i];
    acc.re += yi.re * v.re - yi.im * v.im;
    acc.im += yi.re * v.im + yi.im * v.re;
  }
  u[t.row] = ccast<T>(acc);
}

__global__ void k_init_st(int nseg, GmSt* st, const double* fn2, double tol) {
  int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= nseg) return;
  GmSt z = {};
  z.thr2 = tol * tol * fn2[s];
  st[s] = z;
}

// pass 1 in the operator's storage form
template <typename T>
int gs_pass1(hipStream_t s, const Seg& L, const SellOp<T>& A, const GmSt* st, const GmArr& G, const cx<T>* V,
             int64_t ld, int j, cx<T>* w, double* pt, int grid) {
  if (A.val) k_gs_prod<T, kFormComplex><<<grid, kBlock, 0, s>>>(L, A, st, G, V, ld, j, w, pt);
  else if (A.st) k_gs_prod<T, kFormStencil><<<grid, kBlock, 0, s>>>(L, A, st, G, V, ld, j, w, pt);
  else k_gs_prod<T, kFormSplit><<<grid, kBlock, 0, s>>>(L, A, st, G, V, ld, j, w, pt);
  HZ_HIP(hipGetLastError());
  return HZ_OK;
}

}  // namespace

template <typename T>
int gmres_run(hz_ctx ctx, const SegHost& S, const SellOp<T>& A, const cx<T>* f, cx<T>* u,
              const KrylovCtl& ctl, KrylovOut* out, const std::string& tag) {
  int rc = 0;
  const int m = ctl.restart;
  if (m < 1 || m > kGmMaxM) return hz_fail(HZ_ERR_INVALID, "GMRES restart %d not in 1..%d", m, kGmMaxM);
  const int64_t ld = S.nrows;
  const std::string p = "gm." + tag + (sizeof(T) == 8 ? ".z." : ".c.");
  DevBuf* Vb = ctx->buf(p + "V", sizeof(cx<T>) * ld * (m + 1), &rc);
  if (rc) return rc;
  const int nchunk = ceil_div(m + 1, NV);
  DevBuf* part = ctx->buf(p + "part", sizeof(double) * int64_t(nchunk) * S.nblk * 2 * NV, &rc);
  if (rc) return rc;
  DevBuf* stb = ctx->buf(p + "st", sizeof(GmSt) * S.nseg, &rc);
  if (rc) return rc;
  const int64_t ns = S.nseg;
  DevBuf* small = ctx->buf(p + "small",
                           sizeof(z_t) * ns * ((m + 1) * m + m + (m + 1) + m + 2 * (m + 1)) +
                               sizeof(double) * ns * (m + (m + 1)), &rc);
  if (rc) return rc;
  DevBuf* fnb = ctx->buf(p + "fn2", sizeof(double) * S.nseg, &rc);
  if (rc) return rc;
  GmArr G;
  G.m = m;
  z_t* zp = small->as<z_t>();
  G.H = zp; zp += ns * (m + 1) * m;
  G.sn = zp; zp += ns * m;
  G.g = zp; zp += ns * (m + 1);
  G.y = zp; zp += ns * m;
  G.h1 = zp; zp += ns * (m + 1);
  G.h2 = zp; zp += ns * (m + 1);
  G.cs = reinterpret_cast<double*>(zp);
  G.vs = G.cs + ns * m;
  GmSt* st = stb->as<GmSt>();
  cx<T>* V = Vb->as<cx<T>>();
  double* pt = part->as<double>();
  hipStream_t s = ctx->stream;
  const Seg& L = S.dev;

  std::vector<double> fn2;
  HZ_TRY(seg_norm2_t<T>(ctx, S, f, &fn2));
  out->fnorm.resize(S.nseg);
  for (int i = 0; i < S.nseg; ++i) out->fnorm[i] = std::sqrt(fn2[i]);
  HZ_HIP(hipMemcpyAsync(fnb->p, fn2.data(), sizeof(double) * S.nseg, hipMemcpyHostToDevice, s));
  k_init_st<<<ceil_div(S.nseg, kBlock), kBlock, 0, s>>>(S.nseg, st, fnb->as<double>(), ctl.tol);
  HZ_HIP(hipGetLastError());

  void* hp = nullptr;
  HZ_TRY(ctx_pinned(ctx, sizeof(GmSt) * S.nseg, &hp));
  GmSt* hst = static_cast<GmSt*>(hp);
  std::vector<int64_t> mv(S.nseg, 0);
  int64_t mv_max = 0;
  const int grid = S.nblk;
  for (;;) {
    // residual of the current iterate; converged segments stop here
    if (A.val) k_resid<T, kFormComplex><<<grid, kBlock, 0, s>>>(L, A, f, u, V, pt);
    else if (A.st) k_resid<T, kFormStencil><<<grid, kBlock, 0, s>>>(L, A, f, u, V, pt);
    else k_resid<T, kFormSplit><<<grid, kBlock, 0, s>>>(L, A, f, u, V, pt);
    k_beta_fin<<<S.nseg, kFinBlock, 0, s>>>(L, st, G, pt);
    HZ_HIP(hipGetLastError());
    int mc = int(std::min<int64_t>(m, ctl.max_matvec - mv_max - 1));
    if (mc >= 1) {
      for (int j = 0; j < mc; ++j) {
        cx<T>* w = V + int64_t(j + 1) * ld;
        dim3 gd(grid, ceil_div(j + 1, NV));
        dim3 gf(S.nseg, j + 1);
        HZ_TRY(gs_pass1<T>(s, L, A, st, G, V, ld, j, w, pt, grid));
        k_mdot_fin<<<gf, kFinBlock, 0, s>>>(L, st, G, pt, j, 1);
        if (j + 1 <= 16) k_gs_second<T, 4, 4><<<grid, kBlock, 0, s>>>(L, st, G, V, ld, j, w, pt);
        else if (j + 1 <= 32) k_gs_second<T, 8, 4><<<grid, kBlock, 0, s>>>(L, st, G, V, ld, j, w, pt);
        else if (j + 1 <= 56) k_gs_second<T, 8, 7><<<grid, kBlock, 0, s>>>(L, st, G, V, ld, j, w, pt);
        else {
          // beyond 56 basis vectors: w1 stored, then a multi-dot pass
          k_axpy<T, false><<<grid, kBlock, 0, s>>>(L, st, G, V, ld, j, 1, w, pt);
          k_mdot<T><<<gd, kBlock, 0, s>>>(L, st, G, V, ld, j, w, pt);
        }
        k_mdot_fin<<<gf, kFinBlock, 0, s>>>(L, st, G, pt, j, 2);
        if (j + 1 <= 56) k_gs_third<T><<<grid, kBlock, 0, s>>>(L, st, G, V, ld, j, w, pt);
        else k_axpy<T, true><<<grid, kBlock, 0, s>>>(L, st, G, V, ld, j, 2, w, pt);
        k_givens_fin<<<S.nseg, kFinBlock, 0, s>>>(L, st, G, pt, j);
        HZ_HIP(hipGetLastError());
      }
      k_solve_fin<<<ceil_div(S.nseg, 64), 64, 0, s>>>(st, G, S.nseg);
      k_update<T><<<grid, kBlock, 0, s>>>(L, st, G, V, ld, u);
      HZ_HIP(hipGetLastError());
    }
    HZ_HIP(hipMemcpyAsync(hst, st, sizeof(GmSt) * S.nseg, hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    bool all_done = true;
    for (int i = 0; i < S.nseg; ++i) {
      mv[i] += 1;
      if (!hst[i].done) mv[i] += hst[i].k;
      mv_max = std::max(mv_max, mv[i]);
      all_done = all_done && (hst[i].done || hst[i].nan);
    }
    if (all_done || mc < 1 || mv_max >= ctl.max_matvec) break;
  }
  out->iters.resize(S.nseg);
  out->matvecs.resize(S.nseg);
  out->status.resize(S.nseg);
  out->relres_est.resize(S.nseg);
  for (int i = 0; i < S.nseg; ++i) {
    out->iters[i] = hst[i].iters;
    out->matvecs[i] = int(mv[i]);
    double fnv = out->fnorm[i];
    out->relres_est[i] = fnv > 0 ? hst[i].est / fnv : 0.0;
    out->status[i] = hst[i].nan ? HZ_BREAKDOWN : (hst[i].done ? HZ_OK : HZ_NOT_CONVERGED);
  }
  return HZ_OK;
}

template int gmres_run<double>(hz_ctx, const SegHost&, const SellOp<double>&, const z_t*, z_t*,
                               const KrylovCtl&, KrylovOut*, const std::string&);
template int gmres_run<float>(hz_ctx, const SegHost&, const SellOp<float>&, const c_t*, c_t*,
                              const KrylovCtl&, KrylovOut*, const std::string&);
