// Frequency sweep: A(k_c) x_c = f_c for up to 64 wavenumbers at once.
//
// The columns of all frequencies are stored interleaved, element (row, c) at
// row * s + c (s = column count rounded up to a power of two <= 64), so one
// multi-vector product reads the real parts K, M (and M_eta) of a row once
// and applies them to every column with that column's k_c: the matrix is
// read once per s products.  Restarted GMRES(m) runs on all columns in
// lock-step, each with its own FP64 Hessenberg matrix, Givens rotations and
// convergence flag.  Every restart cycle is one step of iterative
// refinement: the residual of the FP64 iterate is formed in FP64, the Arnoldi
// cycle runs on the right-Jacobi operator in the storage precision (complex64
// in mixed mode, with FP64 Gram-Schmidt coefficients and rotations), and the
// correction is added in FP64.  The cycle's kernel sequence is captured once
// in a HIP graph and replayed.  The product's thread layout (columns per lane,
// block size) is chosen by timing the candidates on first use.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <type_traits>

#include "ops.h"
#include "solve.h"

namespace {

constexpr int NV = 8;   // basis vectors per multi-dot chunk

// Rows of the sweep's operator are stored in a spatial brick order (section
// "row-wise operator data"); every block of kHaloRows consecutive rows has
// the list of columns its rows reference (its halo), and every entry the
// position of its column in that list.
constexpr int kHaloRows = 512;

template <typename R>
struct RowOp {
  const int* rowptr;
  const int* col;
  const R* K;
  const R* M;
  const R* E;       // M_eta or nullptr
  const int* bptr;  // boundary entries of each row
  const int* bcol;
  const cx<R>* B;   // sum_w beta_w B0_w
  const int* hptr = nullptr;       // [nblk + 1] halo of each block of kHaloRows rows
  const int* hidx = nullptr;       // halo columns
  const int16_t* lidx = nullptr;   // per entry: position of its column in the block's halo
  const int16_t* blidx = nullptr;  // per boundary entry: the same
  int hblocks = 0, hmax = 0;
  // stencil form (a box in its own numbering, rows x fastest): per row and
  // slot t, KM[27 row + t] = (K, M) of the entry coupling the row with its
  // neighbour (dx, dy, dz), t = 9 (dz + 1) + 3 (dy + 1) + dx + 1, and
  // SE[27 row + t] its M_eta; zero slots for missing neighbours
  const cx<R>* KM = nullptr;
  const R* SE = nullptr;
  // boundary terms in slot form: BSI[row] indexes BSV[27 * BSI[row] + t]
  // (sum_w beta_w B0_w of slot t) for the rows on absorbing walls, -1 else
  const int* BSI = nullptr;
  const cx<R>* BSV = nullptr;
  int bx = 0, by = 0, bz = 0;      // box nodes per direction (0: no stencil form)
};

struct SwCol {
  double k, k2, beta, thr2, est, inv_next, fn2, pad0;
  int kk, done, cyc, nan, iters, cycles;
};

struct SwArr {
  z_t* H;    // [s][(m+1) m]
  double* cs;
  z_t* sn;   // [s][m]
  z_t* g;    // [s][m+1]
  z_t* y;    // [s][m]
  z_t* h1;   // [s][m+1]
  z_t* h2;
  int m;
};

// Sum of v over the threads of this block that hold the same column
// (column = threadIdx.x % s, s a power of two <= 64); valid in threads 0..s-1.
__device__ __forceinline__ double col_reduce(double v, int s, double* lds /*[4*64]*/) {
  for (int o = 32; o >= s; o >>= 1) v += __shfl_xor(v, o, kWave);
  int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (lane < s) lds[w * kWave + lane] = v;
  __syncthreads();
  double t = 0.0;
  if (int(threadIdx.x) < s)
    for (int ww = 0; ww < int(blockDim.x) / kWave; ++ww) t += lds[ww * kWave + threadIdx.x];
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------- product
// Y[row, c] = (A(k_c) Z[:, c])[row]   or, with RESID, Y = F - A X and partial ||Y_c||^2.
// L lanes per row, CPL columns per lane (s = L * CPL); block of blockDim.x threads.
// XCD: block b takes row tile xcd_tile(b) (each XCD a contiguous range, so
// the rows whose neighbours overlap share that XCD's L2) instead of tile b.
// In complex64 the stiffness part is applied in difference form,
// (K z)_i = sum_j K_ij (z_j - z_i), which holds because every row of K sums
// to zero (constants are in its kernel).  For the smooth fields that dominate
// a Krylov solve, sum_j K_ij z_j is a small difference of terms of size
// |K_ii| |z|: accumulated directly in FP32 it loses about log10(1 / (k h)^2)
// digits (2 to 4 here), the difference form keeps the rounding relative to
// the result.  The FP64 products keep the direct form.
template <typename T>
constexpr bool kDiffK = sizeof(T) == 4;

template <typename T, int L, int CPL, bool RESID, bool XCD>
__global__ void __launch_bounds__(512) k_spmm(int64_t nrows, int s, RowOp<T> A, const double* __restrict__ kc,
                                              const cx<T>* __restrict__ Z, const cx<T>* __restrict__ F,
                                              cx<T>* __restrict__ Y, double* __restrict__ part) {
  const int rpb = blockDim.x / L;
  const int ln = int(threadIdx.x) % L;
  const int tile = XCD ? xcd_tile(blockIdx.x, gridDim.x) : int(blockIdx.x);
  int row = tile * rpb + threadIdx.x / L;
  if (L == kWave) row = __builtin_amdgcn_readfirstlane(row);
  double pn = 0.0;
  if (row < nrows) {
    cx<T> aK[CPL], aM[CPL], aE[CPL], zi[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      aK[q] = aM[q] = aE[q] = cx<T>{T(0), T(0)};
      zi[q] = kDiffK<T> ? Z[int64_t(row) * s + ln + L * q] : cx<T>{T(0), T(0)};
    }
    const int q0 = A.rowptr[row], q1 = A.rowptr[row + 1];
    auto term = [&](int64_t j, T kv, T mv, T ev) {
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        cx<T> z = Z[j * s + ln + L * cc];
        aK[cc].re = fma(kv, z.re - zi[cc].re, aK[cc].re);   // K z = sum_j K_ij (z_j - z_i)
        aK[cc].im = fma(kv, z.im - zi[cc].im, aK[cc].im);
        aM[cc].re = fma(mv, z.re, aM[cc].re);
        aM[cc].im = fma(mv, z.im, aM[cc].im);
        aE[cc].re = fma(ev, z.re, aE[cc].re);
        aE[cc].im = fma(ev, z.im, aE[cc].im);
      }
    };
    if constexpr (L >= 8) {
      // The L lanes of a row load its entries cooperatively, L at a time
      // (lane ln takes entry qc + ln), and broadcast them within the row's
      // lanes: the gathers of consecutive entries no longer wait on a
      // dependent index load each.
      for (int qc = q0; qc < q1; qc += L) {
        const int qq = qc + ln;
        int jl = row;
        T kl = T(0), ml = T(0), el = T(0);
        if (qq < q1) {
          jl = A.col[qq];
          kl = A.K[qq];
          ml = A.M[qq];
          if (A.E) el = A.E[qq];
        }
        const int cnt = min(L, q1 - qc);
        for (int t = 0; t < cnt; ++t)
          term(__shfl(jl, t, L), __shfl(kl, t, L), __shfl(ml, t, L), A.E ? __shfl(el, t, L) : T(0));
      }
    } else {
      for (int q = q0; q < q1; ++q) term(A.col[q], A.K[q], A.M[q], A.E ? A.E[q] : T(0));
    }
    const int b0 = A.bptr[row], b1 = A.bptr[row + 1];
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      const int c = ln + L * cc;
      const T k = T(kc[2 * c]), k2 = T(kc[2 * c + 1]);
      // K z - k^2 M z + i k^2 M_eta z
      cx<T> y = {aK[cc].re - k2 * aM[cc].re - k2 * aE[cc].im, aK[cc].im - k2 * aM[cc].im + k2 * aE[cc].re};
      cx<T> bz = {T(0), T(0)};
      for (int q = b0; q < b1; ++q) cfma(bz, A.B[q], Z[int64_t(A.bcol[q]) * s + c]);
      y.re -= k * bz.im;   // + i k (B z)
      y.im += k * bz.re;
      const int64_t e = int64_t(row) * s + c;
      if (RESID) {
        cx<T> r = F[e] - y;
        Y[e] = r;
        pn += double(r.re) * double(r.re) + double(r.im) * double(r.im);
      } else {
        Y[e] = y;
      }
    }
  }
  if (RESID) {
    __shared__ double lds[8 * kWave];
    // with CPL == 1 a thread's column is threadIdx.x % s
    for (int o = 32; o >= s; o >>= 1) pn += __shfl_xor(pn, o, kWave);
    int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (lane < s) lds[w * kWave + lane] = pn;
    __syncthreads();
    if (int(threadIdx.x) < s) {
      double t = 0.0;
      for (int ww = 0; ww < int(blockDim.x) / kWave; ++ww) t += lds[ww * kWave + threadIdx.x];
      part[int64_t(blockIdx.x) * s + threadIdx.x] = t;
    }
  }
}

// The same product (no residual form) with the gathered rows staged in LDS:
// block b computes rows [512 b, 512 b + 512); for each group of CG columns
// it first copies its halo's CG columns of Z into LDS (consecutive threads
// take consecutive columns of a halo row, so the copy is coalesced), then
// every thread forms its row's CG outputs from LDS.  The gathers of a block
// thus read each distinct row of Z once per column group instead of once per
// nonzero.
template <typename T, int CG>
__global__ void __launch_bounds__(kHaloRows) k_spmm_lds(int64_t nrows, int s, RowOp<T> A,
                                                        const double* __restrict__ kc, const cx<T>* __restrict__ Z,
                                                        cx<T>* __restrict__ Y) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* xs = reinterpret_cast<cx<T>*>(smem_raw);
  const int b = blockIdx.x;
  const int h0 = A.hptr[b], hn = A.hptr[b + 1] - h0;
  const int64_t row = int64_t(b) * kHaloRows + threadIdx.x;
  const bool live = row < nrows;
  int q0 = 0, q1 = 0, b0 = 0, b1 = 0;
  if (live) {
    q0 = A.rowptr[row];
    q1 = A.rowptr[row + 1];
    b0 = A.bptr[row];
    b1 = A.bptr[row + 1];
  }
  for (int cg = 0; cg < s; cg += CG) {
    for (int i = threadIdx.x; i < hn * CG; i += kHaloRows) {
      const int64_t node = A.hidx[h0 + i / CG];
      xs[i] = Z[node * s + cg + i % CG];
    }
    __syncthreads();
    if (live) {
      cx<T> aK[CG], aM[CG], aE[CG], zi[CG];
#pragma unroll
      for (int c = 0; c < CG; ++c) {
        aK[c] = aM[c] = aE[c] = cx<T>{T(0), T(0)};
        zi[c] = kDiffK<T> ? Z[row * s + cg + c] : cx<T>{T(0), T(0)};
      }
      for (int q = q0; q < q1; ++q) {
        const int li = A.lidx[q] * CG;
        const T kv = A.K[q], mv = A.M[q];
        const T ev = A.E ? A.E[q] : T(0);
#pragma unroll
        for (int c = 0; c < CG; ++c) {
          const cx<T> z = xs[li + c];
          aK[c].re = fma(kv, z.re - zi[c].re, aK[c].re);
          aK[c].im = fma(kv, z.im - zi[c].im, aK[c].im);
          aM[c].re = fma(mv, z.re, aM[c].re);
          aM[c].im = fma(mv, z.im, aM[c].im);
          aE[c].re = fma(ev, z.re, aE[c].re);
          aE[c].im = fma(ev, z.im, aE[c].im);
        }
      }
#pragma unroll
      for (int c = 0; c < CG; ++c) {
        const int col = cg + c;
        const T k = T(kc[2 * col]), k2 = T(kc[2 * col + 1]);
        cx<T> y = {aK[c].re - k2 * aM[c].re - k2 * aE[c].im, aK[c].im - k2 * aM[c].im + k2 * aE[c].re};
        cx<T> bz = {T(0), T(0)};
        for (int q = b0; q < b1; ++q) cfma(bz, A.B[q], xs[A.blidx[q] * CG + c]);
        y.re -= k * bz.im;
        y.im += k * bz.re;
        Y[row * s + col] = y;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- stencil-form product
// On a box in its own numbering (row = x + bx (y + by z)) the 64-column
// product runs in the stencil form, one wave per (x, y) line with one column
// per lane.  The wave marches along z: at plane p it holds the 9 in-plane
// neighbours of its line (each a contiguous 1 KiB node row of the 64
// columns) and adds them, with the matrix pairs of the three rows they couple
// with, to the partial sums of its rows in planes p + 1, p and p - 1, kept in
// registers; the row in plane p - 1 is then complete and is written.  The 27
// matrix pairs a plane step needs (9 of each row, stored row by row) come in
// with one vector load, lane t holding pair t, and reach every lane by
// readlane; the next plane's neighbours and pairs are loaded while the
// current plane is computed.  Each (K, M) pair and each input row thus
// crosses L2 about once per tile of lines sharing it, and the input is read
// 9 times per row from L1 (27 times in the row-wise product).  Boundary
// terms are stored in the same slot form for the rows that have them.
// Blocks are patches of PW x PH lines (whose waves share neighbours in L1),
// mapped to XCD-contiguous ranges.
struct ZlGeom {
  int npx = 0, npy = 0;    // patches along x and y
  int zc = 0, nzc = 0;     // planes per wave, z chunks
};

__device__ __forceinline__ double lane_bcast(double v, int t) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(b), t));
  const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(b >> 32), t));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}
__device__ __forceinline__ float lane_bcast(float v, int t) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), t));
}

// Everything one plane step reads: the plane's 9 neighbours (this lane's
// column), pair / loss / boundary value of slot t = lane (lanes 0..26), and
// for the difference form the next row's own value.
template <typename T>
struct ZlStep {
  cx<T> zv[9];
  cx<T> km, bv, zn;
  T ev;
};

// LDS: false, the lanes take pair t by readlane (vector instructions);
// true, the wave stores its 27 pairs in LDS and every lane reads pair t at
// the same address (a broadcast read on the LDS pipe).
// R lines per wave (R = 1: 64 columns; R = 2: 32 columns, 32 lanes per
// line, the lines x and x + 1 of a group; pairs through LDS only).
template <typename T, int R, int PW, int PH, bool ETA, bool LDS>
__global__ void __launch_bounds__(PW * PH * kWave)
    k_spmm_zl(int bx, int by, int bz, ZlGeom g, const cx<T>* __restrict__ KM, const T* __restrict__ SE,
              const int* __restrict__ BSI, const cx<T>* __restrict__ BSV, const double* __restrict__ kc,
              const cx<T>* __restrict__ Z, cx<T>* __restrict__ Y) {
  static_assert(R == 1 || LDS, "several lines per wave take their pairs through LDS");
  constexpr int S = kWave / R;    // columns (lanes per line)
  constexpr int NP = R * kStencil;   // pairs of a plane step
  static_assert(NP <= kWave, "one pair per lane");
  constexpr bool DIFF = kDiffK<T>;
  // block -> patch (XCD-contiguous), wave -> line group of the patch
  int L = xcd_tile(blockIdx.x, gridDim.x);
  const int px = L % g.npx;
  L /= g.npx;
  const int py = L % g.npy;
  const int izc = L / g.npy;
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave);
  const int gx = px * PW + w % PW, y = py * PH + w / PW;
  if (gx * R >= bx || y >= by) return;   // whole wave: this kernel has no barrier
  const int z0 = izc * g.zc, z1 = min(z0 + g.zc, bz);
  const int lane = int(threadIdx.x) % kWave;
  const int r = R == 1 ? 0 : lane / S, c = R == 1 ? lane : lane % S;
  const bool live = R == 1 || gx * R + r < bx;
  // a lane past the box's end loads the group's first line (one line: uniform)
  const int x = R == 1 ? gx : (live ? gx * R + r : gx * R);
  const int64_t plane = int64_t(bx) * by;
  const int64_t line = int64_t(x) + int64_t(bx) * y;
  const int64_t line0 = int64_t(gx) * R + int64_t(bx) * y;
  const T k = T(kc[2 * c]), k2 = T(kc[2 * c + 1]);

  // boundary-slot index of this lane's row in plane zr (-1: none or not ours)
  auto bsi_at = [&](int zr) -> int {
    const int v = zr >= z0 && zr < z1 ? BSI[line + plane * zr] : -1;
    return R == 1 ? __builtin_amdgcn_readfirstlane(v) : v;
  };
  // loads of plane step p; bn, bc, bp: boundary indices of rows p + 1, p, p - 1
  auto fetch = [&](int p, int bn, int bc, int bp, ZlStep<T>& st) {
    const int64_t rowp = line + plane * p;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      const int dy = j / 3 - 1, dx = j % 3 - 1;
      const bool in = x + dx >= 0 && x + dx < bx && y + dy >= 0 && y + dy < by;   // wave-uniform for R = 1
      st.zv[j] = in ? Z[(rowp + dx + int64_t(bx) * dy) * S + c] : cx<T>{T(0), T(0)};
    }
    // lane t < NP: slot tt of line rr, for the rows p + 1 (tt < 9, dz = -1), p
    // (dz = 0), p - 1 (dz = +1) of that line
    const int rr = R == 1 ? 0 : lane / kStencil, tt = R == 1 ? lane : lane % kStencil;
    const int o = tt / 9, zr = p + 1 - o;
    const bool ok = lane < NP && (R == 1 || gx * R + rr < bx) && zr >= z0 && zr < z1;
    const int64_t at = (line0 + rr + plane * zr) * kStencil + tt;
    st.km = ok ? KM[at] : cx<T>{T(0), T(0)};
    if (ETA) st.ev = ok ? SE[at] : T(0);
    int bi = o == 0 ? bn : (o == 1 ? bc : bp);
    if (R > 1) {
      // the boundary indices of line rr's rows live in that line's lanes
      const int src = (rr < R ? rr : 0) * S;
      const int sn = __shfl(bn, src, kWave), sc = __shfl(bc, src, kWave), sp = __shfl(bp, src, kWave);
      bi = o == 0 ? sn : (o == 1 ? sc : sp);
    }
    st.bv = ok && bi >= 0 ? BSV[int64_t(bi) * kStencil + tt] : cx<T>{T(0), T(0)};
    if (DIFF) st.zn = p + 1 < z1 ? Z[(rowp + plane) * S + c] : cx<T>{T(0), T(0)};
  };

  // per wave: the plane step's pairs, loss and boundary values (LDS form)
  __shared__ cx<T> kmS[PW * PH][NP], bvS[PW * PH][NP];
  __shared__ T evS[PW * PH][NP];

  // rows in planes p + 1 (0), p (1), p - 1 (2): partial sums and own values
  cx<T> acc[3], accM[3], accE[3], accB[3], zc[3];
#pragma unroll
  for (int o = 0; o < 3; ++o) acc[o] = accM[o] = accE[o] = accB[o] = zc[o] = cx<T>{T(0), T(0)};

  auto write_row = [&](int zr) {
    cx<T> yv;
    if (DIFF) yv = {acc[2].re - k2 * accM[2].re, acc[2].im - k2 * accM[2].im};
    else yv = acc[2];
    if (ETA) {
      yv.re -= k2 * accE[2].im;   // + i k^2 M_eta z
      yv.im += k2 * accE[2].re;
    }
    yv.re -= k * accB[2].im;   // + i k (B z)
    yv.im += k * accB[2].re;
    if (live) Y[(line + plane * zr) * S + c] = yv;
  };

  const int pa = max(z0 - 1, 0), pb = min(z1, bz - 1);
  // boundary indices of rows p - 1, p, p + 1, p + 2 (p: the current step)
  int bq[4] = {bsi_at(pa - 1), bsi_at(pa), bsi_at(pa + 1), bsi_at(pa + 2)};
  ZlStep<T> cur, nxt;
  fetch(pa, bq[2], bq[1], bq[0], cur);
  for (int p = pa; p <= pb; ++p) {
    const int bnew = bsi_at(p + 3);
    if (p < pb) fetch(p + 1, bq[3], bq[2], bq[1], nxt);
    const bool vn = p + 1 >= z0 && p + 1 < z1;   // wave-uniform
    const bool vc = p >= z0 && p < z1;
    const bool vp = p - 1 >= z0 && p - 1 < z1;
    if (DIFF) {
      // the rows' own values, for the stiffness in difference form
      zc[1] = cur.zv[4];
      zc[0] = cur.zn;
    }
    if (LDS && lane < NP) {
      // the same wave writes and then reads these slots: LDS keeps its order
      kmS[w][lane] = cur.km;
      if (ETA) evS[w][lane] = cur.ev;
      bvS[w][lane] = cur.bv;
    }
    // pipelined reads where they measured faster: complex64, or two lines per
    // wave (FP64 with one line per wave keeps 4 waves per SIMD without them)
    if constexpr (LDS && (R > 1 || sizeof(T) == 4)) {
      // LDS form: the matrix part of every row, also of rows outside the
      // chunk (their pairs are zero and their sums are never written), one
      // neighbour row's three pairs per group, two groups in flight: the
      // reads of group j + 2 take their LDS address from an empty asm
      // statement that consumes the sums after group j's FMAs, so group
      // j + 1's reads run under group j's FMAs and the compiler can neither
      // hoist all 27 pairs nor sink the FMAs below them.
      int base = r * kStencil;
      cx<T> kmg[2][3];
      T evg[2][3];
      auto ld = [&](int j, int b) {
#pragma unroll
        for (int o = 0; o < 3; ++o) {
          kmg[b][o] = kmS[w][base + 9 * o + j];
          if (ETA) evg[b][o] = evS[w][base + 9 * o + j];
        }
      };
      ld(0, 0);
      ld(1, 1);
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        const int b = j & 1;
        const cx<T> z = cur.zv[j];
#pragma unroll
        for (int o = 0; o < 3; ++o) {
          const T K = kmg[b][o].re, M = kmg[b][o].im;
          if (DIFF) {
            acc[o].re = fma(K, z.re - zc[o].re, acc[o].re);
            acc[o].im = fma(K, z.im - zc[o].im, acc[o].im);
            accM[o].re = fma(M, z.re, accM[o].re);
            accM[o].im = fma(M, z.im, accM[o].im);
          } else {
            const T a = fma(-k2, M, K);   // K - k^2 M
            acc[o].re = fma(a, z.re, acc[o].re);
            acc[o].im = fma(a, z.im, acc[o].im);
          }
          if (ETA) {
            accE[o].re = fma(evg[b][o], z.re, accE[o].re);
            accE[o].im = fma(evg[b][o], z.im, accE[o].im);
          }
        }
        if (j + 2 < 9) {
          asm volatile(""
                       : "+v"(base)
                       : "v"(acc[0].re), "v"(acc[0].im), "v"(acc[1].re), "v"(acc[1].im), "v"(acc[2].re),
                         "v"(acc[2].im), "v"(accM[0].re), "v"(accM[0].im), "v"(accM[1].re), "v"(accM[1].im),
                         "v"(accM[2].re), "v"(accM[2].im), "v"(accE[0].re), "v"(accE[1].re), "v"(accE[2].re),
                         "v"(accE[0].im), "v"(accE[1].im), "v"(accE[2].im));
          ld(j + 2, b);
        }
      }
      // boundary terms: rows on absorbing walls only
#pragma unroll
      for (int o = 0; o < 3; ++o) {
        const int bi = bq[2 - o];
        const bool v = o == 0 ? vn : (o == 1 ? vc : vp);
        if (v && bi >= 0) {
#pragma unroll
          for (int j = 0; j < 9; ++j) cfma(accB[o], bvS[w][r * kStencil + 9 * o + j], cur.zv[j]);
        }
      }
    } else {
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      const cx<T> z = cur.zv[j];
      auto add = [&](int o, int bi) {
        const int t = 9 * o + j;   // o = 0: dz = -1 for the row in plane p + 1; 1: dz = 0; 2: dz = +1
        T K, M;
        if (LDS) {
          const cx<T> km = kmS[w][r * kStencil + t];
          K = km.re;
          M = km.im;
        } else {
          K = lane_bcast(cur.km.re, t);
          M = lane_bcast(cur.km.im, t);
        }
        if (DIFF) {
          acc[o].re = fma(K, z.re - zc[o].re, acc[o].re);
          acc[o].im = fma(K, z.im - zc[o].im, acc[o].im);
          accM[o].re = fma(M, z.re, accM[o].re);
          accM[o].im = fma(M, z.im, accM[o].im);
        } else {
          const T a = fma(-k2, M, K);   // K - k^2 M
          acc[o].re = fma(a, z.re, acc[o].re);
          acc[o].im = fma(a, z.im, acc[o].im);
        }
        if (ETA) {
          const T E = LDS ? evS[w][r * kStencil + t] : lane_bcast(cur.ev, t);
          accE[o].re = fma(E, z.re, accE[o].re);
          accE[o].im = fma(E, z.im, accE[o].im);
        }
        if (bi >= 0)
          cfma(accB[o], LDS ? bvS[w][r * kStencil + t] : cx<T>{lane_bcast(cur.bv.re, t), lane_bcast(cur.bv.im, t)},
               z);
      };
      if (vn) add(0, bq[2]);
      if (vc) add(1, bq[1]);
      if (vp) add(2, bq[0]);
    }
    }
    if (vp) write_row(p - 1);
    acc[2] = acc[1];
    acc[1] = acc[0];
    acc[0] = cx<T>{T(0), T(0)};
    accM[2] = accM[1];
    accM[1] = accM[0];
    accM[0] = cx<T>{T(0), T(0)};
    accE[2] = accE[1];
    accE[1] = accE[0];
    accE[0] = cx<T>{T(0), T(0)};
    accB[2] = accB[1];
    accB[1] = accB[0];
    accB[0] = cx<T>{T(0), T(0)};
    zc[2] = zc[1];
    bq[0] = bq[1];
    bq[1] = bq[2];
    bq[2] = bq[3];
    bq[3] = bnew;
    cur = nxt;
  }
  // the last plane of the box has no plane after it
  if (pb == bz - 1 && pb >= z0 && pb < z1) write_row(pb);
}

// ---------------------------------------------------------------- vector kernels over [nrows][s]
// X[row, c] = P[perm[row], c] (internal row order <- caller's node order)
__global__ void k_in(int64_t n, int64_t nrows, int s, int nf, const int* __restrict__ perm,
                     const z_t* __restrict__ P, const z_t* __restrict__ F, z_t* __restrict__ X,
                     z_t* __restrict__ Fs) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= nrows * s) return;
  int64_t row = e / s;
  int c = int(e % s);
  bool ok = row < n && c < nf;
  const int64_t node = ok ? perm[row] : 0;
  X[e] = ok ? P[node * nf + c] : z_t{0.0, 0.0};
  Fs[e] = ok ? F[node * nf + c] : z_t{0.0, 0.0};
}

__global__ void k_out(int64_t n, int s, int nf, const int* __restrict__ perm, const z_t* __restrict__ X,
                      z_t* __restrict__ P) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= n * nf) return;
  int64_t row = e / nf;
  int c = int(e % nf);
  P[int64_t(perm[row]) * nf + c] = X[row * s + c];
}

// dinv[row, c] = 1 / A(k_c)_{row,row}
template <typename T>
__global__ void k_diag(int64_t n, int64_t nrows, int s, const int* __restrict__ dpos, const double* __restrict__ K,
                       const double* __restrict__ M, const double* __restrict__ E, const z_t* __restrict__ Bd,
                       const double* __restrict__ kc, z_t* __restrict__ d64, cx<T>* __restrict__ dT) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= nrows * s) return;
  int64_t row = e / s;
  int c = int(e % s);
  z_t inv = {1.0, 0.0};
  if (row < n) {
    int64_t p = dpos[row];
    double k = kc[2 * c], k2 = kc[2 * c + 1];
    z_t b = Bd[row];
    z_t d = {K[p] - k2 * M[p] - k * b.im, k * b.re + (E ? k2 * E[p] : 0.0)};
    inv = crecip(d);
  }
  d64[e] = inv;
  dT[e] = ccast<T>(inv);
}

// partial ||x_c||^2 per block, grid-stride
template <typename T>
__global__ void __launch_bounds__(kBlock) k_colnorm(int64_t total, int s, const cx<T>* __restrict__ x,
                                                    double* __restrict__ part) {
  __shared__ double lds[4 * kWave];
  double v = 0.0;
  for (int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x; e < total; e += int64_t(gridDim.x) * kBlock)
    v += norm2(ccast<double>(x[e]));
  double t = col_reduce(v, s, lds);
  if (int(threadIdx.x) < s) part[int64_t(blockIdx.x) * s + threadIdx.x] = t;
}

// column c: sum of the partials of every block
__global__ void k_colsum(int nblk, int s, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double lds[kBlock / kWave];
  int c = blockIdx.x;
  double t = block_sum_strided(part + c, nblk, s, lds);
  if (threadIdx.x == 0) out[c] = t;
}

__global__ void k_init_cols(int s, SwCol* st, const double* fn2, double tol) {
  int c = threadIdx.x;
  if (c >= s) return;
  st[c].fn2 = fn2[c];
  st[c].thr2 = tol * tol * fn2[c];
  st[c].iters = 0;
  st[c].cycles = 0;
  st[c].done = 0;
  st[c].nan = 0;
}

// beta_c = ||R_c|| -> cycle start; block per column
__global__ void k_beta_fin(int nblk, int s, SwCol* st, SwArr G, const double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  int c = blockIdx.x;
  double rr = block_sum_strided(part + c, nblk, s, lds);
  if (threadIdx.x != 0) return;
  SwCol& S = st[c];
  double b = sqrt(rr);
  S.beta = b;
  S.est = b;
  S.kk = 0;
  S.nan = S.nan || !isfinite(rr);
  S.done = (rr <= S.thr2) || S.fn2 == 0.0 || S.nan;
  S.cyc = S.done;
  S.inv_next = b > 0.0 ? 1.0 / b : 0.0;
  if (!S.done) S.cycles += 1;
  z_t* g = G.g + int64_t(c) * (G.m + 1);
  g[0] = z_t{b, 0.0};
  for (int i = 1; i <= G.m; ++i) g[i] = z_t{0.0, 0.0};
}

// V0 = R / beta (storage precision), Z = dinv V0
template <typename T>
__global__ void k_v0(int64_t total, int s, const SwCol* __restrict__ st, const z_t* __restrict__ R,
                     const cx<T>* __restrict__ dT, cx<T>* __restrict__ V0, cx<T>* __restrict__ Z) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= total) return;
  int c = int(e % s);
  const SwCol& S = st[c];
  cx<T> v = {T(0), T(0)};
  if (!S.cyc) v = ccast<T>(S.inv_next * R[e]);
  V0[e] = v;
  Z[e] = dT[e] * v;
}

// partial h_i[c] = V_i[:, c]^H w[:, c] for i in chunk blockIdx.y
template <typename T>
__global__ void __launch_bounds__(kBlock) k_mdot(int64_t total, int s, const SwCol* __restrict__ st,
                                                 const cx<T>* __restrict__ V, int64_t ld, int j,
                                                 const cx<T>* __restrict__ w, z_t* __restrict__ part) {
  __shared__ double lds[4 * kWave];
  const int c = threadIdx.x % s;
  const int i0 = blockIdx.y * NV;
  const bool act = !st[c].cyc;
  double acc[2 * NV];
#pragma unroll
  for (int q = 0; q < 2 * NV; ++q) acc[q] = 0.0;
  if (act) {
    for (int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x; e < total; e += int64_t(gridDim.x) * kBlock) {
      z_t wv = ccast<double>(w[e]);
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        int i = i0 + q;
        if (i <= j) {
          z_t a = ccast<double>(V[int64_t(i) * ld + e]);
          acc[2 * q] = fma(a.re, wv.re, fma(a.im, wv.im, acc[2 * q]));
          acc[2 * q + 1] = fma(a.re, wv.im, fma(-a.im, wv.re, acc[2 * q + 1]));
        }
      }
    }
  }
  z_t* out = part + (int64_t(blockIdx.y) * gridDim.x + blockIdx.x) * NV * s;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double re = col_reduce(acc[2 * q], s, lds);
    double im = col_reduce(acc[2 * q + 1], s, lds);
    if (int(threadIdx.x) < s) out[q * s + threadIdx.x] = z_t{re, im};
  }
}

// block (c, i): coefficient i of column c.  pass 1 -> h1; pass 2 -> h2, H[:, j] = h1 + h2
__global__ void k_mdot_fin(int G_, int s, const SwCol* __restrict__ st, SwArr A, const z_t* __restrict__ part,
                           int j, int pass) {
  __shared__ double lds[kBlock / kWave];
  int c = blockIdx.x, i = blockIdx.y;
  if (st[c].cyc) return;
  int ch = i / NV, q = i % NV;
  const double* base = reinterpret_cast<const double*>(part + (int64_t(ch) * G_ * NV + q) * s + c);
  double re = block_sum_strided(base, G_, 2 * NV * s, lds);
  double im = block_sum_strided(base + 1, G_, 2 * NV * s, lds);
  if (threadIdx.x == 0) {
    z_t h = {re, im};
    if (pass == 1) {
      A.h1[int64_t(c) * (A.m + 1) + i] = h;
    } else {
      A.h2[int64_t(c) * (A.m + 1) + i] = h;
      A.H[int64_t(c) * (A.m + 1) * A.m + int64_t(j) * (A.m + 1) + i] = A.h1[int64_t(c) * (A.m + 1) + i] + h;
    }
  }
}

// w -= sum_i h_i V_i per column; NORM: partial ||w_c||^2
template <typename T, bool NORM>
__global__ void __launch_bounds__(kBlock) k_axpy(int64_t total, int s, const SwCol* __restrict__ st, SwArr A,
                                                 const cx<T>* __restrict__ V, int64_t ld, int j, int pass,
                                                 cx<T>* __restrict__ w, double* __restrict__ part) {
  __shared__ double lds[4 * kWave];
  const int c = threadIdx.x % s;
  const bool act = !st[c].cyc;
  const z_t* h = (pass == 1 ? A.h1 : A.h2) + int64_t(c) * (A.m + 1);
  double nn = 0.0;
  if (act) {
    for (int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x; e < total; e += int64_t(gridDim.x) * kBlock) {
      z_t acc = ccast<double>(w[e]);
      for (int i = 0; i <= j; ++i) {
        z_t v = ccast<double>(V[int64_t(i) * ld + e]);
        z_t hi = h[i];
        acc.re -= hi.re * v.re - hi.im * v.im;
        acc.im -= hi.re * v.im + hi.im * v.re;
      }
      cx<T> ws = ccast<T>(acc);
      w[e] = ws;
      if (NORM) nn += norm2(ccast<double>(ws));
    }
  }
  if (NORM) {
    double t = col_reduce(nn, s, lds);
    if (int(threadIdx.x) < s) part[int64_t(blockIdx.x) * s + threadIdx.x] = t;
  }
}

// block per column: subdiagonal, rotations, residual estimate
__global__ void k_givens_fin(int G_, int s, SwCol* st, SwArr A, const double* __restrict__ part, int j,
                             double inner_tol) {
  __shared__ double lds[kBlock / kWave];
  int c = blockIdx.x;
  const int cyc = st[c].cyc;
  __syncthreads();
  if (cyc) return;
  double ww = block_sum_strided(part + c, G_, s, lds);
  if (threadIdx.x != 0) return;
  SwCol& S = st[c];
  const int m = A.m;
  z_t* H = A.H + int64_t(c) * (m + 1) * m + int64_t(j) * (m + 1);
  double* cs = A.cs + int64_t(c) * m;
  z_t* sn = A.sn + int64_t(c) * m;
  z_t* g = A.g + int64_t(c) * (m + 1);
  double hn = sqrt(ww);
  H[j + 1] = z_t{hn, 0.0};
  for (int i = 0; i < j; ++i) {
    z_t a = H[i], b = H[i + 1];
    H[i] = cs[i] * a + sn[i] * b;
    H[i + 1] = (-1.0 * (conj(sn[i]) * a)) + cs[i] * b;
  }
  z_t a = H[j], b = H[j + 1];
  double rho = sqrt(norm2(a) + norm2(b));
  double cc;
  z_t sv;
  if (rho == 0.0) {
    cc = 1.0;
    sv = z_t{0.0, 0.0};
  } else if (norm2(a) == 0.0) {
    cc = 0.0;
    sv = z_t{1.0, 0.0};
  } else {
    double aa = sqrt(norm2(a));
    cc = aa / rho;
    sv = (1.0 / (aa * rho)) * (a * conj(b));
  }
  cs[j] = cc;
  sn[j] = sv;
  H[j] = cc * a + sv * b;
  H[j + 1] = z_t{0.0, 0.0};
  z_t gj = g[j];
  g[j + 1] = -1.0 * (conj(sv) * gj);
  g[j] = cc * gj;
  S.kk = j + 1;
  S.iters += 1;
  S.est = sqrt(norm2(g[j + 1]));
  bool bad = !isfinite(hn) || !isfinite(S.est);
  if (bad) S.nan = 1;
  double lim = inner_tol * S.beta;
  if (bad || hn == 0.0 || S.est * S.est <= S.thr2 || S.est <= lim) S.cyc = 1;
  S.inv_next = hn > 0.0 ? 1.0 / hn : 0.0;
}

// V_{j+1} = w / h, Z = dinv V_{j+1}
template <typename T>
__global__ void k_scale(int64_t total, int s, const SwCol* __restrict__ st, const cx<T>* __restrict__ dT,
                        cx<T>* __restrict__ w, cx<T>* __restrict__ Z) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= total) return;
  int c = int(e % s);
  const SwCol& S = st[c];
  if (S.cyc) return;
  cx<T> v = ccast<T>(S.inv_next * ccast<double>(w[e]));
  w[e] = v;
  Z[e] = dT[e] * v;
}

__global__ void k_solve_y(int s, const SwCol* __restrict__ st, SwArr A) {
  int c = threadIdx.x;
  if (c >= s) return;
  const SwCol& S = st[c];
  if (S.done || S.nan) return;
  const int m = A.m, k = S.kk;
  const z_t* H = A.H + int64_t(c) * (m + 1) * m;
  const z_t* g = A.g + int64_t(c) * (m + 1);
  z_t* y = A.y + int64_t(c) * m;
  for (int i = k - 1; i >= 0; --i) {
    z_t acc = g[i];
    for (int l = i + 1; l < k; ++l) acc = acc - H[int64_t(l) * (m + 1) + i] * y[l];
    y[i] = cdiv(acc, H[int64_t(i) * (m + 1) + i]);
  }
}

// X += dinv (V y)   (FP64)
template <typename T>
__global__ void k_update(int64_t total, int s, const SwCol* __restrict__ st, SwArr A, const cx<T>* __restrict__ V,
                         int64_t ld, const z_t* __restrict__ d64, z_t* __restrict__ X) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= total) return;
  int c = int(e % s);
  const SwCol& S = st[c];
  if (S.done || S.nan || S.kk == 0) return;
  const z_t* y = A.y + int64_t(c) * A.m;
  z_t acc = {0.0, 0.0};
  for (int i = 0; i < S.kk; ++i) {
    z_t v = ccast<double>(V[int64_t(i) * ld + e]);
    cfma(acc, y[i], v);
  }
  z_t dx = d64[e] * acc;
  X[e] = X[e] + dx;
}

// ---------------------------------------------------------------- batched BiCGStab
// Per-column state.  Each column runs its own BiCGStab on the correction
// equation A(k_c) d = R / scale (right Jacobi); when its inner stopping test
// fires (idone) the host runs that column's refinement step: X += scale * u,
// R = F - A X in FP64, then either a restart (FP64 storage) or, in complex64
// storage, a reliable update that replaces the recursive residual by the true
// one and keeps the Krylov recurrence (Sleijpen and van der Vorst's reliable
// updates).  Other columns keep iterating meanwhile.
// At the product cap: every column still inside an inner solve ends it, so
// that one more refinement step adds the correction reached so far to X and
// measures the column's FP64 residual (a capped column reports the residual
// of its best iterate, never that of x0).
template <typename C>
__global__ void k_end_inner(int s, C* st) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= s) return;
  C& S = st[c];
  if (!S.done && !S.nan && !S.idone) S.idone = 1;
}

struct BcCol {
  double k, k2, fn2, thr2, scale, ithr2, rr, ss, rhat2, beta;
  z_t rho, rho_old, alpha, omega;
  int done, idone, early, reset, nan, iters, outer, restart_now, full_next, pad;
};

template <typename T>
struct BcVec {
  cx<T>* r;
  cx<T>* rhat;
  cx<T>* p;
  cx<T>* v;
  cx<T>* s;
  cx<T>* t;
  cx<T>* zp;   // dinv p (input of the product)
  cx<T>* zs;   // dinv s
  cx<T>* u;    // correction since the last refinement step (unscaled)
  const cx<T>* dT;
};

__device__ __forceinline__ bool bc_off(const BcCol& S) { return S.done || S.idone || S.nan; }
__device__ __forceinline__ bool bc_pending(const BcCol& S) { return S.idone && !S.done && !S.nan; }

// refinement step, part 1: X += scale u for columns whose inner solve ended
template <typename T>
__global__ void k_bc_update(int64_t total, int s, const BcCol* __restrict__ st, const cx<T>* __restrict__ u,
                            z_t* __restrict__ X) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= total) return;
  const BcCol& S = st[e % s];
  if (!bc_pending(S) || S.scale == 0.0) return;
  z_t d = ccast<double>(u[e]);
  X[e] = z_t{fma(S.scale, d.re, X[e].re), fma(S.scale, d.im, X[e].im)};
}

// part 2 (block per column, after the FP64 residual): convergence, restart kind
// delta: the inner solve of a step stops when the recursive residual has
// dropped by this factor below the last true one (0: run to the target).
__global__ void k_bc_beta(int nblk, int s, BcCol* st, const double* __restrict__ part, double tol,
                          double delta) {
  __shared__ double lds[kBlock / kWave];
  int c = blockIdx.x;
  const int pend = bc_pending(st[c]);
  __syncthreads();
  if (!pend) return;
  double rr = block_sum_strided(part + c, nblk, s, lds);
  if (threadIdx.x != 0) return;
  BcCol& S = st[c];
  double b = sqrt(rr);
  S.beta = b;
  S.nan = S.nan || !isfinite(rr);
  S.done = (rr <= S.thr2) || S.fn2 == 0.0 || S.nan;
  S.early = 0;
  S.reset = 0;
  if (S.done) return;
  S.outer += 1;
  S.idone = 0;
  if (S.scale > 0.0 && !S.full_next) {
    S.restart_now = 2;                 // reliable update: replace r, keep the recurrence
  } else {
    S.restart_now = 1;                 // fresh start on R / beta
    S.scale = b;
  }
  const double rel = b / S.scale;      // true residual in the scaled system
  const double lim = 0.5 * tol * sqrt(S.fn2) / S.scale;
  const double it = delta * rel > lim ? delta * rel : lim;
  S.ithr2 = it * it;
  S.full_next = 0;
}

template <typename T>
__global__ void k_bc_start(int64_t total, int s, const BcCol* __restrict__ st, const z_t* __restrict__ R,
                           BcVec<T> W) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= total) return;
  const BcCol& S = st[e % s];
  if (!S.restart_now) return;
  cx<T> r = ccast<T>((1.0 / S.scale) * R[e]);
  const cx<T> z = {T(0), T(0)};
  W.r[e] = r;
  W.u[e] = z;
  if (S.restart_now == 1) {
    W.rhat[e] = r;
    W.p[e] = z;
    W.v[e] = z;
  }
}

// partial column dots over [total], three quantities per column:
// NQ == 1: (-, -, |b|^2); NQ == 2: (a^H b, -); NQ == 3: (a^H b, |a|^2); NQ == 4: (a^H b, |b|^2).
// RS: only columns with a pending restart (otherwise: active columns).
template <typename T, int NQ, bool RS>
__global__ void __launch_bounds__(kBlock) k_bc_dots(int64_t total, int s, const BcCol* __restrict__ st,
                                                    const cx<T>* __restrict__ a, const cx<T>* __restrict__ b,
                                                    double* __restrict__ part) {
  __shared__ double lds[4 * kWave];
  const int c = threadIdx.x % s;
  double q[3] = {0.0, 0.0, 0.0};
  const bool on = RS ? st[c].restart_now != 0 : !bc_off(st[c]);
  if (on) {
    for (int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x; e < total; e += int64_t(gridDim.x) * kBlock) {
      z_t y = ccast<double>(b[e]);
      if (NQ == 1) {
        q[2] += norm2(y);
      } else {
        z_t x = ccast<double>(a[e]);
        q[0] = fma(x.re, y.re, fma(x.im, y.im, q[0]));
        q[1] = fma(x.re, y.im, fma(-x.im, y.re, q[1]));
        if (NQ == 3) q[2] += norm2(x);
        if (NQ == 4) q[2] += norm2(y);
      }
    }
  }
  for (int i = 0; i < 3; ++i) {
    double t = col_reduce(q[i], s, lds);
    if (int(threadIdx.x) < s) part[(int64_t(blockIdx.x) * 3 + i) * s + threadIdx.x] = t;
  }
}

// finalize kernels: block per column
__device__ __forceinline__ double bc_sum(int G_, int s, const double* part, int c, int i, double* lds) {
  return block_sum_strided(part + int64_t(i) * s + c, G_, 3 * s, lds);
}

// after a restart (kind 1: rho = ||r||^2) or a reliable update (kind 2: rho = rhat^H r)
__global__ void k_bc_rho0(int G_, int s, BcCol* st, const double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  int c = blockIdx.x;
  const int kind = st[c].restart_now;
  __syncthreads();
  if (!kind) return;
  double re = bc_sum(G_, s, part, c, 0, lds);
  double im = bc_sum(G_, s, part, c, 1, lds);
  double rr = bc_sum(G_, s, part, c, 2, lds);
  if (threadIdx.x != 0) return;
  BcCol& S = st[c];
  S.rr = rr;
  if (kind == 1) {
    S.rho = z_t{rr, 0.0};
    S.rho_old = S.alpha = S.omega = z_t{1.0, 0.0};
    S.rhat2 = rr;
  } else {
    S.rho = z_t{re, im};
  }
  S.restart_now = 0;
  S.idone = (rr == 0.0);
}

// p = r + beta (p - omega v); zp = dinv p
template <typename T>
__global__ void k_bc_p(int64_t total, int s, const BcCol* __restrict__ st, BcVec<T> W) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= total) return;
  const BcCol& S = st[e % s];
  if (bc_off(S)) return;
  cx<T> p;
  if (S.reset) {
    p = W.r[e];
    W.rhat[e] = p;
  } else {
    z_t bt = cdiv(S.rho, S.rho_old) * cdiv(S.alpha, S.omega);
    z_t pv = ccast<double>(W.p[e]) - S.omega * ccast<double>(W.v[e]);
    p = ccast<T>(ccast<double>(W.r[e]) + bt * pv);
  }
  W.p[e] = p;
  W.zp[e] = W.dT[e] * p;
}

__global__ void k_bc_alpha(int G_, int s, BcCol* st, const double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  int c = blockIdx.x;
  const int off = bc_off(st[c]);
  __syncthreads();
  if (off) return;
  double re = bc_sum(G_, s, part, c, 0, lds);
  double im = bc_sum(G_, s, part, c, 1, lds);
  if (threadIdx.x != 0) return;
  BcCol& S = st[c];
  S.reset = 0;
  z_t rv = {re, im};
  if (norm2(rv) == 0.0 || !isfinite(re) || !isfinite(im)) {
    S.alpha = z_t{0.0, 0.0};
    S.reset = 1;
  } else {
    S.alpha = cdiv(S.rho, rv);
  }
}

// s = r - alpha v; zs = dinv s; partial ||s||^2
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bc_s(int64_t total, int s, const BcCol* __restrict__ st, BcVec<T> W,
                                                 double* __restrict__ part) {
  __shared__ double lds[4 * kWave];
  const int c = threadIdx.x % s;
  const BcCol& S = st[c];
  double nn = 0.0;
  if (!bc_off(S)) {
    for (int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x; e < total; e += int64_t(gridDim.x) * kBlock) {
      cx<T> sv = ccast<T>(ccast<double>(W.r[e]) - S.alpha * ccast<double>(W.v[e]));
      W.s[e] = sv;
      W.zs[e] = W.dT[e] * sv;
      nn += norm2(ccast<double>(sv));
    }
  }
  double t = col_reduce(nn, s, lds);
  if (int(threadIdx.x) < s) part[(int64_t(blockIdx.x) * 3 + 2) * s + threadIdx.x] = t;
}

__global__ void k_bc_sfin(int G_, int s, BcCol* st, const double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  int c = blockIdx.x;
  const int off = bc_off(st[c]);
  __syncthreads();
  if (off) return;
  double ss = bc_sum(G_, s, part, c, 2, lds);
  if (threadIdx.x != 0) return;
  st[c].ss = ss;
  st[c].early = ss <= st[c].ithr2 ? 1 : 0;
}

__global__ void k_bc_omega(int G_, int s, BcCol* st, const double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  int c = blockIdx.x;
  const int off = bc_off(st[c]) || st[c].early;
  __syncthreads();
  if (off) return;
  double re = bc_sum(G_, s, part, c, 0, lds);
  double im = bc_sum(G_, s, part, c, 1, lds);
  double tt = bc_sum(G_, s, part, c, 2, lds);
  if (threadIdx.x == 0) st[c].omega = tt > 0.0 ? z_t{re / tt, im / tt} : z_t{0.0, 0.0};
}

// u += alpha zp + omega zs; r = s - omega t; partials rhat^H r, ||r||^2
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bc_xr(int64_t total, int s, const BcCol* __restrict__ st, BcVec<T> W,
                                                  double* __restrict__ part) {
  __shared__ double lds[4 * kWave];
  const int c = threadIdx.x % s;
  const BcCol& S = st[c];
  double q[3] = {0.0, 0.0, 0.0};
  if (!bc_off(S)) {
    for (int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x; e < total; e += int64_t(gridDim.x) * kBlock) {
      z_t u = ccast<double>(W.u[e]) + S.alpha * ccast<double>(W.zp[e]);
      if (S.early) {
        W.u[e] = ccast<T>(u);
        continue;
      }
      z_t sv = ccast<double>(W.s[e]);
      W.u[e] = ccast<T>(u + S.omega * ccast<double>(W.zs[e]));
      cx<T> r = ccast<T>(sv - S.omega * ccast<double>(W.t[e]));
      W.r[e] = r;
      z_t a = ccast<double>(W.rhat[e]), b = ccast<double>(r);
      q[0] = fma(a.re, b.re, fma(a.im, b.im, q[0]));
      q[1] = fma(a.re, b.im, fma(-a.im, b.re, q[1]));
      q[2] += norm2(b);
    }
  }
  for (int i = 0; i < 3; ++i) {
    double t = col_reduce(q[i], s, lds);
    if (int(threadIdx.x) < s) part[(int64_t(blockIdx.x) * 3 + i) * s + threadIdx.x] = t;
  }
}

__global__ void k_bc_rho(int G_, int s, BcCol* st, const double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  int c = blockIdx.x;
  BcCol& S = st[c];
  const int off = bc_off(S), early = S.early;
  __syncthreads();
  if (off) return;
  if (early) {
    if (threadIdx.x == 0) {
      S.iters += 1;
      S.rr = S.ss;
      S.idone = 1;
      S.early = 0;
      S.full_next = 1;   // the recurrence stopped half-way: restart it
    }
    return;
  }
  double re = bc_sum(G_, s, part, c, 0, lds);
  double im = bc_sum(G_, s, part, c, 1, lds);
  double rr = bc_sum(G_, s, part, c, 2, lds);
  if (threadIdx.x != 0) return;
  S.iters += 1;
  S.rho_old = S.rho;
  S.rho = z_t{re, im};
  S.rr = rr;
  if (!isfinite(rr) || !isfinite(re) || !isfinite(im)) {
    S.nan = 1;
  } else if (rr <= S.ithr2) {
    S.idone = 1;
  } else if (sqrt(norm2(S.rho)) < 1e-300 * sqrt(S.rhat2 * rr) || norm2(S.omega) == 0.0) {
    S.reset = 1;
    S.rho = z_t{rr, 0.0};
    S.rho_old = S.alpha = S.omega = z_t{1.0, 0.0};
    S.rhat2 = rr;
  }
}

__global__ void k_bc_init_cols(int s, BcCol* st, const double* fn2, double tol) {
  int c = threadIdx.x;
  if (c >= s) return;
  st[c].fn2 = fn2[c];
  st[c].thr2 = tol * tol * fn2[c];
  st[c].idone = 1;          // every column starts with a refinement step
  st[c].full_next = 1;
}

// compaction: out[row, j] = in[row, map[j]] (j < ns_new; map[j] < 0: zero)
template <typename V>
__global__ void k_gather_cols(int64_t nrows, int s_old, int s_new, const int* __restrict__ map,
                              const V* __restrict__ in, V* __restrict__ out) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= nrows * s_new) return;
  int64_t row = e / s_new;
  int j = int(e % s_new);
  int c = map[j];
  out[e] = c >= 0 ? in[row * s_old + c] : V{0, 0};
}

// P[perm[row], orig] = X[row, c] for the listed (c, orig) pairs
__global__ void k_out_cols(int64_t n, int s, int nf, int ncols, const int* __restrict__ perm,
                           const int* __restrict__ cols, const int* __restrict__ orig, const z_t* __restrict__ X,
                           z_t* __restrict__ P) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= n * ncols) return;
  int64_t row = e / ncols;
  int j = int(e % ncols);
  P[int64_t(perm[row]) * nf + orig[j]] = X[row * s + cols[j]];
}

// ---------------------------------------------------------------- dispatch of product variants
struct Variant {
  int cpl = 1, bs = 256, xcd = 0;
  int lds = 0;          // > 0: LDS-staged product with lds columns per group
  // zl > 0: stencil-form product, blocks of pw x ph lines, nzc z chunks,
  // pairs broadcast by readlane (bc 0) or through LDS (bc 1)
  int zl = 0, pw = 0, ph = 0, nzc = 0, bc = 0;
};

// LDS bytes the staged product needs for a column group of cg columns.
template <typename T>
size_t lds_bytes(const RowOp<T>& A, int cg) { return size_t(A.hmax) * cg * sizeof(cx<T>); }

// LDS a workgroup may allocate on the current device (160 KB on gfx950).
size_t lds_limit() {
  static size_t lim = 0;
  if (!lim) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      v = 64 * 1024;
    lim = size_t(v);
  }
  return lim;
}

template <typename T, int CG>
int launch_lds(hipStream_t stream, int64_t nrows, int s, const RowOp<T>& A, const double* kc, const cx<T>* Z,
               cx<T>* Y) {
  const size_t sh = lds_bytes(A, CG);
  if (sh > 64 * 1024)
    HZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spmm_lds<T, CG>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(sh)));
  k_spmm_lds<T, CG><<<A.hblocks, kHaloRows, sh, stream>>>(nrows, s, A, kc, Z, Y);
  HZ_HIP(hipGetLastError());
  return HZ_OK;
}

// Stencil-form variants: patches of pw x ph line groups (pw ph waves per block).
struct ZlShape {
  int pw, ph;
};
constexpr ZlShape kZlShapes[] = {{1, 1}, {2, 1}, {2, 2}, {4, 2}};

inline ZlGeom zl_geom(int bx, int by, int bz, int R, int pw, int ph, int nzc) {
  ZlGeom g;
  g.npx = ceil_div(ceil_div(bx, R), pw);
  g.npy = ceil_div(by, ph);
  g.nzc = std::max(1, std::min(nzc, bz));
  g.zc = ceil_div(bz, g.nzc);
  g.nzc = ceil_div(bz, g.zc);
  return g;
}

template <typename T>
bool zl_fits(const Variant& v, int s, const RowOp<T>& A) {
  if (v.zl <= 0 || !A.KM || !A.BSI || A.bx <= 0 || v.nzc < 1 || v.bc < 0 || v.bc > 1) return false;
  // 64 columns (one line per wave), or 32 (two lines per wave, pairs through LDS)
  if (!(s == kWave || (s == kWave / 2 && v.bc == 1))) return false;
  bool known = false;
  for (const ZlShape& h : kZlShapes) known |= h.pw == v.pw && h.ph == v.ph;
  return known;
}

// Y[e] = 0 for the e < count given (the padding rows the stencil form does
// not compute; the sweep's vector kernels run over them).  A kernel, not a
// memset: the sweep's loops are captured in HIP graphs.
template <typename T>
__global__ void k_zero_tail(int64_t count, cx<T>* __restrict__ Y) {
  const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e < count) Y[e] = cx<T>{T(0), T(0)};
}

template <typename T, int R, int PW, int PH>
int launch_zl(hipStream_t stream, const Variant& v, int64_t nrows, int s, const RowOp<T>& A, const double* kc,
              const cx<T>* Z, cx<T>* Y) {
  if (s * R != kWave) return hz_fail(HZ_ERR_INVALID, "stencil product for %d columns", s);
  const int64_t n = int64_t(A.bx) * A.by * A.bz;
  if (nrows > n) {
    const int64_t tail = (nrows - n) * s;
    k_zero_tail<T><<<ceil_div(tail, kBlock), kBlock, 0, stream>>>(tail, Y + n * s);
    HZ_HIP(hipGetLastError());
  }
  const ZlGeom g = zl_geom(A.bx, A.by, A.bz, R, PW, PH, v.nzc);
  const int64_t nblk = int64_t(g.npx) * g.npy * g.nzc;
  if (nblk > INT32_MAX) return hz_fail(HZ_ERR_INVALID, "stencil product grid too large");
  const dim3 grid = dim3(unsigned(nblk)), block = dim3(PW * PH * kWave);
  if constexpr (R > 1) {
    if (!v.bc) return hz_fail(HZ_ERR_INVALID, "two lines per wave take their pairs through LDS");
    if (A.SE) k_spmm_zl<T, R, PW, PH, true, true><<<grid, block, 0, stream>>>(A.bx, A.by, A.bz, g, A.KM, A.SE,
                                                                              A.BSI, A.BSV, kc, Z, Y);
    else k_spmm_zl<T, R, PW, PH, false, true><<<grid, block, 0, stream>>>(A.bx, A.by, A.bz, g, A.KM, nullptr,
                                                                          A.BSI, A.BSV, kc, Z, Y);
  } else if (A.SE) {
    if (v.bc) k_spmm_zl<T, 1, PW, PH, true, true><<<grid, block, 0, stream>>>(A.bx, A.by, A.bz, g, A.KM, A.SE,
                                                                              A.BSI, A.BSV, kc, Z, Y);
    else k_spmm_zl<T, 1, PW, PH, true, false><<<grid, block, 0, stream>>>(A.bx, A.by, A.bz, g, A.KM, A.SE, A.BSI,
                                                                          A.BSV, kc, Z, Y);
  } else {
    if (v.bc) k_spmm_zl<T, 1, PW, PH, false, true><<<grid, block, 0, stream>>>(A.bx, A.by, A.bz, g, A.KM, nullptr,
                                                                               A.BSI, A.BSV, kc, Z, Y);
    else k_spmm_zl<T, 1, PW, PH, false, false><<<grid, block, 0, stream>>>(A.bx, A.by, A.bz, g, A.KM, nullptr,
                                                                           A.BSI, A.BSV, kc, Z, Y);
  }
  HZ_HIP(hipGetLastError());
  return HZ_OK;
}

template <typename T, bool RESID>
int launch_spmm(hipStream_t stream, const Variant& v, int64_t nrows, int s, const RowOp<T>& A, const double* st,
                const cx<T>* Z, const cx<T>* F, cx<T>* Y, double* part, int* nblk_out) {
  if (!RESID && v.zl > 0) {
    if (!zl_fits<T>(v, s, A)) return hz_fail(HZ_ERR_INVALID, "bad stencil product variant");
    auto go = [&](auto Rc) -> int {
      constexpr int R = decltype(Rc)::value;
      if (v.pw == 1 && v.ph == 1) return launch_zl<T, R, 1, 1>(stream, v, nrows, s, A, st, Z, Y);
      if (v.pw == 2 && v.ph == 1) return launch_zl<T, R, 2, 1>(stream, v, nrows, s, A, st, Z, Y);
      if (v.pw == 2 && v.ph == 2) return launch_zl<T, R, 2, 2>(stream, v, nrows, s, A, st, Z, Y);
      if (v.pw == 4 && v.ph == 2) return launch_zl<T, R, 4, 2>(stream, v, nrows, s, A, st, Z, Y);
      return hz_fail(HZ_ERR_INVALID, "no stencil product variant");
    };
    return s == kWave ? go(std::integral_constant<int, 1>{}) : go(std::integral_constant<int, 2>{});
  }
  if (!RESID && v.lds > 0) {
    if (A.hblocks <= 0 || s % v.lds || lds_bytes(A, v.lds) > lds_limit())
      return hz_fail(HZ_ERR_INVALID, "bad staged product variant");
    switch (v.lds) {
      case 1: return launch_lds<T, 1>(stream, nrows, s, A, st, Z, Y);
      case 2: return launch_lds<T, 2>(stream, nrows, s, A, st, Z, Y);
      case 4: return launch_lds<T, 4>(stream, nrows, s, A, st, Z, Y);
      case 8: return launch_lds<T, 8>(stream, nrows, s, A, st, Z, Y);
      case 16: return launch_lds<T, 16>(stream, nrows, s, A, st, Z, Y);
      default: return hz_fail(HZ_ERR_INVALID, "no staged product for %d columns per group", v.lds);
    }
  }
  const int L = s / v.cpl;
  const int rpb = v.bs / L;
  const int nblk = int((nrows + rpb - 1) / rpb);
  if (nblk_out) *nblk_out = nblk;
  const dim3 grid(nblk);
#define HZ_SPMM_CASE(LL, CC)                                                                               \
  if (L == LL && v.cpl == CC) {                                                                             \
    if (v.xcd) k_spmm<T, LL, CC, RESID, true><<<grid, v.bs, 0, stream>>>(nrows, s, A, st, Z, F, Y, part);   \
    else k_spmm<T, LL, CC, RESID, false><<<grid, v.bs, 0, stream>>>(nrows, s, A, st, Z, F, Y, part);        \
    HZ_HIP(hipGetLastError());                                                                              \
    return HZ_OK;                                                                                           \
  }
  HZ_SPMM_CASE(1, 1) HZ_SPMM_CASE(2, 1) HZ_SPMM_CASE(4, 1) HZ_SPMM_CASE(8, 1) HZ_SPMM_CASE(16, 1)
  HZ_SPMM_CASE(32, 1) HZ_SPMM_CASE(64, 1)
  if (!RESID) {
    HZ_SPMM_CASE(1, 2) HZ_SPMM_CASE(2, 2) HZ_SPMM_CASE(4, 2) HZ_SPMM_CASE(8, 2) HZ_SPMM_CASE(16, 2)
    HZ_SPMM_CASE(32, 2)
  }
#undef HZ_SPMM_CASE
  return hz_fail(HZ_ERR_INVALID, "no product variant for s=%d cpl=%d", s, v.cpl);
}

// ---------------------------------------------------------------- row-wise operator data
struct SweepData {
  int64_t nrows = 0;
  DevBuf rowptr, col, K64, M64, E64, K32, M32, E32, bptr, bcol, B64, B32, Bdiag, dpos;
  DevBuf perm;                      // sweep row -> the caller's node id
  DevBuf hptr, hidx, lidx, blidx;   // halos of the blocks of kHaloRows rows
  int hblocks = 0, hmax = 0;
  bool eta = false;
  // stencil form (boxes in their own numbering): (K, M) pairs and M_eta, 27 slots per row
  DevBuf KM64, KM32, SE64, SE32, BSI, BSV64, BSV32;
  int box[3] = {0, 0, 0};
  int64_t n = 0, nnz = 0, nb = 0;   // mesh nodes, stored entries, boundary entries
};

// Algorithmic bytes of one multi-vector product over s columns in variant
// v: the operator's values (K, M, with M_eta when present; column indices
// and row pointers for the row-wise forms, none for the stencil form, whose
// zero slots are not counted), the boundary lists, one read of the input
// and one write of the output.
int64_t spmm_bytes(const Variant& v, const SweepData& D, int s, int tsize) {
  const int64_t n = D.n, vals = (D.eta ? 3 : 2) * int64_t(tsize) * D.nnz;
  // row-wise: row pointers, columns and values of the boundary lists;
  // stencil form: the per-row slot index and the listed values
  const int64_t bnd = v.zl > 0 ? 4 * n + 2 * int64_t(tsize) * D.nb : 4 * (n + 1) + (4 + 2 * int64_t(tsize)) * D.nb;
  const int64_t vec = 2 * 2 * int64_t(tsize) * n * s;
  const int64_t idx = v.zl > 0 ? 0 : 4 * D.nnz + 4 * (n + 1);
  return vals + idx + bnd + vec;
}

template <typename V>
int upload(DevBuf& b, const std::vector<V>& h) {
  HZ_TRY(b.ensure(sizeof(V) * std::max<size_t>(h.size(), 1)));
  if (!h.empty()) HZ_HIP(hipMemcpy(b.p, h.data(), sizeof(V) * h.size(), hipMemcpyHostToDevice));
  return HZ_OK;
}

// Spatial brick order of the nodes: bricks of about 8 x 8 x 8 node spacings
// (brick index from the coordinates, z slowest), nodes inside a brick by
// (z, y, x).  Consecutive rows then cover compact boxes of space, so a block
// of 512 rows references about 2 x 512 distinct columns instead of the
// ~27 x 512 of a row range in the natural order, which is what lets the
// multi-vector product stage its gathered rows in LDS.
std::vector<int> brick_order(const HostAsm& a) {
  const int64_t n = a.n;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], a.xyz[3 * i + d]);
      hi[d] = std::max(hi[d], a.xyz[3 * i + d]);
    }
  double ext[3], vol = 1.0;
  for (int d = 0; d < 3; ++d) {
    ext[d] = std::max(hi[d] - lo[d], 1e-300);
    vol *= ext[d];
  }
  const double h = std::cbrt(vol / double(std::max<int64_t>(n, 1)));
  int64_t nb[3];
  double edge[3];
  for (int d = 0; d < 3; ++d) {
    nb[d] = std::max<int64_t>(1, int64_t(std::ceil(ext[d] / (8.0 * h) - 1e-9)));
    edge[d] = ext[d] / double(nb[d]) * (1.0 + 1e-12);
  }
  std::vector<int64_t> key(n);
  for (int64_t i = 0; i < n; ++i) {
    int64_t b[3];
    for (int d = 0; d < 3; ++d)
      b[d] = std::min<int64_t>(nb[d] - 1, int64_t((a.xyz[3 * i + d] - lo[d]) / edge[d]));
    key[i] = (b[2] * nb[1] + b[1]) * nb[0] + b[0];
  }
  std::vector<int> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = int(i);
  std::sort(order.begin(), order.end(), [&](int x, int y) {
    if (key[x] != key[y]) return key[x] < key[y];
    for (int d = 2; d >= 0; --d)
      if (a.xyz[3 * x + d] != a.xyz[3 * y + d]) return a.xyz[3 * x + d] < a.xyz[3 * y + d];
    return x < y;
  });
  return order;
}

int build_sweep_data(hz_ctx ctx, SweepData* D) {
  const HostAsm& a = ctx->h;
  const int64_t n = a.n, nrows = ctx->sell.n_rows;
  D->nrows = nrows;
  // a structured box in its own numbering keeps its rows (x fastest: a
  // wave's rows are consecutive along x and share their neighbours' lines;
  // measured faster than the brick order at 80x48x40: 64-frequency TFQMR
  // sweep 0.88 vs 1.35 s); other meshes take the spatial brick order
  std::vector<int> perm;
  if (ctx->stencil_ok) {
    perm.resize(n);
    for (int64_t i = 0; i < n; ++i) perm[i] = int(i);
  } else {
    perm = brick_order(a);
  }
  std::vector<int> iperm(n);
  for (int64_t i = 0; i < n; ++i) iperm[perm[i]] = int(i);
  // boundary entries of each node: (column, sum_w beta_w B0_w)
  std::vector<std::vector<std::pair<int, z_t>>> bnd(n);
  {
    int64_t row = 0;
    std::vector<int64_t> order(a.bpos.size());
    for (size_t e = 0; e < order.size(); ++e) order[e] = int64_t(e);
    std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return a.bpos[x] < a.bpos[y]; });
    for (int64_t t = 0; t < int64_t(order.size()); ++t) {
      const int64_t e = order[t], pos = a.bpos[e];
      while (a.rowptr[row + 1] <= pos) ++row;
      double re = 0.0, im = 0.0;
      for (int w = 0; w < 6; ++w) {
        re += ctx->beta[w].real() * a.bmass[e * a.ntags + w];
        im += ctx->beta[w].imag() * a.bmass[e * a.ntags + w];
      }
      bnd[row].push_back({a.col[pos], z_t{re, im}});
    }
  }
  // the operator in the internal order
  const int64_t nnz = int64_t(a.col.size());
  std::vector<int> rowptr(nrows + 1, 0), col(nnz), dpos(n), bptr(nrows + 1, 0), bcol;
  std::vector<double> K(nnz), M(nnz), E(D->eta ? nnz : 0);
  D->eta = ctx->have_eta && !a.Meta.empty();
  if (D->eta) E.resize(nnz);
  std::vector<z_t> B64, Bd(n, z_t{0.0, 0.0});
  std::vector<c_t> B32;
  int64_t q = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int node = perm[i];
    for (int64_t p = a.rowptr[node]; p < a.rowptr[node + 1]; ++p, ++q) {
      col[q] = iperm[a.col[p]];
      K[q] = a.K[p];
      M[q] = a.M[p];
      if (D->eta) E[q] = a.Meta[p];
      if (a.col[p] == node) dpos[i] = int(q);
    }
    rowptr[i + 1] = int(q);
    for (const auto& b : bnd[node]) {
      bcol.push_back(iperm[b.first]);
      B64.push_back(b.second);
      B32.push_back(c_t{float(b.second.re), float(b.second.im)});
      if (b.first == node) Bd[i] = b.second;
    }
    bptr[i + 1] = int(bcol.size());
  }
  for (int64_t i = n; i < nrows; ++i) {
    rowptr[i + 1] = rowptr[i];
    bptr[i + 1] = bptr[i];
  }
  {
    // sweep row -> the caller's node id (through the context's numbering)
    std::vector<int> to_mesh(perm);
    if (!ctx->perm.empty())
      for (int& v : to_mesh) v = ctx->perm[v];
    HZ_TRY(upload(D->perm, to_mesh));
  }
  HZ_TRY(upload(D->rowptr, rowptr));
  HZ_TRY(upload(D->col, col));
  HZ_TRY(upload(D->K64, K));
  HZ_TRY(upload(D->M64, M));
  std::vector<float> f(nnz);
  for (int64_t p = 0; p < nnz; ++p) f[p] = float(K[p]);
  HZ_TRY(upload(D->K32, f));
  for (int64_t p = 0; p < nnz; ++p) f[p] = float(M[p]);
  HZ_TRY(upload(D->M32, f));
  if (D->eta) {
    HZ_TRY(upload(D->E64, E));
    for (int64_t p = 0; p < nnz; ++p) f[p] = float(E[p]);
    HZ_TRY(upload(D->E32, f));
  }
  HZ_TRY(upload(D->bptr, bptr));
  HZ_TRY(upload(D->bcol, bcol));
  HZ_TRY(upload(D->B64, B64));
  HZ_TRY(upload(D->B32, B32));
  HZ_TRY(upload(D->Bdiag, Bd));
  HZ_TRY(upload(D->dpos, dpos));
  D->n = n;
  D->nnz = nnz;
  D->nb = int64_t(bcol.size());
  if (ctx->stencil_ok) {
    // the rows are the box's nodes (x fastest): each entry goes to the slot
    // of its neighbour's offset
    const int64_t bx = ctx->elems[0] + 1, by = ctx->elems[1] + 1, bz = ctx->elems[2] + 1;
    if (bx * by * bz != n) return hz_fail(HZ_ERR_INVALID, "stencil box does not match the mesh");
    std::vector<z_t> km(size_t(kStencil) * nrows, z_t{0.0, 0.0});
    std::vector<c_t> km32(km.size(), c_t{0.f, 0.f});
    std::vector<double> se(D->eta ? km.size() : 0, 0.0);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t x = i % bx, y = i / bx % by, z = i / (bx * by);
      for (int q = rowptr[i]; q < rowptr[i + 1]; ++q) {
        const int64_t j = col[q];
        const int64_t dx = j % bx - x, dy = j / bx % by - y, dz = j / (bx * by) - z;
        if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1)
          return hz_fail(HZ_ERR_INVALID, "entry outside the 27-point stencil");
        const size_t at = size_t(i) * kStencil + size_t(9 * (dz + 1) + 3 * (dy + 1) + dx + 1);
        km[at] = z_t{K[q], M[q]};
        km32[at] = c_t{float(K[q]), float(M[q])};
        if (D->eta) se[at] = E[q];
      }
    }
    HZ_TRY(upload(D->KM64, km));
    HZ_TRY(upload(D->KM32, km32));
    // boundary entries of the rows on absorbing walls, in slot form
    std::vector<int> bsi(nrows, -1);
    std::vector<z_t> bsv;
    std::vector<c_t> bsv32;
    for (int64_t i = 0; i < n; ++i) {
      if (bptr[i] == bptr[i + 1]) continue;
      bsi[i] = int(bsv.size() / kStencil);
      bsv.resize(bsv.size() + kStencil, z_t{0.0, 0.0});
      const int64_t x = i % bx, y = i / bx % by, z = i / (bx * by);
      for (int q = bptr[i]; q < bptr[i + 1]; ++q) {
        const int64_t j = bcol[q];
        const int64_t dx = j % bx - x, dy = j / bx % by - y, dz = j / (bx * by) - z;
        if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1)
          return hz_fail(HZ_ERR_INVALID, "boundary entry outside the 27-point stencil");
        z_t& v = bsv[size_t(bsi[i]) * kStencil + size_t(9 * (dz + 1) + 3 * (dy + 1) + dx + 1)];
        v.re += B64[q].re;
        v.im += B64[q].im;
      }
    }
    bsv32.resize(bsv.size());
    for (size_t t = 0; t < bsv.size(); ++t) bsv32[t] = c_t{float(bsv[t].re), float(bsv[t].im)};
    HZ_TRY(upload(D->BSI, bsi));
    HZ_TRY(upload(D->BSV64, bsv));
    HZ_TRY(upload(D->BSV32, bsv32));
    if (D->eta) {
      HZ_TRY(upload(D->SE64, se));
      std::vector<float> se32(se.size());
      for (size_t t = 0; t < se.size(); ++t) se32[t] = float(se[t]);
      HZ_TRY(upload(D->SE32, se32));
    }
    D->box[0] = int(bx);
    D->box[1] = int(by);
    D->box[2] = int(bz);
  }
  // halos of the blocks of kHaloRows rows
  const int64_t nblk = (nrows + kHaloRows - 1) / kHaloRows;
  std::vector<int> hptr(nblk + 1, 0), hidx, cols;
  std::vector<int16_t> lidx(nnz, 0), blidx(bcol.size(), 0);
  int hmax = 0;
  bool ok = true;
  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t r0 = b * kHaloRows, r1 = std::min<int64_t>(n, r0 + kHaloRows);
    cols.clear();
    for (int64_t i = r0; i < r1; ++i) {
      for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) cols.push_back(col[p]);
      for (int p = bptr[i]; p < bptr[i + 1]; ++p) cols.push_back(bcol[p]);
    }
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    if (cols.size() > 32767) ok = false;
    hmax = std::max<int>(hmax, int(cols.size()));
    for (int64_t i = r0; i < r1 && ok; ++i) {
      for (int p = rowptr[i]; p < rowptr[i + 1]; ++p)
        lidx[p] = int16_t(std::lower_bound(cols.begin(), cols.end(), col[p]) - cols.begin());
      for (int p = bptr[i]; p < bptr[i + 1]; ++p)
        blidx[p] = int16_t(std::lower_bound(cols.begin(), cols.end(), bcol[p]) - cols.begin());
    }
    hidx.insert(hidx.end(), cols.begin(), cols.end());
    hptr[b + 1] = int(hidx.size());
  }
  D->hblocks = ok ? int(nblk) : 0;
  D->hmax = ok ? hmax : 0;
  if (ok) {
    HZ_TRY(upload(D->hptr, hptr));
    HZ_TRY(upload(D->hidx, hidx));
    HZ_TRY(upload(D->lidx, lidx));
    HZ_TRY(upload(D->blidx, blidx));
  }
  return HZ_OK;
}

template <typename T> RowOp<T> row_op(const SweepData& D);
template <typename T>
void add_halo(const SweepData& D, RowOp<T>* A) {
  A->hblocks = D.hblocks;
  A->hmax = D.hmax;
  if (D.hblocks) {
    A->hptr = D.hptr.as<int>();
    A->hidx = D.hidx.as<int>();
    A->lidx = D.lidx.as<int16_t>();
    A->blidx = D.blidx.as<int16_t>();
  }
}
template <typename T>
void add_stencil(const SweepData& D, const DevBuf& km, const DevBuf& se, RowOp<T>* A) {
  if (D.box[0] <= 0) return;
  A->KM = km.as<cx<T>>();
  A->SE = D.eta ? se.as<T>() : nullptr;
  A->BSI = D.BSI.as<int>();
  A->BSV = (sizeof(T) == 8 ? D.BSV64 : D.BSV32).as<cx<T>>();
  A->bx = D.box[0];
  A->by = D.box[1];
  A->bz = D.box[2];
}
template <> RowOp<double> row_op<double>(const SweepData& D) {
  RowOp<double> A = {D.rowptr.as<int>(), D.col.as<int>(), D.K64.as<double>(), D.M64.as<double>(),
                     D.eta ? D.E64.as<double>() : nullptr, D.bptr.as<int>(), D.bcol.as<int>(), D.B64.as<z_t>()};
  add_halo(D, &A);
  add_stencil(D, D.KM64, D.SE64, &A);
  return A;
}
template <> RowOp<float> row_op<float>(const SweepData& D) {
  RowOp<float> A = {D.rowptr.as<int>(), D.col.as<int>(), D.K32.as<float>(), D.M32.as<float>(),
                    D.eta ? D.E32.as<float>() : nullptr, D.bptr.as<int>(), D.bcol.as<int>(), D.B32.as<c_t>()};
  add_halo(D, &A);
  add_stencil(D, D.KM32, D.SE32, &A);
  return A;
}

// ---------------------------------------------------------------- autotuner
// Decimal code of a variant (tuning cache, HZ_SPMM_VARIANT): digits lds (as
// 1 + log2 of its column group, 0 for none), xcd, cpl, then three digits of
// the block size.
inline int log2p1(int v) {
  int r = 0;
  while (v > 0) {
    ++r;
    v >>= 1;
  }
  return r;
}
// A stencil-form variant has eight digits: 1, the broadcast (0 readlane,
// 1 LDS), pw, ph, then four of nzc.
inline int variant_code(const Variant& v) {
  if (v.zl > 0) return 10000000 + v.bc * 1000000 + v.pw * 100000 + v.ph * 10000 + v.nzc;
  return ((log2p1(v.lds) * 10 + v.xcd) * 10 + v.cpl) * 1000 + v.bs;
}
inline Variant variant_decode(int code) {
  auto un = [](int d) { return d == 0 ? 0 : 1 << (d - 1); };
  Variant v;
  if (code >= 10000000) {
    v.zl = 1;
    v.bc = code / 1000000 % 10;
    v.nzc = code % 10000;
    v.ph = code / 10000 % 10;
    v.pw = code / 100000 % 10;
    return v;
  }
  v.bs = code % 1000;
  code /= 1000;
  v.cpl = code % 10;
  code /= 10;
  v.xcd = code % 10;
  code /= 10;
  v.lds = un(code % 10);
  return v;
}
std::string tune_key(int64_t n, int64_t nnz, int s, int bytes) {
  std::ostringstream o;
  o << "spmm5 n=" << n << " nnz=" << nnz << " s=" << s << " t=" << bytes;
  return o.str();
}

void load_tune_cache(hz_ctx ctx) {
  const char* path = std::getenv("HZ_AUTOTUNE_CACHE");
  if (!path) return;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    auto p = line.rfind('|');
    if (p == std::string::npos) continue;
    ctx->tuned[line.substr(0, p)] = std::atoi(line.c_str() + p + 1);
  }
}

void save_tune_entry(const std::string& key, int code) {
  const char* path = std::getenv("HZ_AUTOTUNE_CACHE");
  if (!path) return;
  std::ofstream out(path, std::ios::app);
  out << key << "|" << code << "\n";
}

template <typename T>
int autotune(hz_ctx ctx, hipStream_t stream, int64_t nrows, int s, const RowOp<T>& A, const double* st,
             const cx<T>* Z, cx<T>* Y, Variant* best) {
  const std::string key = tune_key(ctx->h.n, int64_t(ctx->h.col.size()), s, int(sizeof(T)));
  if (const char* fv = std::getenv("HZ_SPMM_VARIANT")) {
    // one given variant (tests and measurements), if it fits this width
    const Variant v = variant_decode(std::atoi(fv));
    const bool fits = v.zl > 0    ? zl_fits<T>(v, s, A)
                      : v.lds > 0 ? (A.hblocks > 0 && s % v.lds == 0 && lds_bytes(A, v.lds) <= lds_limit())
                                  : (v.cpl <= s && v.bs >= s / v.cpl);
    if (fits) {
      *best = v;
      return HZ_OK;
    }
  }
  if (ctx->tuned.empty()) load_tune_cache(ctx);
  const char* force = std::getenv("HZ_SPMM_STAGED");   // "1": staged variants only, "0": none
  auto it = ctx->tuned.find(key);
  if (it != ctx->tuned.end() && !force) {
    *best = variant_decode(it->second);
    return HZ_OK;
  }
  std::vector<Variant> cands;
  if (!(force && force[0] == '1'))
    for (int xcd : {0, 1})
      for (int cpl : {1, 2})
        for (int bs : {128, 256, 512}) {
          if (cpl > s) continue;
          if (bs < s / cpl) continue;
          Variant v;
          v.cpl = cpl;
          v.bs = bs;
          v.xcd = xcd;
          cands.push_back(v);
        }
  if (!(force && force[0] == '0'))
    for (int cg : {1, 2, 4, 8, 16})
      if (A.hblocks > 0 && cg <= s && lds_bytes(A, cg) <= lds_limit()) {
        Variant v;
        v.bs = kHaloRows;
        v.lds = cg;
        cands.push_back(v);
      }
  if (!(force && force[0] == '1'))
    for (int bc : {0, 1})
      for (const ZlShape& h : kZlShapes)
        for (int nzc : {2, 4, 8, 16}) {
          Variant v;
          v.zl = 1;
          v.bc = bc;
          v.pw = h.pw;
          v.ph = h.ph;
          v.nzc = nzc;
          if (zl_fits<T>(v, s, A)) cands.push_back(v);
        }
  if (cands.empty()) cands.push_back(Variant{});
  hipEvent_t e0, e1;
  HZ_HIP(hipEventCreate(&e0));
  HZ_HIP(hipEventCreate(&e1));
  float best_ms = 1e30f;
  for (const Variant& v : cands) {
    // a variant the device cannot launch (e.g. more LDS than it grants) is skipped
    if (launch_spmm<T, false>(stream, v, nrows, s, A, st, Z, nullptr, Y, nullptr, nullptr) < 0) {
      (void)hipGetLastError();
      continue;
    }
    HZ_HIP(hipEventRecord(e0, stream));
    for (int r = 0; r < 5; ++r)
      HZ_TRY((launch_spmm<T, false>(stream, v, nrows, s, A, st, Z, nullptr, Y, nullptr, nullptr)));
    HZ_HIP(hipEventRecord(e1, stream));
    HZ_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    HZ_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      *best = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const int code = variant_code(*best);
  ctx->tuned[key] = code;
  save_tune_entry(key, code);
  return HZ_OK;
}

// Buffers and common set-up of one sweep call.
template <typename T>
struct Sweep {
  int s = 1, nf = 0, Gr = 1, nblk_res = 1;
  int64_t n = 0, nrows = 0, total = 0;
  const int* perm = nullptr;      // internal row -> node
  z_t *X = nullptr, *Fs = nullptr, *R = nullptr, *d64 = nullptr;
  cx<T>* dT = nullptr;
  double *kc = nullptr, *part = nullptr, *cn = nullptr;
  Variant vres, vin;
  RowOp<double> A64;
  RowOp<T> AT;
};

template <typename T>
int sweep_setup(hz_ctx ctx, SweepData& D, int nf, const double* freqs, const z_t* Fin, const z_t* Pio,
                Sweep<T>* W, const std::string& p, cx<T>* tune_z, cx<T>* tune_y) {
  int rc = 0;
  int s = 1;
  while (s < nf) s <<= 1;
  W->s = s;
  W->nf = nf;
  W->n = ctx->h.n;
  W->nrows = D.nrows;
  W->perm = D.perm.as<int>();
  W->total = D.nrows * s;
  const int64_t total = W->total;
  auto buf = [&](const char* nm, size_t bytes) -> void* {
    DevBuf* b = ctx->buf(p + nm, bytes, &rc);
    return rc ? nullptr : b->p;
  };
  W->X = static_cast<z_t*>(buf("X", sizeof(z_t) * total));
  W->Fs = static_cast<z_t*>(buf("F", sizeof(z_t) * total));
  W->R = static_cast<z_t*>(buf("R", sizeof(z_t) * total));
  W->d64 = static_cast<z_t*>(buf("d64", sizeof(z_t) * total));
  W->dT = static_cast<cx<T>*>(buf("dT", sizeof(cx<T>) * total));
  W->kc = static_cast<double*>(buf("kc", sizeof(double) * 2 * s));
  W->cn = static_cast<double*>(buf("cn", sizeof(double) * s));
  if (rc) return rc;
  W->Gr = int(std::min<int64_t>(std::max<int64_t>(total / kBlock, 1), 2048));
  W->nblk_res = int((D.nrows + kBlock / s - 1) / (kBlock / s));
  W->part = static_cast<double*>(buf("part", sizeof(double) * 3 * std::max<int64_t>(W->Gr, W->nblk_res) * s));
  if (rc) return rc;
  hipStream_t cs = ctx->stream;
  std::vector<double> kc(2 * s, 0.0);   // padding columns: k = 0 and a zero right-hand side
  for (int c = 0; c < nf; ++c) {
    double k = 2.0 * M_PI * freqs[c] / ctx->c;
    kc[2 * c] = k;
    kc[2 * c + 1] = mass_coefficient(k, ctx->h.gls_h);
  }
  HZ_HIP(hipMemcpyAsync(W->kc, kc.data(), sizeof(double) * 2 * s, hipMemcpyHostToDevice, cs));
  k_in<<<ceil_div(total, kBlock), kBlock, 0, cs>>>(W->n, W->nrows, s, nf, D.perm.as<int>(), Pio, Fin, W->X, W->Fs);
  k_diag<T><<<ceil_div(total, kBlock), kBlock, 0, cs>>>(W->n, W->nrows, s, D.dpos.as<int>(), D.K64.as<double>(),
                                                       D.M64.as<double>(), D.eta ? D.E64.as<double>() : nullptr,
                                                       D.Bdiag.as<z_t>(), W->kc, W->d64, W->dT);
  k_colnorm<double><<<W->Gr, kBlock, 0, cs>>>(total, s, W->Fs, W->part);
  k_colsum<<<s, kBlock, 0, cs>>>(W->Gr, s, W->part, W->cn);
  HZ_HIP(hipGetLastError());
  W->A64 = row_op<double>(D);
  W->AT = row_op<T>(D);
  W->vres.cpl = 1;            // FP64 residual product: one lane per column
  W->vres.bs = kBlock;
  HZ_TRY(autotune<T>(ctx, cs, W->nrows, s, W->AT, W->kc, tune_z, tune_y, &W->vin));
  return HZ_OK;
}

// A graph captured on a private stream that is ordered after the context
// stream (the null stream cannot be captured).
struct Graph {
  hipStream_t gs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev = nullptr;
  ~Graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ev) (void)hipEventDestroy(ev);
    if (gs) (void)hipStreamDestroy(gs);
  }
  int stream(hipStream_t after) {
    if (!gs) HZ_HIP(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
    if (!ev) HZ_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HZ_HIP(hipEventRecord(ev, after));
    HZ_HIP(hipStreamWaitEvent(gs, ev, 0));
    return HZ_OK;
  }
  template <class F>
  int capture(F body) {
    HZ_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
    int crc = body(gs);
    hipError_t ce = hipStreamEndCapture(gs, &graph);
    if (crc < 0) return crc;
    if (ce != hipSuccess) return hz_fail(HZ_ERR_HIP, "graph capture: %s", hipGetErrorString(ce));
    HZ_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    return HZ_OK;
  }
  int launch() {
    HZ_HIP(hipGraphLaunch(exec, gs));
    return HZ_OK;
  }
};

// Residual of the final iterate (FP64), copy-out and per-column results.
template <typename T>
int sweep_report(Sweep<T>& W, hipStream_t q, z_t* Pio, const std::vector<double>& fn2,
                 const std::vector<int>& iters, const std::vector<int64_t>& mv, const std::vector<int64_t>& imv,
                 const std::vector<int>& nan, const hz_solve_opts& o,
                 std::chrono::steady_clock::time_point t0, hz_solve_info* infos) {
  int nb = 0;
  HZ_TRY((launch_spmm<double, true>(q, W.vres, W.nrows, W.s, W.A64, W.kc, W.X, W.Fs, W.R, W.part, &nb)));
  k_colsum<<<W.s, kBlock, 0, q>>>(nb, W.s, W.part, W.cn);
  k_out<<<ceil_div(W.n * W.nf, kBlock), kBlock, 0, q>>>(W.n, W.s, W.nf, W.perm, W.X, Pio);
  HZ_HIP(hipGetLastError());
  std::vector<double> rr(W.s);
  HZ_HIP(hipMemcpyAsync(rr.data(), W.cn, sizeof(double) * W.s, hipMemcpyDeviceToHost, q));
  HZ_HIP(hipStreamSynchronize(q));
  double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = HZ_OK;
  for (int c = 0; c < W.nf; ++c) {
    hz_solve_info inf = {};
    double fnv = std::sqrt(fn2[c]);
    inf.relres_true = fnv > 0 ? std::sqrt(rr[c]) / fnv : 0.0;
    inf.relres_est = inf.relres_true;
    inf.iters = iters[c];
    inf.matvecs = int(mv[c]);
    inf.inner_matvecs = int(imv[c]);
    inf.seconds = secs;
    inf.status = nan[c] ? HZ_BREAKDOWN : (inf.relres_true <= o.tol ? HZ_OK : HZ_NOT_CONVERGED);
    if (!std::isfinite(inf.relres_true)) inf.status = HZ_BREAKDOWN;
    worst = std::max(worst, inf.status);
    if (infos) infos[c] = inf;
  }
  return worst;
}

template <typename T>
int run_sweep_gmres(hz_ctx ctx, SweepData& D, int nf, const double* freqs, const z_t* Fin, z_t* Pio,
                    const hz_solve_opts& o, hz_solve_info* infos) {
  auto t0 = std::chrono::steady_clock::now();
  int rc = 0;
  const int m = o.restart;
  const std::string p = std::string("sw.") + (sizeof(T) == 8 ? "z." : "c.");
  int s = 1;
  while (s < nf) s <<= 1;
  const int64_t total = D.nrows * s;
  auto buf = [&](const char* nm, size_t bytes) -> void* {
    DevBuf* b = ctx->buf(p + nm, bytes, &rc);
    return rc ? nullptr : b->p;
  };
  cx<T>* V = static_cast<cx<T>*>(buf("V", sizeof(cx<T>) * total * (m + 1)));
  cx<T>* Z = static_cast<cx<T>*>(buf("Z", sizeof(cx<T>) * total));
  if (rc) return rc;
  Sweep<T> W;
  HZ_TRY(sweep_setup<T>(ctx, D, nf, freqs, Fin, Pio, &W, p, Z, V + total));
  const int Gr = W.Gr;
  const int nch = ceil_div(m + 1, NV);
  z_t* mpart = static_cast<z_t*>(buf("mpart", sizeof(z_t) * int64_t(nch) * Gr * NV * s));
  SwCol* st = static_cast<SwCol*>(buf("st", sizeof(SwCol) * s));
  const int64_t zs = int64_t(s) * ((m + 1) * m + m + (m + 1) + m + 2 * (m + 1));
  z_t* small = static_cast<z_t*>(buf("small", sizeof(z_t) * zs + sizeof(double) * s * m));
  if (rc) return rc;
  SwArr A;
  A.m = m;
  z_t* zp = small;
  A.H = zp; zp += int64_t(s) * (m + 1) * m;
  A.sn = zp; zp += int64_t(s) * m;
  A.g = zp; zp += int64_t(s) * (m + 1);
  A.y = zp; zp += int64_t(s) * m;
  A.h1 = zp; zp += int64_t(s) * (m + 1);
  A.h2 = zp; zp += int64_t(s) * (m + 1);
  A.cs = reinterpret_cast<double*>(zp);
  hipStream_t cs = ctx->stream;
  HZ_HIP(hipMemsetAsync(st, 0, sizeof(SwCol) * s, cs));
  k_init_cols<<<1, 64, 0, cs>>>(s, st, W.cn, o.tol);
  HZ_HIP(hipGetLastError());

  auto cycle = [&](hipStream_t q) -> int {
    int nb = 0;
    HZ_TRY((launch_spmm<double, true>(q, W.vres, W.nrows, s, W.A64, W.kc, W.X, W.Fs, W.R, W.part, &nb)));
    k_beta_fin<<<s, kBlock, 0, q>>>(nb, s, st, A, W.part);
    k_v0<T><<<ceil_div(total, kBlock), kBlock, 0, q>>>(total, s, st, W.R, W.dT, V, Z);
    for (int j = 0; j < m; ++j) {
      cx<T>* w = V + int64_t(j + 1) * total;
      HZ_TRY((launch_spmm<T, false>(q, W.vin, W.nrows, s, W.AT, W.kc, Z, nullptr, w, nullptr, nullptr)));
      dim3 gd(Gr, ceil_div(j + 1, NV)), gf(s, j + 1);
      k_mdot<T><<<gd, kBlock, 0, q>>>(total, s, st, V, total, j, w, mpart);
      k_mdot_fin<<<gf, kBlock, 0, q>>>(Gr, s, st, A, mpart, j, 1);
      k_axpy<T, false><<<Gr, kBlock, 0, q>>>(total, s, st, A, V, total, j, 1, w, W.part);
      k_mdot<T><<<gd, kBlock, 0, q>>>(total, s, st, V, total, j, w, mpart);
      k_mdot_fin<<<gf, kBlock, 0, q>>>(Gr, s, st, A, mpart, j, 2);
      k_axpy<T, true><<<Gr, kBlock, 0, q>>>(total, s, st, A, V, total, j, 2, w, W.part);
      k_givens_fin<<<s, kBlock, 0, q>>>(Gr, s, st, A, W.part, j, o.inner_tol);
      k_scale<T><<<ceil_div(total, kBlock), kBlock, 0, q>>>(total, s, st, W.dT, w, Z);
    }
    k_solve_y<<<1, 64, 0, q>>>(s, st, A);
    k_update<T><<<ceil_div(total, kBlock), kBlock, 0, q>>>(total, s, st, A, V, total, W.d64, W.X);
    HZ_HIP(hipGetLastError());
    return HZ_OK;
  };
  Graph G;
  HZ_TRY(G.stream(cs));
  HZ_TRY(G.capture(cycle));
  void* hp = nullptr;
  HZ_TRY(ctx_pinned(ctx, sizeof(SwCol) * s, &hp));
  SwCol* hs = static_cast<SwCol*>(hp);
  std::vector<int64_t> mv(s, 0), imv(s, 0);
  for (;;) {
    HZ_TRY(G.launch());
    HZ_HIP(hipMemcpyAsync(hs, st, sizeof(SwCol) * s, hipMemcpyDeviceToHost, G.gs));
    HZ_HIP(hipStreamSynchronize(G.gs));
    bool all = true;
    int64_t mx = 0;
    for (int c = 0; c < nf; ++c) {
      mv[c] += 1;
      if (!hs[c].done) imv[c] += hs[c].kk;
      mx = std::max(mx, mv[c] + imv[c]);
      all = all && (hs[c].done || hs[c].nan);
    }
    if (all || mx + m + 1 > o.max_matvec) break;
  }
  std::vector<double> fn2(s);
  std::vector<int> iters(s), nan(s);
  for (int c = 0; c < s; ++c) {
    fn2[c] = hs[c].fn2;
    iters[c] = hs[c].iters;
    nan[c] = hs[c].nan;
  }
  return sweep_report(W, G.gs, Pio, fn2, iters, mv, imv, nan, o, t0, infos);
}

// Buffers of one column width s.
template <typename T>
struct BcWidth {
  int s = 0, Gr = 1;
  int64_t total = 0;
  z_t *X = nullptr, *Fs = nullptr, *R = nullptr, *d64 = nullptr;
  cx<T>* dT = nullptr;
  double *kc = nullptr, *part = nullptr, *cn = nullptr;
  BcCol* st = nullptr;
  BcVec<T> V;
  Variant vin, vres;
};

template <typename T>
int bc_alloc(hz_ctx ctx, int64_t nrows, int s, BcWidth<T>* W) {
  int rc = 0;
  const std::string p = std::string("swb.") + (sizeof(T) == 8 ? "z." : "c.") + std::to_string(s) + ".";
  const int64_t total = nrows * s;
  auto buf = [&](const char* nm, size_t bytes) -> void* {
    DevBuf* b = ctx->buf(p + nm, bytes, &rc);
    return rc ? nullptr : b->p;
  };
  W->s = s;
  W->total = total;
  W->Gr = int(std::min<int64_t>(std::max<int64_t>(total / kBlock, 1), 2048));
  const int64_t nblk_res = (nrows + kBlock / s - 1) / (kBlock / s);
  W->X = static_cast<z_t*>(buf("X", sizeof(z_t) * total));
  W->Fs = static_cast<z_t*>(buf("F", sizeof(z_t) * total));
  W->R = static_cast<z_t*>(buf("R", sizeof(z_t) * total));
  W->d64 = static_cast<z_t*>(buf("d64", sizeof(z_t) * total));
  W->dT = static_cast<cx<T>*>(buf("dT", sizeof(cx<T>) * total));
  W->kc = static_cast<double*>(buf("kc", sizeof(double) * 2 * s));
  W->cn = static_cast<double*>(buf("cn", sizeof(double) * s));
  W->part = static_cast<double*>(buf("part", sizeof(double) * 3 * std::max<int64_t>(W->Gr, nblk_res) * s));
  W->st = static_cast<BcCol*>(buf("st", sizeof(BcCol) * s));
  cx<T>** vv[9] = {&W->V.r, &W->V.rhat, &W->V.p, &W->V.v, &W->V.s, &W->V.t, &W->V.zp, &W->V.zs, &W->V.u};
  const char* names[9] = {"r", "rhat", "p", "v", "s", "t", "zp", "zs", "u"};
  for (int i = 0; i < 9; ++i) *vv[i] = static_cast<cx<T>*>(buf(names[i], sizeof(cx<T>) * total));
  if (rc) return rc;
  W->V.dT = W->dT;
  W->vres.cpl = 1;
  W->vres.bs = kBlock;
  return HZ_OK;
}

template <typename T>
int run_sweep_bicgstab(hz_ctx ctx, SweepData& D, int nf, const double* freqs, const z_t* Fin, z_t* Pio,
                       const hz_solve_opts& o, hz_solve_info* infos) {
  auto t0 = std::chrono::steady_clock::now();
  // complex64 recurrences drift: refresh the residual each time the recursive
  // one has fallen 10x below the last true one; FP64 runs straight to the target
  const double delta = sizeof(T) == 4 ? (o.inner_tol > 0 ? o.inner_tol : 0.1) : 0.0;
  const int chunk = 16;
  const int64_t nrows = D.nrows, n = ctx->h.n;
  const RowOp<double> A64 = row_op<double>(D);
  const RowOp<T> AT = row_op<T>(D);
  int s = 1;
  while (s < nf) s <<= 1;
  BcWidth<T> W;
  HZ_TRY(bc_alloc<T>(ctx, nrows, s, &W));
  hipStream_t cs = ctx->stream;
  std::vector<int> cols(nf);                   // current column j -> frequency index
  for (int c = 0; c < nf; ++c) cols[c] = c;
  auto upload_kc = [&](BcWidth<T>& w, hipStream_t q) -> int {
    std::vector<double> kc(2 * w.s, 0.0);
    for (size_t j = 0; j < cols.size(); ++j) {
      double k = 2.0 * M_PI * freqs[cols[j]] / ctx->c;
      kc[2 * j] = k;
      kc[2 * j + 1] = mass_coefficient(k, ctx->h.gls_h);
    }
    HZ_HIP(hipMemcpyAsync(w.kc, kc.data(), sizeof(double) * 2 * w.s, hipMemcpyHostToDevice, q));
    HZ_HIP(hipStreamSynchronize(q));
    return HZ_OK;
  };
  // set-up at the full width
  HZ_TRY(upload_kc(W, cs));
  k_in<<<ceil_div(W.total, kBlock), kBlock, 0, cs>>>(n, nrows, s, nf, D.perm.as<int>(), Pio, Fin, W.X, W.Fs);
  k_diag<T><<<ceil_div(W.total, kBlock), kBlock, 0, cs>>>(n, nrows, s, D.dpos.as<int>(), D.K64.as<double>(),
                                                         D.M64.as<double>(), D.eta ? D.E64.as<double>() : nullptr,
                                                         D.Bdiag.as<z_t>(), W.kc, W.d64, W.dT);
  k_colnorm<double><<<W.Gr, kBlock, 0, cs>>>(W.total, s, W.Fs, W.part);
  k_colsum<<<s, kBlock, 0, cs>>>(W.Gr, s, W.part, W.cn);
  HZ_HIP(hipMemsetAsync(W.st, 0, sizeof(BcCol) * s, cs));
  k_bc_init_cols<<<1, 64, 0, cs>>>(s, W.st, W.cn, o.tol);
  HZ_HIP(hipGetLastError());
  HZ_TRY(autotune<T>(ctx, cs, nrows, s, AT, W.kc, W.V.zp, W.V.v, &W.vin));

  auto iters_body = [&](hipStream_t q) -> int {
    const int s_ = W.s;
    const int64_t total = W.total;
    const int Gr = W.Gr, eb = ceil_div(total, kBlock);
    for (int it = 0; it < chunk; ++it) {
      k_bc_p<T><<<eb, kBlock, 0, q>>>(total, s_, W.st, W.V);
      HZ_TRY((launch_spmm<T, false>(q, W.vin, nrows, s_, AT, W.kc, W.V.zp, nullptr, W.V.v, nullptr, nullptr)));
      k_bc_dots<T, 2, false><<<Gr, kBlock, 0, q>>>(total, s_, W.st, W.V.rhat, W.V.v, W.part);
      k_bc_alpha<<<s_, kBlock, 0, q>>>(Gr, s_, W.st, W.part);
      k_bc_s<T><<<Gr, kBlock, 0, q>>>(total, s_, W.st, W.V, W.part);
      k_bc_sfin<<<s_, kBlock, 0, q>>>(Gr, s_, W.st, W.part);
      HZ_TRY((launch_spmm<T, false>(q, W.vin, nrows, s_, AT, W.kc, W.V.zs, nullptr, W.V.t, nullptr, nullptr)));
      k_bc_dots<T, 3, false><<<Gr, kBlock, 0, q>>>(total, s_, W.st, W.V.t, W.V.s, W.part);
      k_bc_omega<<<s_, kBlock, 0, q>>>(Gr, s_, W.st, W.part);
      k_bc_xr<T><<<Gr, kBlock, 0, q>>>(total, s_, W.st, W.V, W.part);
      k_bc_rho<<<s_, kBlock, 0, q>>>(Gr, s_, W.st, W.part);
    }
    HZ_HIP(hipGetLastError());
    return HZ_OK;
  };
  auto outer = [&](hipStream_t q) -> int {
    const int s_ = W.s;
    const int64_t total = W.total;
    const int eb = ceil_div(total, kBlock);
    int nb = 0;
    k_bc_update<T><<<eb, kBlock, 0, q>>>(total, s_, W.st, W.V.u, W.X);
    HZ_TRY((launch_spmm<double, true>(q, W.vres, nrows, s_, A64, W.kc, W.X, W.Fs, W.R, W.part, &nb)));
    k_bc_beta<<<s_, kBlock, 0, q>>>(nb, s_, W.st, W.part, o.tol, delta);
    k_bc_start<T><<<eb, kBlock, 0, q>>>(total, s_, W.st, W.R, W.V);
    k_bc_dots<T, 4, true><<<W.Gr, kBlock, 0, q>>>(total, s_, W.st, W.V.rhat, W.V.r, W.part);
    k_bc_rho0<<<s_, kBlock, 0, q>>>(W.Gr, s_, W.st, W.part);
    HZ_HIP(hipGetLastError());
    return HZ_OK;
  };

  std::unique_ptr<Graph> G(new Graph());
  HZ_TRY(G->stream(cs));
  HZ_TRY(G->capture(iters_body));
  hipStream_t q = G->gs;
  void* hp = nullptr;
  HZ_TRY(ctx_pinned(ctx, sizeof(BcCol) * 64, &hp));
  BcCol* hs = static_cast<BcCol*>(hp);
  std::vector<hz_solve_info> res(nf);
  std::vector<char> finished(nf, 0);
  int worst = HZ_OK;
  auto record = [&](int j, double secs) {
    const BcCol& S = hs[j];
    const int f = cols[j];
    hz_solve_info inf = {};
    double fnv = std::sqrt(S.fn2);
    inf.relres_true = fnv > 0 ? S.beta / fnv : 0.0;
    inf.relres_est = inf.relres_true;
    inf.iters = S.iters;
    inf.matvecs = S.outer + 1;
    inf.inner_matvecs = 2 * S.iters;
    inf.seconds = secs;
    inf.status = S.nan ? HZ_BREAKDOWN : (S.done && inf.relres_true <= o.tol * (1 + 1e-12) ? HZ_OK : HZ_NOT_CONVERGED);
    if (!std::isfinite(inf.relres_true)) inf.status = HZ_BREAKDOWN;
    res[f] = inf;
    finished[f] = 1;
  };
  DevBuf* mapb = nullptr;
  int rc = 0;
  mapb = ctx->buf("swb.map", sizeof(int) * 128, &rc);
  if (rc) return rc;
  bool capped = false;
  bool stop = false;
  while (!stop) {
    HZ_HIP(hipMemcpyAsync(hs, W.st, sizeof(BcCol) * W.s, hipMemcpyDeviceToHost, q));
    HZ_HIP(hipStreamSynchronize(q));
    const int nreal = int(cols.size());
    int active = 0;
    bool pending = false;
    int64_t mx = 0;
    for (int j = 0; j < nreal; ++j) {
      const BcCol& S = hs[j];
      if (S.done || S.nan) continue;
      ++active;
      pending = pending || S.idone;
      mx = std::max<int64_t>(mx, 2 * int64_t(S.iters) + S.outer + 1);
    }
    if (active == 0) break;
    if (pending) {
      HZ_TRY(outer(q));
      continue;
    }
    // two products stay in reserve for the refinement step at the cap
    if (mx + 2 * chunk + 3 > o.max_matvec) {
      if (capped) break;
      capped = true;
      k_end_inner<BcCol><<<1, 64, 0, q>>>(W.s, W.st);
      HZ_TRY(outer(q));
      continue;
    }
    if (active <= W.s / 2) {
      // compaction: finished columns leave, the rest move to a narrower width
      std::vector<int> keep, gone_j, gone_f;
      for (int j = 0; j < nreal; ++j) {
        if (hs[j].done || hs[j].nan) {
          gone_j.push_back(j);
          gone_f.push_back(cols[j]);
        } else {
          keep.push_back(j);
        }
      }
      double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      for (int j : gone_j) record(j, secs);
      if (!gone_j.empty()) {
        std::vector<int> h2(gone_j);
        h2.insert(h2.end(), gone_f.begin(), gone_f.end());
        HZ_HIP(hipMemcpyAsync(mapb->p, h2.data(), sizeof(int) * h2.size(), hipMemcpyHostToDevice, q));
        const int ng = int(gone_j.size());
        k_out_cols<<<ceil_div(n * ng, kBlock), kBlock, 0, q>>>(n, W.s, nf, ng, D.perm.as<int>(), mapb->as<int>(),
                                                                mapb->as<int>() + ng, W.X, Pio);
        HZ_HIP(hipGetLastError());
        HZ_HIP(hipStreamSynchronize(q));
      }
      int s2 = 1;
      while (s2 < int(keep.size())) s2 <<= 1;
      BcWidth<T> W2;
      HZ_TRY(bc_alloc<T>(ctx, nrows, s2, &W2));
      std::vector<int> map(s2, -1);
      for (size_t jn = 0; jn < keep.size(); ++jn) map[jn] = keep[jn];
      HZ_HIP(hipMemcpyAsync(mapb->p, map.data(), sizeof(int) * s2, hipMemcpyHostToDevice, q));
      const int gb = ceil_div(nrows * s2, kBlock);
      const int* mp = mapb->as<int>();
      k_gather_cols<z_t><<<gb, kBlock, 0, q>>>(nrows, W.s, s2, mp, W.X, W2.X);
      k_gather_cols<z_t><<<gb, kBlock, 0, q>>>(nrows, W.s, s2, mp, W.Fs, W2.Fs);
      k_gather_cols<z_t><<<gb, kBlock, 0, q>>>(nrows, W.s, s2, mp, W.d64, W2.d64);
      k_gather_cols<cx<T>><<<gb, kBlock, 0, q>>>(nrows, W.s, s2, mp, W.dT, W2.dT);
      cx<T>* from[9] = {W.V.r, W.V.rhat, W.V.p, W.V.v, W.V.s, W.V.t, W.V.zp, W.V.zs, W.V.u};
      cx<T>* to[9] = {W2.V.r, W2.V.rhat, W2.V.p, W2.V.v, W2.V.s, W2.V.t, W2.V.zp, W2.V.zs, W2.V.u};
      for (int i = 0; i < 9; ++i) k_gather_cols<cx<T>><<<gb, kBlock, 0, q>>>(nrows, W.s, s2, mp, from[i], to[i]);
      HZ_HIP(hipGetLastError());
      std::vector<BcCol> ns(s2);
      for (int jn = 0; jn < s2; ++jn) {
        if (map[jn] >= 0) {
          ns[jn] = hs[map[jn]];
        } else {
          ns[jn] = BcCol{};
          ns[jn].done = 1;
        }
      }
      std::vector<int> ncols;
      for (int j : keep) ncols.push_back(cols[j]);
      cols = ncols;
      HZ_HIP(hipMemcpyAsync(W2.st, ns.data(), sizeof(BcCol) * s2, hipMemcpyHostToDevice, q));
      HZ_TRY(upload_kc(W2, q));
      HZ_TRY(autotune<T>(ctx, q, nrows, s2, AT, W2.kc, W2.V.zp, W2.V.v, &W2.vin));
      W = W2;
      // new graph ordered after the old stream; the old graph and stream go once idle
      std::unique_ptr<Graph> G2(new Graph());
      HZ_TRY(G2->stream(q));
      HZ_TRY(G2->capture(iters_body));
      HZ_HIP(hipStreamSynchronize(q));
      G = std::move(G2);
      q = G->gs;
      continue;
    }
    HZ_TRY(G->launch());
  }
  // remaining columns: copy out and record
  HZ_HIP(hipMemcpyAsync(hs, W.st, sizeof(BcCol) * W.s, hipMemcpyDeviceToHost, q));
  HZ_HIP(hipStreamSynchronize(q));
  {
    const int nreal = int(cols.size());
    std::vector<int> h2(2 * nreal);
    for (int j = 0; j < nreal; ++j) {
      h2[j] = j;
      h2[nreal + j] = cols[j];
    }
    if (nreal > 0) {
      HZ_HIP(hipMemcpyAsync(mapb->p, h2.data(), sizeof(int) * h2.size(), hipMemcpyHostToDevice, q));
      k_out_cols<<<ceil_div(n * nreal, kBlock), kBlock, 0, q>>>(n, W.s, nf, nreal, D.perm.as<int>(), mapb->as<int>(),
                                                                 mapb->as<int>() + nreal, W.X, Pio);
      HZ_HIP(hipGetLastError());
      HZ_HIP(hipStreamSynchronize(q));
    }
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int j = 0; j < nreal; ++j) record(j, secs);
  }
  for (int f = 0; f < nf; ++f) {
    worst = std::max(worst, res[f].status);
    if (infos) infos[f] = res[f];
  }
  (void)stop;
  return worst;
}

// ---------------------------------------------------------------- batched BiCGStab(l)
// Each column runs its own BiCGStab(l) (the cycle of the single-system
// solver: l bi-conjugate gradient steps, a Gram-matrix minimal-residual step)
// on the correction equation B(k_c) y = R_c / scale_c, B = A D^-1.  When the
// inner stopping test fires, or the column breaks down, the host runs that
// column's refinement step: X += scale D^-1 y, R = F - A X in FP64, restart.
// In FP64 storage the inner solve runs to the target, so the step only
// confirms convergence; in complex64 storage it runs to inner_tol.
constexpr int kSlMaxL = 8;

struct SlCol {
  double fn2, thr2, scale, ithr2, rr, beta, rhat2, pad0;
  z_t rho0, alpha, omega, bet;
  z_t gam[kSlMaxL + 1];
  int done, idone, nan, iters, outer, restart_now, trunc, pad1;
};

template <typename T>
struct SlVec {
  cx<T>* y;      // inner iterate (scaled unknowns)
  cx<T>* rt;
  cx<T>* Z;      // D^-1 (chain vector): input of the products
  cx<T>* r[kSlMaxL + 1];
  cx<T>* u[kSlMaxL + 1];
  const cx<T>* dT;
};

__device__ __forceinline__ bool sl_off(const SlCol& S) { return S.done || S.idone || S.nan; }
__device__ __forceinline__ bool sl_pending(const SlCol& S) { return S.idone && !S.done && !S.nan; }

// refinement, part 1: X += scale D^-1 y for columns whose inner solve ended
template <typename T>
__global__ void k_sl_addx(int64_t total, int s, const SlCol* __restrict__ st, SlVec<T> V, z_t* __restrict__ X) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= total) return;
  const SlCol& S = st[e & (s - 1)];
  if (!sl_pending(S) || S.scale == 0.0) return;
  z_t d = ccast<double>(V.dT[e]) * ccast<double>(V.y[e]);
  X[e] = z_t{fma(S.scale, d.re, X[e].re), fma(S.scale, d.im, X[e].im)};
}

// part 2 (block per column, after the FP64 residual): convergence, inner threshold
__global__ void k_sl_true(int nblk, int s, SlCol* st, const double* __restrict__ part, double tol, double delta) {
  __shared__ double lds[kBlock / kWave];
  const int c = blockIdx.x;
  const int pend = sl_pending(st[c]);
  __syncthreads();
  if (!pend) return;
  const double rr = block_sum_strided(part + c, nblk, s, lds);
  if (threadIdx.x != 0) return;
  SlCol& S = st[c];
  const double b = sqrt(rr);
  S.beta = b;
  S.nan = S.nan || !isfinite(rr);
  S.done = (rr <= S.thr2) || S.fn2 == 0.0 || S.nan;
  if (S.done) return;
  S.outer += 1;
  S.idone = 0;
  S.restart_now = 1;
  S.scale = b;
  const double lim = 0.5 * tol * sqrt(S.fn2) / b;   // the target in the scaled system
  const double it = delta > lim ? delta : lim;
  S.ithr2 = it * it;
}

// part 3: r_0 = R / scale, rt = r_0, u_0 = y = 0 for restarting columns
template <typename T>
__global__ void k_sl_start(int64_t total, int s, const SlCol* __restrict__ st, const z_t* __restrict__ R,
                           SlVec<T> V) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= total) return;
  const SlCol& S = st[e & (s - 1)];
  if (!S.restart_now) return;
  const cx<T> r = ccast<T>((1.0 / S.scale) * R[e]);
  const cx<T> z = {T(0), T(0)};
  V.r[0][e] = r;
  V.rt[e] = r;
  V.u[0][e] = z;
  V.y[e] = z;
}

__global__ void k_sl_start_fin(int s, SlCol* st) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= s) return;
  SlCol& S = st[c];
  if (!S.restart_now) return;
  S.restart_now = 0;
  S.rr = 1.0;                       // ||R / scale|| = 1
  S.rhat2 = 1.0;
  S.rho0 = z_t{1.0, 0.0};           // rt^H r_0
  S.alpha = S.bet = z_t{0.0, 0.0};
  S.omega = z_t{1.0, 0.0};
  S.trunc = 0;
}

// partial a^H b per column (NQ = 2) or a^H b and ||b||^2 (NQ = 3), grid-stride
template <typename T, int NQ>
__global__ void __launch_bounds__(kBlock) k_sl_dots(int64_t total, int s, const SlCol* __restrict__ st,
                                                    const cx<T>* __restrict__ a, const cx<T>* __restrict__ b,
                                                    double* __restrict__ part) {
  __shared__ double lds[4 * kWave];
  const int c = threadIdx.x & (s - 1);
  double q[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) q[i] = 0.0;
  if (!sl_off(st[c])) {
    for (int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x; e < total; e += int64_t(gridDim.x) * kBlock) {
      const z_t x = ccast<double>(a[e]), y = ccast<double>(b[e]);
      q[0] = fma(x.re, y.re, fma(x.im, y.im, q[0]));
      q[1] = fma(x.re, y.im, fma(-x.im, y.re, q[1]));
      if (NQ == 3) q[2] += norm2(y);
    }
  }
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const double t = col_reduce(q[i], s, lds);
    if (int(threadIdx.x) < s) part[(int64_t(blockIdx.x) * NQ + i) * s + threadIdx.x] = t;
  }
}

__device__ __forceinline__ double sl_sum(int G_, int s, int nq, const double* part, int c, int i, double* lds) {
  return block_sum_strided(part + int64_t(i) * s + c, G_, nq * s, lds);
}

// u_i = r_i - beta u_i (i <= j); Z = D^-1 u_j
template <typename T>
__global__ void k_sl_u(int64_t total, int s, const SlCol* __restrict__ st, SlVec<T> V, int j) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= total) return;
  const SlCol& S = st[e & (s - 1)];
  if (sl_off(S)) return;
  const z_t b = S.bet;
  z_t uj = {0.0, 0.0};
  for (int i = 0; i <= j; ++i) {
    uj = ccast<double>(V.r[i][e]) - b * ccast<double>(V.u[i][e]);
    V.u[i][e] = ccast<T>(uj);
  }
  V.Z[e] = ccast<T>(ccast<double>(V.dT[e]) * ccast<double>(ccast<T>(uj)));
}

// alpha = rho0 / rt^H u_{j+1}
__global__ void k_sl_alpha(int G_, int s, SlCol* st, const double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  const int c = blockIdx.x;
  const int off = sl_off(st[c]);
  __syncthreads();
  if (off) return;
  const double re = sl_sum(G_, s, 2, part, c, 0, lds);
  const double im = sl_sum(G_, s, 2, part, c, 1, lds);
  if (threadIdx.x != 0) return;
  SlCol& S = st[c];
  const z_t sg = {re, im};
  if (norm2(sg) == 0.0 || !isfinite(re) || !isfinite(im)) S.idone = 1;   // breakdown: refine and restart
  else S.alpha = cdiv(S.rho0, sg);
}

// r_i -= alpha u_{i+1} (i <= j); y += alpha u_0; Z = D^-1 r_j
template <typename T>
__global__ void k_sl_r(int64_t total, int s, const SlCol* __restrict__ st, SlVec<T> V, int j) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= total) return;
  const SlCol& S = st[e & (s - 1)];
  if (sl_off(S)) return;
  const z_t a = S.alpha;
  cx<T> rj = {T(0), T(0)};
  for (int i = 0; i <= j; ++i) {
    rj = ccast<T>(ccast<double>(V.r[i][e]) - a * ccast<double>(V.u[i + 1][e]));
    V.r[i][e] = rj;
  }
  V.y[e] = ccast<T>(ccast<double>(V.y[e]) + a * ccast<double>(V.u[0][e]));
  V.Z[e] = ccast<T>(ccast<double>(V.dT[e]) * ccast<double>(rj));
}

// rho1 = rt^H r_{j+1}; beta = alpha rho1 / rho0; rho0 = rho1
__global__ void k_sl_beta(int G_, int s, SlCol* st, const double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  const int c = blockIdx.x;
  const int off = sl_off(st[c]);
  __syncthreads();
  if (off) return;
  const double re = sl_sum(G_, s, 2, part, c, 0, lds);
  const double im = sl_sum(G_, s, 2, part, c, 1, lds);
  if (threadIdx.x != 0) return;
  SlCol& S = st[c];
  const z_t rho1 = {re, im};
  if (norm2(S.rho0) == 0.0 || !isfinite(re) || !isfinite(im)) {
    S.idone = 1;
  } else {
    S.bet = S.alpha * cdiv(rho1, S.rho0);
    S.rho0 = rho1;
  }
}

template <int LL> constexpr int sl_nq() { return 2 * (LL + LL * (LL + 1) / 2); }

// partials of c_i = r_i^H r_0 and G_ij = r_i^H r_j (1 <= i <= j <= LL) per column
template <typename T, int LL>
__global__ void __launch_bounds__(kBlock) k_sl_gram(int64_t total, int s, const SlCol* __restrict__ st, SlVec<T> V,
                                                    double* __restrict__ part) {
  constexpr int NQ = sl_nq<LL>();
  __shared__ double lds[4 * kWave];
  const int c = threadIdx.x & (s - 1);
  double q[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) q[i] = 0.0;
  if (!sl_off(st[c])) {
    for (int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x; e < total; e += int64_t(gridDim.x) * kBlock) {
      z_t r[LL + 1];
#pragma unroll
      for (int i = 0; i <= LL; ++i) r[i] = ccast<double>(V.r[i][e]);
      int k = 0;
#pragma unroll
      for (int i = 1; i <= LL; ++i, k += 2) {
        q[k] = fma(r[i].re, r[0].re, fma(r[i].im, r[0].im, q[k]));
        q[k + 1] = fma(r[i].re, r[0].im, fma(-r[i].im, r[0].re, q[k + 1]));
      }
#pragma unroll
      for (int i = 1; i <= LL; ++i)
#pragma unroll
        for (int jj = i; jj <= LL; ++jj, k += 2) {
          q[k] = fma(r[i].re, r[jj].re, fma(r[i].im, r[jj].im, q[k]));
          q[k + 1] = fma(r[i].re, r[jj].im, fma(-r[i].im, r[jj].re, q[k + 1]));
        }
    }
  }
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const double t = col_reduce(q[i], s, lds);
    if (int(threadIdx.x) < s) part[(int64_t(blockIdx.x) * NQ + i) * s + threadIdx.x] = t;
  }
}

// Cholesky solve of G gamma = c per column (truncated at the first pivot
// below piv times its diagonal entry)
template <int LL>
__global__ void k_sl_mr(int G_, int s, SlCol* st, const double* __restrict__ part, double piv) {
  constexpr int NQ = sl_nq<LL>();
  __shared__ double lds[kBlock / kWave];
  __shared__ double tot[NQ];
  const int c = blockIdx.x;
  const int off = sl_off(st[c]);
  __syncthreads();
  if (off) return;
  for (int i = 0; i < NQ; ++i) {
    const double t = sl_sum(G_, s, NQ, part, c, i, lds);
    if (threadIdx.x == 0) tot[i] = t;
  }
  if (threadIdx.x != 0) return;
  SlCol& S = st[c];
  z_t cv[LL], G[LL][LL];
  int k = 0;
  for (int i = 0; i < LL; ++i, k += 2) cv[i] = z_t{tot[k], tot[k + 1]};
  for (int i = 0; i < LL; ++i)
    for (int jj = i; jj < LL; ++jj, k += 2) {
      G[i][jj] = z_t{tot[k], tot[k + 1]};
      G[jj][i] = conj(G[i][jj]);
    }
  int m = LL;
  for (int jj = 0; jj < LL; ++jj) {
    double d = G[jj][jj].re;
    for (int p = 0; p < jj; ++p) d -= norm2(G[jj][p]);
    if (!(d > piv * G[jj][jj].re) || !isfinite(d)) {
      m = jj;
      break;
    }
    const double cd = sqrt(d);
    G[jj][jj] = z_t{cd, 0.0};
    for (int i = jj + 1; i < LL; ++i) {
      z_t v = G[i][jj];
      for (int p = 0; p < jj; ++p) v = v - G[i][p] * conj(G[jj][p]);
      G[i][jj] = (1.0 / cd) * v;
    }
  }
  z_t g[LL];
  for (int i = 0; i < LL; ++i) g[i] = z_t{0.0, 0.0};
  if (m == 0) {
    S.idone = 1;
    return;
  }
  z_t yv[LL];
  for (int i = 0; i < m; ++i) {
    z_t v = cv[i];
    for (int p = 0; p < i; ++p) v = v - G[i][p] * yv[p];
    yv[i] = (1.0 / G[i][i].re) * v;
  }
  for (int i = m - 1; i >= 0; --i) {
    z_t v = yv[i];
    for (int p = i + 1; p < m; ++p) v = v - conj(G[p][i]) * g[p];
    g[i] = (1.0 / G[i][i].re) * v;
  }
  for (int i = 0; i < LL; ++i)
    if (!isfinite(g[i].re) || !isfinite(g[i].im)) {
      S.idone = 1;
      return;
    }
  for (int i = 0; i < LL; ++i) S.gam[i + 1] = g[i];
  S.omega = g[LL - 1];
  S.trunc = m < LL;
}

// y += sum gamma_j r_{j-1}; r_0 -= sum gamma_j r_j; u_0 -= sum gamma_j u_j
template <typename T, int LL>
__global__ void k_sl_update(int64_t total, int s, const SlCol* __restrict__ st, SlVec<T> V) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= total) return;
  const SlCol& S = st[e & (s - 1)];
  if (sl_off(S)) return;
  z_t y = ccast<double>(V.y[e]), r0 = ccast<double>(V.r[0][e]), u0 = ccast<double>(V.u[0][e]);
  z_t rprev = r0;
#pragma unroll
  for (int jj = 1; jj <= LL; ++jj) {
    const z_t g = S.gam[jj];
    const z_t rj = ccast<double>(V.r[jj][e]);
    y = y + g * rprev;
    r0 = r0 - g * rj;
    u0 = u0 - g * ccast<double>(V.u[jj][e]);
    rprev = rj;
  }
  V.y[e] = ccast<T>(y);
  V.r[0][e] = ccast<T>(r0);
  V.u[0][e] = ccast<T>(u0);
}

// after the update: rho1 = rt^H r_0, ||r_0||^2; next cycle's beta, or done
__global__ void k_sl_cycle(int G_, int s, SlCol* st, const double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  const int c = blockIdx.x;
  const int off = sl_off(st[c]);
  __syncthreads();
  if (off) return;
  const double re = sl_sum(G_, s, 3, part, c, 0, lds);
  const double im = sl_sum(G_, s, 3, part, c, 1, lds);
  const double rr = sl_sum(G_, s, 3, part, c, 2, lds);
  if (threadIdx.x != 0) return;
  SlCol& S = st[c];
  S.iters += 1;
  S.rr = rr;
  const z_t rho1 = {re, im};
  if (!isfinite(rr) || !isfinite(re) || !isfinite(im)) {
    S.nan = 1;
    return;
  }
  if (rr <= S.ithr2) {
    S.idone = 1;
    return;
  }
  const z_t rho0 = -1.0 * (S.omega * S.rho0);
  if (S.trunc || norm2(rho0) == 0.0 || sqrt(norm2(rho1)) < 1e-300 * sqrt(S.rhat2 * rr)) {
    S.idone = 1;               // refinement step and restart
    return;
  }
  S.bet = S.alpha * cdiv(rho1, rho0);
  S.rho0 = rho1;
}

__global__ void k_sl_init(int s, SlCol* st, const double* fn2, double tol) {
  const int c = threadIdx.x;
  if (c >= s) return;
  st[c].fn2 = fn2[c];
  st[c].thr2 = tol * tol * fn2[c];
  st[c].idone = 1;                 // every column starts with a refinement step
}

// Buffers of one column width s.
template <typename T>
struct SlWidth {
  int s = 0, Gr = 1, l = 4;
  int64_t total = 0;
  z_t *X = nullptr, *Fs = nullptr, *R = nullptr;
  cx<T>* dT = nullptr;
  double *kc = nullptr, *part = nullptr, *cn = nullptr;
  SlCol* st = nullptr;
  SlVec<T> V;
  Variant vin, vres;
};

template <typename T>
int sl_alloc(hz_ctx ctx, int64_t nrows, int s, int l, SlWidth<T>* W) {
  int rc = 0;
  const std::string p = std::string("swl.") + (sizeof(T) == 8 ? "z." : "c.") + std::to_string(s) + ".";
  const int64_t total = nrows * s;
  auto buf = [&](const std::string& nm, size_t bytes) -> void* {
    DevBuf* b = ctx->buf(p + nm, bytes, &rc);
    return rc ? nullptr : b->p;
  };
  W->s = s;
  W->l = l;
  W->total = total;
  W->Gr = int(std::min<int64_t>(std::max<int64_t>(total / kBlock, 1), 1024));
  const int64_t nblk_res = (nrows + kBlock / s - 1) / (kBlock / s);
  W->X = static_cast<z_t*>(buf("X", sizeof(z_t) * total));
  W->Fs = static_cast<z_t*>(buf("F", sizeof(z_t) * total));
  W->R = static_cast<z_t*>(buf("R", sizeof(z_t) * total));
  W->dT = static_cast<cx<T>*>(buf("dT", sizeof(cx<T>) * total));
  W->kc = static_cast<double*>(buf("kc", sizeof(double) * 2 * s));
  W->cn = static_cast<double*>(buf("cn", sizeof(double) * s));
  const int64_t npart = std::max<int64_t>(int64_t(W->Gr) * sl_nq<kSlMaxL>(), nblk_res) * s;
  W->part = static_cast<double*>(buf("part", sizeof(double) * npart));
  W->st = static_cast<SlCol*>(buf("st", sizeof(SlCol) * s));
  W->V = SlVec<T>{};
  W->V.y = static_cast<cx<T>*>(buf("y", sizeof(cx<T>) * total));
  W->V.rt = static_cast<cx<T>*>(buf("rt", sizeof(cx<T>) * total));
  W->V.Z = static_cast<cx<T>*>(buf("Z", sizeof(cx<T>) * total));
  for (int i = 0; i <= l; ++i) {
    W->V.r[i] = static_cast<cx<T>*>(buf("r" + std::to_string(i), sizeof(cx<T>) * total));
    W->V.u[i] = static_cast<cx<T>*>(buf("u" + std::to_string(i), sizeof(cx<T>) * total));
  }
  if (rc) return rc;
  W->V.dT = W->dT;
  W->vres.cpl = 1;
  W->vres.bs = kBlock;
  return HZ_OK;
}

template <typename T, int LL>
int sl_enqueue_mr(hipStream_t q, SlWidth<T>& W) {
  const int eb = ceil_div(W.total, kBlock);
  k_sl_gram<T, LL><<<W.Gr, kBlock, 0, q>>>(W.total, W.s, W.st, W.V, W.part);
  k_sl_mr<LL><<<W.s, kBlock, 0, q>>>(W.Gr, W.s, W.st, W.part, 1e-13);
  k_sl_update<T, LL><<<eb, kBlock, 0, q>>>(W.total, W.s, W.st, W.V);
  HZ_HIP(hipGetLastError());
  return HZ_OK;
}

template <typename T>
int run_sweep_bicgstabl(hz_ctx ctx, SweepData& D, int nf, const double* freqs, const z_t* Fin, z_t* Pio,
                        const hz_solve_opts& o, hz_solve_info* infos) {
  auto t0 = std::chrono::steady_clock::now();
  const int l = o.restart;
  // complex64 inner solves stop at inner_tol relative to their right-hand side
  const double delta = sizeof(T) == 4 ? (o.inner_tol > 0 ? o.inner_tol : 1e-3) : 0.0;
  const int chunk = std::max(1, 16 / l);      // cycles per graph launch (~32 products)
  const int64_t nrows = D.nrows, n = ctx->h.n;
  const RowOp<double> A64 = row_op<double>(D);
  const RowOp<T> AT = row_op<T>(D);
  int s = 1;
  while (s < nf) s <<= 1;
  SlWidth<T> W;
  HZ_TRY(sl_alloc<T>(ctx, nrows, s, l, &W));
  hipStream_t cs = ctx->stream;
  std::vector<int> cols(nf);                   // current column j -> frequency index
  for (int c = 0; c < nf; ++c) cols[c] = c;
  auto upload_kc = [&](SlWidth<T>& w, hipStream_t q) -> int {
    std::vector<double> kc(2 * w.s, 0.0);
    for (size_t j = 0; j < cols.size(); ++j) {
      double k = 2.0 * M_PI * freqs[cols[j]] / ctx->c;
      kc[2 * j] = k;
      kc[2 * j + 1] = mass_coefficient(k, ctx->h.gls_h);
    }
    HZ_HIP(hipMemcpyAsync(w.kc, kc.data(), sizeof(double) * 2 * w.s, hipMemcpyHostToDevice, q));
    HZ_HIP(hipStreamSynchronize(q));
    return HZ_OK;
  };
  {
    // set-up at the full width; the FP64 diagonal goes through R as scratch
    HZ_TRY(upload_kc(W, cs));
    k_in<<<ceil_div(W.total, kBlock), kBlock, 0, cs>>>(n, nrows, s, nf, D.perm.as<int>(), Pio, Fin, W.X, W.Fs);
    k_diag<T><<<ceil_div(W.total, kBlock), kBlock, 0, cs>>>(n, nrows, s, D.dpos.as<int>(), D.K64.as<double>(),
                                                           D.M64.as<double>(), D.eta ? D.E64.as<double>() : nullptr,
                                                           D.Bdiag.as<z_t>(), W.kc, W.R, W.dT);
    k_colnorm<double><<<W.Gr, kBlock, 0, cs>>>(W.total, s, W.Fs, W.part);
    k_colsum<<<s, kBlock, 0, cs>>>(W.Gr, s, W.part, W.cn);
    HZ_HIP(hipMemsetAsync(W.st, 0, sizeof(SlCol) * s, cs));
    k_sl_init<<<1, 64, 0, cs>>>(s, W.st, W.cn, o.tol);
    HZ_HIP(hipGetLastError());
    HZ_TRY(autotune<T>(ctx, cs, nrows, s, AT, W.kc, W.V.Z, W.V.u[1], &W.vin));
  }
  auto cycles_body = [&](hipStream_t q) -> int {
    const int s_ = W.s, Gr = W.Gr, eb = ceil_div(W.total, kBlock);
    const int64_t total = W.total;
    for (int it = 0; it < chunk; ++it) {
      for (int j = 0; j < l; ++j) {
        k_sl_u<T><<<eb, kBlock, 0, q>>>(total, s_, W.st, W.V, j);
        HZ_TRY((launch_spmm<T, false>(q, W.vin, nrows, s_, AT, W.kc, W.V.Z, nullptr, W.V.u[j + 1], nullptr,
                                      nullptr)));
        k_sl_dots<T, 2><<<Gr, kBlock, 0, q>>>(total, s_, W.st, W.V.rt, W.V.u[j + 1], W.part);
        k_sl_alpha<<<s_, kBlock, 0, q>>>(Gr, s_, W.st, W.part);
        k_sl_r<T><<<eb, kBlock, 0, q>>>(total, s_, W.st, W.V, j);
        HZ_TRY((launch_spmm<T, false>(q, W.vin, nrows, s_, AT, W.kc, W.V.Z, nullptr, W.V.r[j + 1], nullptr,
                                      nullptr)));
        if (j + 1 < l) {
          k_sl_dots<T, 2><<<Gr, kBlock, 0, q>>>(total, s_, W.st, W.V.rt, W.V.r[j + 1], W.part);
          k_sl_beta<<<s_, kBlock, 0, q>>>(Gr, s_, W.st, W.part);
        }
      }
      switch (l) {
        case 1: HZ_TRY((sl_enqueue_mr<T, 1>(q, W))); break;
        case 2: HZ_TRY((sl_enqueue_mr<T, 2>(q, W))); break;
        case 3: HZ_TRY((sl_enqueue_mr<T, 3>(q, W))); break;
        case 4: HZ_TRY((sl_enqueue_mr<T, 4>(q, W))); break;
        case 5: HZ_TRY((sl_enqueue_mr<T, 5>(q, W))); break;
        case 6: HZ_TRY((sl_enqueue_mr<T, 6>(q, W))); break;
        case 7: HZ_TRY((sl_enqueue_mr<T, 7>(q, W))); break;
        default: HZ_TRY((sl_enqueue_mr<T, 8>(q, W))); break;
      }
      k_sl_dots<T, 3><<<Gr, kBlock, 0, q>>>(total, s_, W.st, W.V.rt, W.V.r[0], W.part);
      k_sl_cycle<<<s_, kBlock, 0, q>>>(Gr, s_, W.st, W.part);
    }
    HZ_HIP(hipGetLastError());
    return HZ_OK;
  };
  auto outer = [&](hipStream_t q) -> int {
    const int s_ = W.s;
    const int64_t total = W.total;
    const int eb = ceil_div(total, kBlock);
    int nb = 0;
    k_sl_addx<T><<<eb, kBlock, 0, q>>>(total, s_, W.st, W.V, W.X);
    HZ_TRY((launch_spmm<double, true>(q, W.vres, nrows, s_, A64, W.kc, W.X, W.Fs, W.R, W.part, &nb)));
    k_sl_true<<<s_, kBlock, 0, q>>>(nb, s_, W.st, W.part, o.tol, delta);
    k_sl_start<T><<<eb, kBlock, 0, q>>>(total, s_, W.st, W.R, W.V);
    k_sl_start_fin<<<1, 64, 0, q>>>(s_, W.st);
    HZ_HIP(hipGetLastError());
    return HZ_OK;
  };

  std::unique_ptr<Graph> G(new Graph());
  HZ_TRY(G->stream(cs));
  HZ_TRY(G->capture(cycles_body));
  hipStream_t q = G->gs;
  void* hp = nullptr;
  HZ_TRY(ctx_pinned(ctx, sizeof(SlCol) * 64, &hp));
  SlCol* hs = static_cast<SlCol*>(hp);
  std::vector<hz_solve_info> res(nf);
  int worst = HZ_OK;
  auto record = [&](int j, double secs) {
    const SlCol& S = hs[j];
    hz_solve_info inf = {};
    const double fnv = std::sqrt(S.fn2);
    inf.relres_true = fnv > 0 ? S.beta / fnv : 0.0;
    inf.relres_est = inf.relres_true;
    inf.iters = S.iters;
    inf.matvecs = S.outer + 1;
    inf.inner_matvecs = 2 * l * S.iters;
    inf.seconds = secs;
    inf.status = S.nan ? HZ_BREAKDOWN : (S.done && inf.relres_true <= o.tol * (1 + 1e-12) ? HZ_OK : HZ_NOT_CONVERGED);
    if (!std::isfinite(inf.relres_true)) inf.status = HZ_BREAKDOWN;
    res[cols[j]] = inf;
  };
  int rc = 0;
  DevBuf* mapb = ctx->buf("swl.map", sizeof(int) * 128, &rc);
  if (rc) return rc;
  bool capped = false;
  for (;;) {
    HZ_HIP(hipMemcpyAsync(hs, W.st, sizeof(SlCol) * W.s, hipMemcpyDeviceToHost, q));
    HZ_HIP(hipStreamSynchronize(q));
    const int nreal = int(cols.size());
    int active = 0;
    bool pending = false;
    int64_t mx = 0;
    for (int j = 0; j < nreal; ++j) {
      const SlCol& S = hs[j];
      if (S.done || S.nan) continue;
      ++active;
      pending = pending || S.idone;
      mx = std::max<int64_t>(mx, 2 * int64_t(l) * S.iters + S.outer + 1);
    }
    if (active == 0) break;
    if (pending) {
      HZ_TRY(outer(q));
      continue;
    }
    // two products stay in reserve for the refinement step at the cap
    if (mx + 2 * int64_t(l) * chunk + 3 > o.max_matvec) {
      if (capped) break;
      capped = true;
      k_end_inner<SlCol><<<1, 64, 0, q>>>(W.s, W.st);
      HZ_TRY(outer(q));
      continue;
    }
    if (active <= W.s / 2) {
      // compaction: finished columns leave, the rest move to a narrower width
      std::vector<int> keep, gone_j, gone_f;
      for (int j = 0; j < nreal; ++j) {
        if (hs[j].done || hs[j].nan) {
          gone_j.push_back(j);
          gone_f.push_back(cols[j]);
        } else {
          keep.push_back(j);
        }
      }
      const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      for (int j : gone_j) record(j, secs);
      if (!gone_j.empty()) {
        std::vector<int> h2(gone_j);
        h2.insert(h2.end(), gone_f.begin(), gone_f.end());
        HZ_HIP(hipMemcpyAsync(mapb->p, h2.data(), sizeof(int) * h2.size(), hipMemcpyHostToDevice, q));
        const int ng = int(gone_j.size());
        k_out_cols<<<ceil_div(n * ng, kBlock), kBlock, 0, q>>>(n, W.s, nf, ng, D.perm.as<int>(), mapb->as<int>(),
                                                                mapb->as<int>() + ng, W.X, Pio);
        HZ_HIP(hipGetLastError());
        HZ_HIP(hipStreamSynchronize(q));
      }
      int s2 = 1;
      while (s2 < int(keep.size())) s2 <<= 1;
      SlWidth<T> W2;
      HZ_TRY(sl_alloc<T>(ctx, nrows, s2, l, &W2));
      std::vector<int> map(s2, -1);
      for (size_t jn = 0; jn < keep.size(); ++jn) map[jn] = keep[jn];
      HZ_HIP(hipMemcpyAsync(mapb->p, map.data(), sizeof(int) * s2, hipMemcpyHostToDevice, q));
      const int gb = ceil_div(nrows * s2, kBlock);
      const int* mp = mapb->as<int>();
      k_gather_cols<z_t><<<gb, kBlock, 0, q>>>(nrows, W.s, s2, mp, W.X, W2.X);
      k_gather_cols<z_t><<<gb, kBlock, 0, q>>>(nrows, W.s, s2, mp, W.Fs, W2.Fs);
      k_gather_cols<cx<T>><<<gb, kBlock, 0, q>>>(nrows, W.s, s2, mp, W.dT, W2.dT);
      k_gather_cols<cx<T>><<<gb, kBlock, 0, q>>>(nrows, W.s, s2, mp, W.V.y, W2.V.y);
      k_gather_cols<cx<T>><<<gb, kBlock, 0, q>>>(nrows, W.s, s2, mp, W.V.rt, W2.V.rt);
      for (int i = 0; i <= l; ++i) {
        k_gather_cols<cx<T>><<<gb, kBlock, 0, q>>>(nrows, W.s, s2, mp, W.V.r[i], W2.V.r[i]);
        k_gather_cols<cx<T>><<<gb, kBlock, 0, q>>>(nrows, W.s, s2, mp, W.V.u[i], W2.V.u[i]);
      }
      HZ_HIP(hipGetLastError());
      std::vector<SlCol> ns(s2);
      for (int jn = 0; jn < s2; ++jn) {
        if (map[jn] >= 0) {
          ns[jn] = hs[map[jn]];
        } else {
          ns[jn] = SlCol{};
          ns[jn].done = 1;
        }
      }
      std::vector<int> ncols;
      for (int j : keep) ncols.push_back(cols[j]);
      cols = ncols;
      HZ_HIP(hipMemcpyAsync(W2.st, ns.data(), sizeof(SlCol) * s2, hipMemcpyHostToDevice, q));
      HZ_TRY(upload_kc(W2, q));
      HZ_TRY(autotune<T>(ctx, q, nrows, s2, AT, W2.kc, W2.V.Z, W2.V.u[1], &W2.vin));
      W = W2;
      // new graph ordered after the old stream; the old graph and stream go once idle
      std::unique_ptr<Graph> G2(new Graph());
      HZ_TRY(G2->stream(q));
      HZ_TRY(G2->capture(cycles_body));
      HZ_HIP(hipStreamSynchronize(q));
      G = std::move(G2);
      q = G->gs;
      continue;
    }
    HZ_TRY(G->launch());
  }
  // remaining columns: copy out and record
  HZ_HIP(hipMemcpyAsync(hs, W.st, sizeof(SlCol) * W.s, hipMemcpyDeviceToHost, q));
  HZ_HIP(hipStreamSynchronize(q));
  {
    const int nreal = int(cols.size());
    std::vector<int> h2(2 * nreal);
    for (int j = 0; j < nreal; ++j) {
      h2[j] = j;
      h2[nreal + j] = cols[j];
    }
    if (nreal > 0) {
      HZ_HIP(hipMemcpyAsync(mapb->p, h2.data(), sizeof(int) * h2.size(), hipMemcpyHostToDevice, q));
      k_out_cols<<<ceil_div(n * nreal, kBlock), kBlock, 0, q>>>(n, W.s, nf, nreal, D.perm.as<int>(), mapb->as<int>(),
                                                                 mapb->as<int>() + nreal, W.X, Pio);
      HZ_HIP(hipGetLastError());
      HZ_HIP(hipStreamSynchronize(q));
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int j = 0; j < nreal; ++j) record(j, secs);
  }
  for (int f = 0; f < nf; ++f) {
    worst = std::max(worst, res[f].status);
    if (infos) infos[f] = res[f];
  }
  return worst;
}

// ---------------------------------------------------------------- batched transpose-free QMR
// Each column runs Freund's TFQMR (the pair of half-steps of the
// single-system solver) on the correction equation B(k_c) y = R_c / scale_c;
// when its quasi-residual bound meets the inner target the column applies
// its last update and the host runs the refinement step (X += scale D^-1 y,
// R = F - A X in FP64): done, or restart.  A breakdown also ends the inner
// solve with a refinement step.
// Stagnation test of complex64 inner TFQMR solves: checkpoint spacing in
// half-steps (a bound that has not halved over one spacing ends the solve).
constexpr int kTsStagHalfSteps = 4096;

struct TsCol {
  z_t alpha, rho, beta, eta;
  double theta, tau, ithr, fn2, thr2, scale, beta_true, rr;
  double chk;    // quasi-residual bound at the last stagnation checkpoint
  int done, idone, nan, m, iters, outer, restart_now, last;
  int mchk;      // half-step count at that checkpoint
  int stag;      // checkpoint spacing in half-steps (0: no stagnation test)
  // The even half-step's d = u + ge d and the odd half-step's x-update are
  // applied late, in the next odd kernel (d holds the previous odd
  // half-step's d until then): ge and that odd half-step's eta are kept
  // here, and yp marks an odd x-update not yet applied (the refinement step
  // adds it when the column stops between pairs).
  z_t ge, eta_o;
  int yp, pad;
};

// Diagonal of A(k_c) recomputed per element from four (five with an
// absorption field) real values per row and the column's (k, m(k)), in place
// of a stored n x s table of D^-1:
//   A(k)_rr = K_rr - m(k) M_rr - k Im(B_rr) + i (k Re(B_rr) + m(k) E_rr).
// Padding rows hold (1, 0, 0, 0): diagonal 1.
struct TsDiag {
  const double4* a;   // (K_rr, M_rr, Re B_rr, Im B_rr) per row
  const double* e;    // E_rr per row, or null
  const double* kc;   // (k, m(k)) per column
  int ls;             // log2 of the width
};

__device__ __forceinline__ z_t ts_dg(const TsDiag& G, int64_t row, double k, double k2) {
  const double4 r = G.a[row];
  return z_t{r.x - k2 * r.y - k * r.w, k * r.z + (G.e ? k2 * G.e[row] : 0.0)};
}

// 1 / d as conj(d) / |d|^2: one division (a diagonal entry of these
// operators is far from the range where |d|^2 over- or underflows)
__device__ __forceinline__ z_t ts_inv(z_t d) {
  const double q = 1.0 / fma(d.re, d.re, d.im * d.im);
  return z_t{d.re * q, -d.im * q};
}

__global__ void k_ts_rowdiag(int64_t n, int64_t nrows, const int* __restrict__ dpos, const double* __restrict__ K,
                             const double* __restrict__ M, const double* __restrict__ E, const z_t* __restrict__ Bd,
                             double4* __restrict__ a, double* __restrict__ e) {
  int64_t row = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (row >= nrows) return;
  if (row < n) {
    const int64_t p = dpos[row];
    a[row] = double4{K[p], M[p], Bd[row].re, Bd[row].im};
    if (e) e[row] = E[p];
  } else {
    a[row] = double4{1.0, 0.0, 0.0, 0.0};
    if (e) e[row] = 0.0;
  }
}

// The two product inputs are stored already scaled by D^-1 (right Jacobi:
// B = A D^-1): u holds D^-1 u and un holds D^-1 un; a kernel that needs u or
// un itself multiplies by the diagonal.
template <typename T>
struct TsVec {
  cx<T>* y;      // inner iterate (scaled unknowns)
  cx<T>* rs;     // shadow vector
  cx<T>* w;
  cx<T>* u;      // D^-1 u at the start of a pair of half-steps (odd product's input)
  cx<T>* un;     // D^-1 un, un = u after the even half-step (even product's input)
  cx<T>* v;
  cx<T>* uhe;    // B un = A (D^-1 un) (product of the even half-step)
  cx<T>* uh;     // B u (product of the odd half-step, or of a restart)
  cx<T>* d;
  TsDiag G;
};

__device__ __forceinline__ bool ts_off(const TsCol& S) { return S.done || S.idone || S.nan; }
__device__ __forceinline__ bool ts_pending(const TsCol& S) { return S.idone && !S.done && !S.nan; }
// x-update of a half-step: always while active, once more right after the stop
__device__ __forceinline__ bool ts_apply(const TsCol& S) { return !S.done && !S.nan && (!S.idone || S.last); }

template <typename T>
__global__ void k_ts_addx(int64_t total, int s, const TsCol* __restrict__ st, TsVec<T> V, z_t* __restrict__ X) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= total) return;
  const int c = int(e & (s - 1));
  const TsCol& S = st[c];
  if (!ts_pending(S) || S.scale == 0.0) return;
  const z_t iv = ts_inv(ts_dg(V.G, e >> V.G.ls, V.G.kc[2 * c], V.G.kc[2 * c + 1]));
  z_t y = ccast<double>(V.y[e]);
  if (S.yp) y = y + S.eta * ccast<double>(V.d[e]);
  z_t d = iv * y;
  X[e] = z_t{fma(S.scale, d.re, X[e].re), fma(S.scale, d.im, X[e].im)};
}

__global__ void k_ts_true(int nblk, int s, TsCol* st, const double* __restrict__ part, double tol, double delta) {
  __shared__ double lds[kBlock / kWave];
  const int c = blockIdx.x;
  const int pend = ts_pending(st[c]);
  __syncthreads();
  if (!pend) return;
  const double rr = block_sum_strided(part + c, nblk, s, lds);
  if (threadIdx.x != 0) return;
  TsCol& S = st[c];
  const double b = sqrt(rr);
  S.beta_true = b;
  S.yp = 0;        // k_ts_addx has applied any deferred x-update
  S.nan = S.nan || !isfinite(rr);
  S.done = (rr <= S.thr2) || S.fn2 == 0.0 || S.nan;
  if (S.done) return;
  S.outer += 1;
  S.idone = 0;
  S.last = 0;
  S.restart_now = 1;
  S.scale = b;
  const double lim = 0.5 * tol * sqrt(S.fn2) / b;
  S.ithr = delta > lim ? delta : lim;
}

// restart: r0 = R / scale; r* = w = u = r0 (u stored as D^-1 u); d = y = 0
template <typename T>
__global__ void k_ts_start(int64_t total, int s, const TsCol* __restrict__ st, const z_t* __restrict__ R,
                           TsVec<T> V) {
  int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= total) return;
  const int c = int(e & (s - 1));
  const TsCol& S = st[c];
  if (!S.restart_now) return;
  const cx<T> r = ccast<T>((1.0 / S.scale) * R[e]);
  const cx<T> z = {T(0), T(0)};
  const z_t iv = ts_inv(ts_dg(V.G, e >> V.G.ls, V.G.kc[2 * c], V.G.kc[2 * c + 1]));
  V.rs[e] = r;
  V.w[e] = r;
  V.u[e] = ccast<T>(iv * ccast<double>(r));
  V.d[e] = z;
  V.y[e] = z;
}

// after the restart product uh = B u: v = uh; partial r*^H v
template <typename T>
__global__ void __launch_bounds__(kBlock) k_ts_v0(int64_t total, int s, const TsCol* __restrict__ st, TsVec<T> V,
                                                  double* __restrict__ part) {
  __shared__ double lds[4 * kWave];
  const int c = threadIdx.x & (s - 1);
  double q[2] = {0.0, 0.0};
  if (st[c].restart_now) {
    for (int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x; e < total; e += int64_t(gridDim.x) * kBlock) {
      const cx<T> v = V.uh[e];
      V.v[e] = v;
      const z_t a = ccast<double>(V.rs[e]), b = ccast<double>(v);
      q[0] = fma(a.re, b.re, fma(a.im, b.im, q[0]));
      q[1] = fma(a.re, b.im, fma(-a.im, b.re, q[1]));
    }
  }
  for (int i = 0; i < 2; ++i) {
    const double t = col_reduce(q[i], s, lds);
    if (int(threadIdx.x) < s) part[(int64_t(blockIdx.x) * 2 + i) * s + threadIdx.x] = t;
  }
}

__global__ void k_ts_start_fin(int G_, int s, TsCol* st, const double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  const int c = blockIdx.x;
  const int go = st[c].restart_now;
  __syncthreads();
  if (!go) return;
  const double re = sl_sum(G_, s, 2, part, c, 0, lds);
  const double im = sl_sum(G_, s, 2, part, c, 1, lds);
  if (threadIdx.x != 0) return;
  TsCol& S = st[c];
  S.restart_now = 0;
  S.rr = 1.0;
  S.tau = 1.0;                      // ||R / scale||
  S.theta = 0.0;
  S.eta = z_t{0.0, 0.0};
  S.eta_o = z_t{0.0, 0.0};
  S.ge = z_t{0.0, 0.0};
  S.yp = 0;
  S.rho = z_t{1.0, 0.0};            // r*^H r0
  S.m = 0;
  S.chk = 1.0;
  S.mchk = 0;
  const z_t sg = {re, im};
  if (norm2(sg) == 0.0 || !isfinite(re) || !isfinite(im)) S.nan = 1;
  else S.alpha = cdiv(S.rho, sg);
}

__device__ __forceinline__ void ts_qmr(TsCol& S, double ww) {
  S.theta = sqrt(ww) / S.tau;
  const double c2 = 1.0 / (1.0 + S.theta * S.theta);
  S.tau = S.tau * S.theta * sqrt(c2);
  S.eta = c2 * S.alpha;
  S.iters += 1;
  if (!isfinite(ww)) {
    S.nan = 1;
    return;
  }
  const double bound = S.tau * sqrt(double(S.m + 1));
  if (bound <= S.ithr) {
    S.idone = 1;
    S.last = 1;
  } else if (S.stag > 0 && S.m - S.mchk >= S.stag) {
    // complex64 inner solve: a bound that has not halved over the last
    // checkpoint interval ends the inner solve, so the refinement step adds
    // the correction reached so far and restarts from the FP64 residual
    if (bound > 0.5 * S.chk) {
      S.idone = 1;
      S.last = 1;
    }
    S.chk = bound;
    S.mchk = S.m;
  }
  S.m += 1;
}

// Buffers of a pair of half-steps: u holds D^-1 u at the start of the pair,
// the even half-step writes D^-1 un into un (never copied back: the odd
// half-step reads it and writes the next D^-1 u into u), the even product
// writes uhe and the odd (or restart) product writes uh, so the odd
// half-step's v needs no staging; d keeps the odd half-steps' d only (the
// even half-step's is rebuilt from u where it is used).
// even half-step, part 1: un = u - alpha v (stored as D^-1 un, the even
// product's input; unused if the column stops); w -= alpha uh;
// partial ||w||^2
template <typename T>
__global__ void __launch_bounds__(kBlock) k_ts_even1(int64_t total, int s, const TsCol* __restrict__ st, TsVec<T> V,
                                                     double* __restrict__ part) {
  __shared__ double lds[4 * kWave];
  const int c = threadIdx.x & (s - 1);
  const TsCol& S = st[c];
  double ww = 0.0;
  if (!ts_off(S)) {
    const z_t a = S.alpha;
    const double k = V.G.kc[2 * c], k2 = V.G.kc[2 * c + 1];
    for (int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x; e < total; e += int64_t(gridDim.x) * kBlock) {
      const z_t dg = ts_dg(V.G, e >> V.G.ls, k, k2);
      const z_t u = dg * ccast<double>(V.u[e]);
      V.un[e] = ccast<T>(ts_inv(dg) * (u - a * ccast<double>(V.v[e])));
      const cx<T> w = ccast<T>(ccast<double>(V.w[e]) - a * ccast<double>(V.uh[e]));
      V.w[e] = w;
      ww += norm2(ccast<double>(w));
    }
  }
  const double t = col_reduce(ww, s, lds);
  if (int(threadIdx.x) < s) part[int64_t(blockIdx.x) * s + threadIdx.x] = t;
}

__global__ void k_ts_qmr_fin(int G_, int s, TsCol* st, const double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  const int c = blockIdx.x;
  const int off = ts_off(st[c]), idn = st[c].idone;
  __syncthreads();
  if (off) {
    if (threadIdx.x == 0 && idn) st[c].last = 0;
    return;
  }
  const double ww = sl_sum(G_, s, 1, part, c, 0, lds);
  if (threadIdx.x != 0) return;
  TsCol& S = st[c];
  S.ge = (S.theta * S.theta) * cdiv(S.eta, S.alpha);   // the even half-step's d = u + ge d
  S.eta_o = S.eta;                                      // the previous odd half-step's eta
  ts_qmr(S, ww);
}

// odd half-step, part 1, with the x-updates of the previous odd half-step
// and of the even half-step folded in (while the even half-step applies):
// de = u + ge d (the even half-step's d; d holds the previous odd's);
// y += eta_o d + eta de; then (column running) w -= alpha uhe;
// d = un + g de; partials ||w||^2, r*^H w
template <typename T>
__global__ void __launch_bounds__(kBlock) k_ts_odd1(int64_t total, int s, const TsCol* __restrict__ st, TsVec<T> V,
                                                    double* __restrict__ part) {
  __shared__ double lds[4 * kWave];
  const int c = threadIdx.x & (s - 1);
  const TsCol& S = st[c];
  double q[3] = {0.0, 0.0, 0.0};
  const bool run = !ts_off(S);
  if (ts_apply(S)) {
    const z_t eta = S.eta, eta_o = S.eta_o, ge = S.ge;
    const z_t a = S.alpha;
    const z_t g = run ? (S.theta * S.theta) * cdiv(S.eta, a) : z_t{0.0, 0.0};
    const double k = V.G.kc[2 * c], k2 = V.G.kc[2 * c + 1];
    for (int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x; e < total; e += int64_t(gridDim.x) * kBlock) {
      const z_t dg = ts_dg(V.G, e >> V.G.ls, k, k2);
      const z_t dold = ccast<double>(V.d[e]);
      const z_t dv = dg * ccast<double>(V.u[e]) + ge * dold;
      V.y[e] = ccast<T>(ccast<double>(V.y[e]) + (eta_o * dold + eta * dv));
      if (!run) continue;
      const cx<T> w = ccast<T>(ccast<double>(V.w[e]) - a * ccast<double>(V.uhe[e]));
      V.w[e] = w;
      const z_t un = dg * ccast<double>(V.un[e]);
      V.d[e] = ccast<T>(un + g * dv);
      const z_t wv = ccast<double>(w), r = ccast<double>(V.rs[e]);
      q[0] += norm2(wv);
      q[1] = fma(r.re, wv.re, fma(r.im, wv.im, q[1]));
      q[2] = fma(r.re, wv.im, fma(-r.im, wv.re, q[2]));
    }
  }
  for (int i = 0; i < 3; ++i) {
    const double t = col_reduce(q[i], s, lds);
    if (int(threadIdx.x) < s) part[(int64_t(blockIdx.x) * 3 + i) * s + threadIdx.x] = t;
  }
}

__global__ void k_ts_odd_fin(int G_, int s, TsCol* st, const double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  const int c = blockIdx.x;
  const int off = ts_off(st[c]), idn = st[c].idone;
  __syncthreads();
  if (off) {
    if (threadIdx.x == 0 && idn) {
      if (st[c].last) st[c].yp = 0;     // k_ts_odd1 applied the deferred x-update
      st[c].last = 0;
    }
    return;
  }
  const double ww = sl_sum(G_, s, 3, part, c, 0, lds);
  const double re = sl_sum(G_, s, 3, part, c, 1, lds);
  const double im = sl_sum(G_, s, 3, part, c, 2, lds);
  if (threadIdx.x != 0) return;
  TsCol& S = st[c];
  ts_qmr(S, ww);
  const z_t rho1 = {re, im};
  if (norm2(S.rho) == 0.0 || !isfinite(re) || !isfinite(im)) {
    if (!S.idone) {
      S.idone = 1;       // breakdown: refinement step and restart
      S.last = 1;
    }
  } else {
    S.beta = cdiv(rho1, S.rho);
    S.rho = rho1;
  }
  S.yp = S.idone ? 0 : 1;   // a running column defers this half-step's x-update
}

// odd half-step, part 2: a column stopping here applies its x-update
// y += eta d now; a running one defers it and forms u = w + beta un, stored
// as D^-1 u = D^-1 w + beta (D^-1 un)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_ts_odd2(int64_t total, int s, const TsCol* __restrict__ st, TsVec<T> V) {
  const int c = threadIdx.x & (s - 1);
  const TsCol& S = st[c];
  if (!ts_apply(S)) return;
  const int64_t e0 = int64_t(blockIdx.x) * kBlock + threadIdx.x, stride = int64_t(gridDim.x) * kBlock;
  if (S.idone) {
    const z_t eta = S.eta;
    for (int64_t e = e0; e < total; e += stride)
      V.y[e] = ccast<T>(ccast<double>(V.y[e]) + eta * ccast<double>(V.d[e]));
    return;
  }
  const z_t b = S.beta;
  const double k = V.G.kc[2 * c], k2 = V.G.kc[2 * c + 1];
  for (int64_t e = e0; e < total; e += stride) {
    const z_t iv = ts_inv(ts_dg(V.G, e >> V.G.ls, k, k2));
    V.u[e] = ccast<T>(iv * ccast<double>(V.w[e]) + b * ccast<double>(V.un[e]));
  }
}

// odd half-step, part 3 (after uh = B u): v = uh + beta uhe + beta^2 v; partial r*^H v
template <typename T>
__global__ void __launch_bounds__(kBlock) k_ts_odd3(int64_t total, int s, const TsCol* __restrict__ st, TsVec<T> V,
                                                    double* __restrict__ part) {
  __shared__ double lds[4 * kWave];
  const int c = threadIdx.x & (s - 1);
  double q[2] = {0.0, 0.0};
  if (!ts_off(st[c])) {
    const z_t bt = st[c].beta;
    const z_t bt2 = bt * bt;
    for (int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x; e < total; e += int64_t(gridDim.x) * kBlock) {
      const cx<T> v = ccast<T>(ccast<double>(V.uh[e]) + (bt * ccast<double>(V.uhe[e]) + bt2 * ccast<double>(V.v[e])));
      V.v[e] = v;
      const z_t a = ccast<double>(V.rs[e]), b = ccast<double>(v);
      q[0] = fma(a.re, b.re, fma(a.im, b.im, q[0]));
      q[1] = fma(a.re, b.im, fma(-a.im, b.re, q[1]));
    }
  }
  for (int i = 0; i < 2; ++i) {
    const double t = col_reduce(q[i], s, lds);
    if (int(threadIdx.x) < s) part[(int64_t(blockIdx.x) * 2 + i) * s + threadIdx.x] = t;
  }
}

__global__ void k_ts_alpha_fin(int G_, int s, TsCol* st, const double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  const int c = blockIdx.x;
  const int off = ts_off(st[c]), idn = st[c].idone;
  __syncthreads();
  if (off) {
    if (threadIdx.x == 0 && idn) st[c].last = 0;
    return;
  }
  const double re = sl_sum(G_, s, 2, part, c, 0, lds);
  const double im = sl_sum(G_, s, 2, part, c, 1, lds);
  if (threadIdx.x != 0) return;
  TsCol& S = st[c];
  const z_t sg = {re, im};
  if (norm2(sg) == 0.0 || !isfinite(re) || !isfinite(im)) S.idone = 1;   // refinement step and restart
  else S.alpha = cdiv(S.rho, sg);
}

__global__ void k_ts_init(int s, TsCol* st, const double* fn2, double tol, int stag) {
  const int c = threadIdx.x;
  if (c >= s) return;
  st[c].fn2 = fn2[c];
  st[c].thr2 = tol * tol * fn2[c];
  st[c].stag = stag;
  st[c].idone = 1;                 // every column starts with a refinement step
}

constexpr int kTsVecs = 9;   // column vectors of a width (TsVec's pointers)

template <typename T>
struct TsWidth {
  int s = 0, Gr = 1;
  int64_t total = 0;
  z_t *X = nullptr, *Fs = nullptr, *R = nullptr;
  double *kc = nullptr, *part = nullptr, *cn = nullptr;
  TsCol* st = nullptr;
  TsVec<T> V;
  Variant vin, vres;
};

template <typename T>
int ts_alloc(hz_ctx ctx, int64_t nrows, int s, const double4* rda, const double* rde, TsWidth<T>* W) {
  int rc = 0;
  const std::string p = std::string("swt.") + (sizeof(T) == 8 ? "z." : "c.") + std::to_string(s) + ".";
  const int64_t total = nrows * s;
  auto buf = [&](const std::string& nm, size_t bytes) -> void* {
    DevBuf* b = ctx->buf(p + nm, bytes, &rc);
    return rc ? nullptr : b->p;
  };
  W->s = s;
  W->total = total;
  W->Gr = int(std::min<int64_t>(std::max<int64_t>(total / kBlock, 1), 1024));
  const int64_t nblk_res = (nrows + kBlock / s - 1) / (kBlock / s);
  W->X = static_cast<z_t*>(buf("X", sizeof(z_t) * total));
  W->Fs = static_cast<z_t*>(buf("F", sizeof(z_t) * total));
  W->R = static_cast<z_t*>(buf("R", sizeof(z_t) * total));
  W->kc = static_cast<double*>(buf("kc", sizeof(double) * 2 * s));
  W->cn = static_cast<double*>(buf("cn", sizeof(double) * s));
  W->part = static_cast<double*>(buf("part", sizeof(double) * std::max<int64_t>(int64_t(W->Gr) * 3, nblk_res) * s));
  W->st = static_cast<TsCol*>(buf("st", sizeof(TsCol) * s));
  W->V = TsVec<T>{};
  cx<T>** vv[kTsVecs] = {&W->V.y, &W->V.rs, &W->V.w, &W->V.u, &W->V.un, &W->V.v, &W->V.uhe, &W->V.uh, &W->V.d};
  const char* names[kTsVecs] = {"y", "rs", "w", "u", "un", "v", "uhe", "uh", "d"};
  for (int i = 0; i < kTsVecs; ++i) *vv[i] = static_cast<cx<T>*>(buf(names[i], sizeof(cx<T>) * total));
  if (rc) return rc;
  int ls = 0;
  while ((1 << ls) < s) ++ls;
  W->V.G = TsDiag{rda, rde, W->kc, ls};
  W->vres.cpl = 1;
  W->vres.bs = kBlock;
  return HZ_OK;
}

template <typename T>
int run_sweep_tfqmr(hz_ctx ctx, SweepData& D, int nf, const double* freqs, const z_t* Fin, z_t* Pio,
                    const hz_solve_opts& o, hz_solve_info* infos) {
  auto t0 = std::chrono::steady_clock::now();
  const double delta = sizeof(T) == 4 ? (o.inner_tol > 0 ? o.inner_tol : 1e-3) : 0.0;
  const int chunk = 16;                         // pairs of half-steps per graph launch
  const int64_t nrows = D.nrows, n = ctx->h.n;
  const RowOp<double> A64 = row_op<double>(D);
  const RowOp<T> AT = row_op<T>(D);
  int s = 1;
  while (s < nf) s <<= 1;
  int rc = 0;
  DevBuf* rdab = ctx->buf("swt.rda", sizeof(double4) * nrows, &rc);
  if (rc) return rc;
  DevBuf* rdeb = nullptr;
  if (D.eta) {
    rdeb = ctx->buf("swt.rde", sizeof(double) * nrows, &rc);
    if (rc) return rc;
  }
  const double4* rda = static_cast<const double4*>(rdab->p);
  const double* rde = rdeb ? static_cast<const double*>(rdeb->p) : nullptr;
  TsWidth<T> W;
  HZ_TRY(ts_alloc<T>(ctx, nrows, s, rda, rde, &W));
  hipStream_t cs = ctx->stream;
  std::vector<int> cols(nf);
  for (int c = 0; c < nf; ++c) cols[c] = c;
  auto upload_kc = [&](TsWidth<T>& w, hipStream_t q) -> int {
    std::vector<double> kc(2 * w.s, 0.0);
    for (size_t j = 0; j < cols.size(); ++j) {
      double k = 2.0 * M_PI * freqs[cols[j]] / ctx->c;
      kc[2 * j] = k;
      kc[2 * j + 1] = mass_coefficient(k, ctx->h.gls_h);
    }
    HZ_HIP(hipMemcpyAsync(w.kc, kc.data(), sizeof(double) * 2 * w.s, hipMemcpyHostToDevice, q));
    HZ_HIP(hipStreamSynchronize(q));
    return HZ_OK;
  };
  HZ_TRY(upload_kc(W, cs));
  k_in<<<ceil_div(W.total, kBlock), kBlock, 0, cs>>>(n, nrows, s, nf, D.perm.as<int>(), Pio, Fin, W.X, W.Fs);
  k_ts_rowdiag<<<ceil_div(nrows, kBlock), kBlock, 0, cs>>>(n, nrows, D.dpos.as<int>(), D.K64.as<double>(),
                                                           D.M64.as<double>(), D.eta ? D.E64.as<double>() : nullptr,
                                                           D.Bdiag.as<z_t>(), static_cast<double4*>(rdab->p),
                                                           rdeb ? static_cast<double*>(rdeb->p) : nullptr);
  k_colnorm<double><<<W.Gr, kBlock, 0, cs>>>(W.total, s, W.Fs, W.part);
  k_colsum<<<s, kBlock, 0, cs>>>(W.Gr, s, W.part, W.cn);
  HZ_HIP(hipMemsetAsync(W.st, 0, sizeof(TsCol) * s, cs));
  k_ts_init<<<1, 64, 0, cs>>>(s, W.st, W.cn, o.tol, sizeof(T) == 4 ? kTsStagHalfSteps : 0);
  HZ_HIP(hipGetLastError());
  HZ_TRY(autotune<T>(ctx, cs, nrows, s, AT, W.kc, W.V.u, W.V.uh, &W.vin));

  auto pairs_body = [&](hipStream_t q) -> int {
    const int s_ = W.s, Gr = W.Gr;
    const int64_t total = W.total;
    for (int it = 0; it < chunk; ++it) {
      k_ts_even1<T><<<Gr, kBlock, 0, q>>>(total, s_, W.st, W.V, W.part);
      k_ts_qmr_fin<<<s_, kBlock, 0, q>>>(Gr, s_, W.st, W.part);
      HZ_TRY((launch_spmm<T, false>(q, W.vin, nrows, s_, AT, W.kc, W.V.un, nullptr, W.V.uhe, nullptr, nullptr)));
      k_ts_odd1<T><<<Gr, kBlock, 0, q>>>(total, s_, W.st, W.V, W.part);
      k_ts_odd_fin<<<s_, kBlock, 0, q>>>(Gr, s_, W.st, W.part);
      k_ts_odd2<T><<<Gr, kBlock, 0, q>>>(total, s_, W.st, W.V);
      HZ_TRY((launch_spmm<T, false>(q, W.vin, nrows, s_, AT, W.kc, W.V.u, nullptr, W.V.uh, nullptr, nullptr)));
      k_ts_odd3<T><<<Gr, kBlock, 0, q>>>(total, s_, W.st, W.V, W.part);
      k_ts_alpha_fin<<<s_, kBlock, 0, q>>>(Gr, s_, W.st, W.part);
    }
    HZ_HIP(hipGetLastError());
    return HZ_OK;
  };
  auto outer = [&](hipStream_t q) -> int {
    const int s_ = W.s;
    const int64_t total = W.total;
    const int eb = ceil_div(total, kBlock);
    int nb = 0;
    k_ts_addx<T><<<eb, kBlock, 0, q>>>(total, s_, W.st, W.V, W.X);
    HZ_TRY((launch_spmm<double, true>(q, W.vres, nrows, s_, A64, W.kc, W.X, W.Fs, W.R, W.part, &nb)));
    k_ts_true<<<s_, kBlock, 0, q>>>(nb, s_, W.st, W.part, o.tol, delta);
    k_ts_start<T><<<eb, kBlock, 0, q>>>(total, s_, W.st, W.R, W.V);
    HZ_TRY((launch_spmm<T, false>(q, W.vin, nrows, s_, AT, W.kc, W.V.u, nullptr, W.V.uh, nullptr, nullptr)));
    k_ts_v0<T><<<W.Gr, kBlock, 0, q>>>(total, s_, W.st, W.V, W.part);
    k_ts_start_fin<<<s_, kBlock, 0, q>>>(W.Gr, s_, W.st, W.part);
    HZ_HIP(hipGetLastError());
    return HZ_OK;
  };

  std::unique_ptr<Graph> G(new Graph());
  HZ_TRY(G->stream(cs));
  HZ_TRY(G->capture(pairs_body));
  hipStream_t q = G->gs;
  void* hp = nullptr;
  HZ_TRY(ctx_pinned(ctx, sizeof(TsCol) * 64, &hp));
  TsCol* hs = static_cast<TsCol*>(hp);
  std::vector<hz_solve_info> res(nf);
  int worst = HZ_OK;
  auto record = [&](int j, double secs) {
    const TsCol& S = hs[j];
    hz_solve_info inf = {};
    const double fnv = std::sqrt(S.fn2);
    inf.relres_true = fnv > 0 ? S.beta_true / fnv : 0.0;
    inf.relres_est = inf.relres_true;
    inf.iters = S.iters;
    inf.matvecs = S.outer + 1;
    inf.inner_matvecs = S.iters + S.outer;
    inf.seconds = secs;
    inf.status = S.nan ? HZ_BREAKDOWN : (S.done && inf.relres_true <= o.tol * (1 + 1e-12) ? HZ_OK : HZ_NOT_CONVERGED);
    if (!std::isfinite(inf.relres_true)) inf.status = HZ_BREAKDOWN;
    res[cols[j]] = inf;
  };
  DevBuf* mapb = ctx->buf("swt.map", sizeof(int) * 128, &rc);
  if (rc) return rc;
  bool capped = false;
  for (;;) {
    HZ_HIP(hipMemcpyAsync(hs, W.st, sizeof(TsCol) * W.s, hipMemcpyDeviceToHost, q));
    HZ_HIP(hipStreamSynchronize(q));
    const int nreal = int(cols.size());
    int active = 0;
    bool pending = false;
    int64_t mx = 0;
    for (int j = 0; j < nreal; ++j) {
      const TsCol& S = hs[j];
      if (S.done || S.nan) continue;
      ++active;
      pending = pending || S.idone;
      mx = std::max<int64_t>(mx, int64_t(S.iters) + 2 * int64_t(S.outer) + 1);
    }
    if (active == 0) break;
    if (pending) {
      HZ_TRY(outer(q));
      continue;
    }
    // two products stay in reserve for the refinement step at the cap
    if (mx + 2 * chunk + 3 > o.max_matvec) {
      if (capped) break;
      capped = true;
      k_end_inner<TsCol><<<1, 64, 0, q>>>(W.s, W.st);
      HZ_TRY(outer(q));
      continue;
    }
    if (active <= W.s / 2) {
      std::vector<int> keep, gone_j, gone_f;
      for (int j = 0; j < nreal; ++j) {
        if (hs[j].done || hs[j].nan) {
          gone_j.push_back(j);
          gone_f.push_back(cols[j]);
        } else {
          keep.push_back(j);
        }
      }
      const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      for (int j : gone_j) record(j, secs);
      if (!gone_j.empty()) {
        std::vector<int> h2(gone_j);
        h2.insert(h2.end(), gone_f.begin(), gone_f.end());
        HZ_HIP(hipMemcpyAsync(mapb->p, h2.data(), sizeof(int) * h2.size(), hipMemcpyHostToDevice, q));
        const int ng = int(gone_j.size());
        k_out_cols<<<ceil_div(n * ng, kBlock), kBlock, 0, q>>>(n, W.s, nf, ng, D.perm.as<int>(), mapb->as<int>(),
                                                                mapb->as<int>() + ng, W.X, Pio);
        HZ_HIP(hipGetLastError());
        HZ_HIP(hipStreamSynchronize(q));
      }
      int s2 = 1;
      while (s2 < int(keep.size())) s2 <<= 1;
      TsWidth<T> W2;
      HZ_TRY(ts_alloc<T>(ctx, nrows, s2, rda, rde, &W2));
      std::vector<int> map(s2, -1);
      for (size_t jn = 0; jn < keep.size(); ++jn) map[jn] = keep[jn];
      HZ_HIP(hipMemcpyAsync(mapb->p, map.data(), sizeof(int) * s2, hipMemcpyHostToDevice, q));
      const int gb = ceil_div(nrows * s2, kBlock);
      const int* mp = mapb->as<int>();
      k_gather_cols<z_t><<<gb, kBlock, 0, q>>>(nrows, W.s, s2, mp, W.X, W2.X);
      k_gather_cols<z_t><<<gb, kBlock, 0, q>>>(nrows, W.s, s2, mp, W.Fs, W2.Fs);
      cx<T>* from[kTsVecs] = {W.V.y, W.V.rs, W.V.w, W.V.u, W.V.un, W.V.v, W.V.uhe, W.V.uh, W.V.d};
      cx<T>* to[kTsVecs] = {W2.V.y, W2.V.rs, W2.V.w, W2.V.u, W2.V.un, W2.V.v, W2.V.uhe, W2.V.uh, W2.V.d};
      for (int i = 0; i < kTsVecs; ++i) k_gather_cols<cx<T>><<<gb, kBlock, 0, q>>>(nrows, W.s, s2, mp, from[i], to[i]);
      HZ_HIP(hipGetLastError());
      std::vector<TsCol> ns(s2);
      for (int jn = 0; jn < s2; ++jn) {
        if (map[jn] >= 0) {
          ns[jn] = hs[map[jn]];
        } else {
          ns[jn] = TsCol{};
          ns[jn].done = 1;
        }
      }
      std::vector<int> ncols;
      for (int j : keep) ncols.push_back(cols[j]);
      cols = ncols;
      HZ_HIP(hipMemcpyAsync(W2.st, ns.data(), sizeof(TsCol) * s2, hipMemcpyHostToDevice, q));
      HZ_TRY(upload_kc(W2, q));
      // uhe is dead between pairs: scratch output of the tuning runs
      HZ_TRY(autotune<T>(ctx, q, nrows, s2, AT, W2.kc, W2.V.u, W2.V.uhe, &W2.vin));
      W = W2;
      std::unique_ptr<Graph> G2(new Graph());
      HZ_TRY(G2->stream(q));
      HZ_TRY(G2->capture(pairs_body));
      HZ_HIP(hipStreamSynchronize(q));
      G = std::move(G2);
      q = G->gs;
      continue;
    }
    HZ_TRY(G->launch());
  }
  HZ_HIP(hipMemcpyAsync(hs, W.st, sizeof(TsCol) * W.s, hipMemcpyDeviceToHost, q));
  HZ_HIP(hipStreamSynchronize(q));
  {
    const int nreal = int(cols.size());
    std::vector<int> h2(2 * nreal);
    for (int j = 0; j < nreal; ++j) {
      h2[j] = j;
      h2[nreal + j] = cols[j];
    }
    if (nreal > 0) {
      HZ_HIP(hipMemcpyAsync(mapb->p, h2.data(), sizeof(int) * h2.size(), hipMemcpyHostToDevice, q));
      k_out_cols<<<ceil_div(n * nreal, kBlock), kBlock, 0, q>>>(n, W.s, nf, nreal, D.perm.as<int>(), mapb->as<int>(),
                                                                 mapb->as<int>() + nreal, W.X, Pio);
      HZ_HIP(hipGetLastError());
      HZ_HIP(hipStreamSynchronize(q));
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int j = 0; j < nreal; ++j) record(j, secs);
  }
  for (int f = 0; f < nf; ++f) {
    worst = std::max(worst, res[f].status);
    if (infos) infos[f] = res[f];
  }
  return worst;
}

}  // namespace

int sweep_solve(hz_ctx ctx, int nfreq, const double* freqs, const z_t* F, z_t* P, const hz_solve_opts& o,
                hz_solve_info* infos) {
  if (!ctx->sweep_data || ctx->sweep_version != ctx->params_version) {
    ctx->sweep_data.reset();
    std::shared_ptr<void> d(new SweepData(), [](void* q) { delete static_cast<SweepData*>(q); });
    HZ_TRY(build_sweep_data(ctx, static_cast<SweepData*>(d.get())));
    ctx->sweep_data = d;
    ctx->sweep_version = ctx->params_version;
  }
  SweepData& D = *static_cast<SweepData*>(ctx->sweep_data.get());
  ctx->have_freq = false;   // the sweep leaves no single-frequency operator behind
  const bool mixed = o.precision == HZ_MIXED;
  if (o.method == HZ_BICGSTAB)
    return mixed ? run_sweep_bicgstab<float>(ctx, D, nfreq, freqs, F, P, o, infos)
                 : run_sweep_bicgstab<double>(ctx, D, nfreq, freqs, F, P, o, infos);
  if (o.method == HZ_BICGSTABL)
    return mixed ? run_sweep_bicgstabl<float>(ctx, D, nfreq, freqs, F, P, o, infos)
                 : run_sweep_bicgstabl<double>(ctx, D, nfreq, freqs, F, P, o, infos);
  if (o.method == HZ_TFQMR)
    return mixed ? run_sweep_tfqmr<float>(ctx, D, nfreq, freqs, F, P, o, infos)
                 : run_sweep_tfqmr<double>(ctx, D, nfreq, freqs, F, P, o, infos);
  return mixed ? run_sweep_gmres<float>(ctx, D, nfreq, freqs, F, P, o, infos)
               : run_sweep_gmres<double>(ctx, D, nfreq, freqs, F, P, o, infos);
}

// Measurement of the sweep's multi-vector product (declared in hz.h).
template <typename T>
static int time_spmm_t(hz_ctx ctx, SweepData& D, int nf, const double* freqs, int reps, double* avg_ms,
                       int32_t* variant, int64_t* bytes) {
  int s = 1;
  while (s < nf) s <<= 1;
  const int64_t total = D.nrows * s;
  int rc = 0;
  const std::string p = std::string("tspmm.") + (sizeof(T) == 8 ? "z" : "c");
  DevBuf* xb = ctx->buf(p + ".x", sizeof(cx<T>) * total, &rc);
  if (rc) return rc;
  DevBuf* yb = ctx->buf(p + ".y", sizeof(cx<T>) * total, &rc);
  if (rc) return rc;
  DevBuf* kb = ctx->buf(p + ".kc", sizeof(double) * 2 * s, &rc);
  if (rc) return rc;
  std::vector<double> kc(2 * s, 0.0);
  for (int c = 0; c < nf; ++c) {
    const double k = 2.0 * M_PI * freqs[c] / ctx->c;
    kc[2 * c] = k;
    kc[2 * c + 1] = mass_coefficient(k, ctx->h.gls_h);
  }
  hipStream_t q = ctx->stream;
  HZ_HIP(hipMemcpyAsync(kb->p, kc.data(), sizeof(double) * 2 * s, hipMemcpyHostToDevice, q));
  HZ_HIP(hipMemsetAsync(xb->p, 0, sizeof(cx<T>) * total, q));
  const RowOp<T> A = row_op<T>(D);
  Variant v;
  HZ_TRY(autotune<T>(ctx, q, D.nrows, s, A, kb->as<double>(), xb->as<cx<T>>(), yb->as<cx<T>>(), &v));
  HZ_TRY((launch_spmm<T, false>(q, v, D.nrows, s, A, kb->as<double>(), xb->as<cx<T>>(), nullptr, yb->as<cx<T>>(),
                                nullptr, nullptr)));
  hipEvent_t e0, e1;
  HZ_HIP(hipEventCreate(&e0));
  HZ_HIP(hipEventCreate(&e1));
  HZ_HIP(hipEventRecord(e0, q));
  for (int r = 0; r < reps; ++r)
    HZ_TRY((launch_spmm<T, false>(q, v, D.nrows, s, A, kb->as<double>(), xb->as<cx<T>>(), nullptr,
                                  yb->as<cx<T>>(), nullptr, nullptr)));
  HZ_HIP(hipEventRecord(e1, q));
  HZ_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  HZ_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = double(ms) / reps;
  if (variant) *variant = variant_code(v);
  if (bytes) *bytes = spmm_bytes(v, D, s, int(sizeof(T)));
  return HZ_OK;
}

// The sweep's operator data for the current parameters (built on first use).
static int sweep_data_for(hz_ctx ctx, SweepData** out) {
  if (!ctx->sweep_data || ctx->sweep_version != ctx->params_version) {
    ctx->sweep_data.reset();
    std::shared_ptr<void> d(new SweepData(), [](void* q) { delete static_cast<SweepData*>(q); });
    HZ_TRY(build_sweep_data(ctx, static_cast<SweepData*>(d.get())));
    ctx->sweep_data = d;
    ctx->sweep_version = ctx->params_version;
  }
  *out = static_cast<SweepData*>(ctx->sweep_data.get());
  return HZ_OK;
}

int sweep_time_spmm(hz_ctx ctx, int nfreq, const double* freqs, int precision, int reps, double* avg_ms,
                    int32_t* variant, int64_t* bytes) {
  SweepData* D = nullptr;
  HZ_TRY(sweep_data_for(ctx, &D));
  return precision == HZ_MIXED ? time_spmm_t<float>(ctx, *D, nfreq, freqs, reps, avg_ms, variant, bytes)
                               : time_spmm_t<double>(ctx, *D, nfreq, freqs, reps, avg_ms, variant, bytes);
}

// ---------------------------------------------------------------- one multi-vector product
template <typename T>
__global__ void k_apply_in(int64_t nrows, int64_t n, int s, int nf, const int* __restrict__ perm,
                           const z_t* __restrict__ P, cx<T>* __restrict__ X) {
  const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= nrows * s) return;
  const int64_t row = e / s;
  const int c = int(e % s);
  z_t v = {0.0, 0.0};
  if (row < n && c < nf) v = P[int64_t(perm[row]) * nf + c];
  X[e] = cx<T>{T(v.re), T(v.im)};
}

template <typename T>
__global__ void k_apply_out(int64_t n, int s, int nf, const int* __restrict__ perm, const cx<T>* __restrict__ Y,
                            z_t* __restrict__ P) {
  const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= n * nf) return;
  const int64_t row = e / nf;
  const int c = int(e % nf);
  const cx<T> y = Y[row * s + c];
  P[int64_t(perm[row]) * nf + c] = z_t{double(y.re), double(y.im)};
}

template <typename T>
static int apply_t(hz_ctx ctx, SweepData& D, int nf, const double* freqs, const z_t* X, z_t* Y,
                   int32_t* variant) {
  int s = 1;
  while (s < nf) s <<= 1;
  const int64_t n = ctx->h.n, total = D.nrows * s;
  int rc = 0;
  const std::string p = std::string("aspmm.") + (sizeof(T) == 8 ? "z" : "c");
  DevBuf* xb = ctx->buf(p + ".x", sizeof(cx<T>) * total, &rc);
  if (rc) return rc;
  DevBuf* yb = ctx->buf(p + ".y", sizeof(cx<T>) * total, &rc);
  if (rc) return rc;
  DevBuf* kb = ctx->buf(p + ".kc", sizeof(double) * 2 * s, &rc);
  if (rc) return rc;
  std::vector<double> kc(2 * s, 0.0);
  for (int c = 0; c < nf; ++c) {
    const double k = 2.0 * M_PI * freqs[c] / ctx->c;
    kc[2 * c] = k;
    kc[2 * c + 1] = mass_coefficient(k, ctx->h.gls_h);
  }
  hipStream_t q = ctx->stream;
  HZ_HIP(hipMemcpyAsync(kb->p, kc.data(), sizeof(double) * 2 * s, hipMemcpyHostToDevice, q));
  const int* perm = D.perm.as<int>();
  k_apply_in<T><<<ceil_div(total, kBlock), kBlock, 0, q>>>(D.nrows, n, s, nf, perm, X, xb->as<cx<T>>());
  HZ_HIP(hipGetLastError());
  const RowOp<T> A = row_op<T>(D);
  Variant v;
  HZ_TRY(autotune<T>(ctx, q, D.nrows, s, A, kb->as<double>(), xb->as<cx<T>>(), yb->as<cx<T>>(), &v));
  HZ_TRY((launch_spmm<T, false>(q, v, D.nrows, s, A, kb->as<double>(), xb->as<cx<T>>(), nullptr, yb->as<cx<T>>(),
                                nullptr, nullptr)));
  if (n * nf > 0) {
    k_apply_out<T><<<ceil_div(n * nf, kBlock), kBlock, 0, q>>>(n, s, nf, perm, yb->as<cx<T>>(), Y);
    HZ_HIP(hipGetLastError());
  }
  HZ_HIP(hipStreamSynchronize(q));
  if (variant) *variant = variant_code(v);
  return HZ_OK;
}

int sweep_apply(hz_ctx ctx, int nfreq, const double* freqs, int precision, const z_t* X, z_t* Y,
                int32_t* variant) {
  SweepData* D = nullptr;
  HZ_TRY(sweep_data_for(ctx, &D));
  return precision == HZ_MIXED ? apply_t<float>(ctx, *D, nfreq, freqs, X, Y, variant)
                               : apply_t<double>(ctx, *D, nfreq, freqs, X, Y, variant);
}
