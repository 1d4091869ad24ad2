// Device building blocks shared by the Krylov solvers.
//
// Row layout.  A solve works on one system, or on a batch of independent
// systems ("segments") stacked one after the other, each padded to a whole
// number of 256-row blocks.  Every vector kernel runs one block per 256 rows,
// so each block belongs to exactly one segment; reductions write one partial
// per block and a finalize kernel (one block per segment) sums that segment's
// partials in block order.  Sums are therefore reproducible bit for bit, and
// every segment carries its own Krylov scalars and convergence flag: a batch
// of subdomain solves advances in lock-step but each one is its own Krylov
// iteration.  Padding rows hold zero matrix rows and zero vector entries.
#pragma once

#include <vector>

#include "common.h"

struct Seg {
  int nseg = 0;
  int nblk = 0;
  int64_t nrows = 0;              // nblk * kBlock
  const int* blk_seg = nullptr;   // [nblk]
  const int* seg_blk = nullptr;   // [nseg + 1]
};

// A sliced-ELL operator in one of two storage forms.
//  complex form (val != NULL): one complex value per stored entry.
//  split form (val == NULL): the real part of every stored entry (re) plus,
//    per row, a short list of the entries whose imaginary part can be
//    nonzero (imeta/icol/iim, interleaved per slice).  Without an absorption
//    field only the entries that touch the absorbing walls are complex (the
//    wall term and the Jacobi scaling of wall columns), so this form streams
//    8 (FP64) or 4 (FP32) bytes per entry instead of 16 or 8.
//  Column indices are int32 (col) or, when every |col - row| fits, int16
//  offsets from the row (dcol).
//  stencil form (st != NULL, structured boxes): the split form's real parts
//    stored with implied columns: slot k of every row is the neighbour at
//    offset soff[k] (the 27 neighbours of a node of the box, ascending), a
//    missing neighbour holds 0; 64-row slices of 27 slots, slot k of lane l
//    at 27 * 64 * slice + 64 k + l.  No index is streamed; the imaginary
//    entries are the split form's row lists.
constexpr int kStencil = 27;
struct StencilOffsets {
  int o[kStencil];
};
// Imaginary entries of one 64-row slice (split and stencil forms).  The
// lanes whose row has any (bit l of mask) keep their lists interleaved:
// entry k of the j-th such lane at base + k nl + j, every list padded with
// zero values (column: the row itself) to the slice's longest, w.  Each step
// of the lists' loop then loads consecutive values and columns across the
// lanes, instead of one scattered list per lane.
struct ImSlice {
  int base, nl, w, pad;
  unsigned long long mask;
};
template <typename T>
struct SellOp {
  const int* ptr = nullptr;       // [nrows / 64 + 1] slice offsets
  const int* col = nullptr;
  const cx<T>* val = nullptr;
  const T* re = nullptr;          // split form
  const int16_t* dcol = nullptr;  // split form: column - row (NULL: use col)
  const ImSlice* imeta = nullptr; // [nrows / 64] imaginary entries of each slice
  const int* icol = nullptr;      // their columns and values, interleaved per slice
  const T* iim = nullptr;
  const T* st = nullptr;          // stencil form
  int64_t nrows = 0;              // stencil form: rows of the vectors (gathers are clamped to them)
  StencilOffsets soff = {};
};

// Non-temporal loads for the streamed matrix data (read once per product):
// keeps L2 / Infinity Cache for the gathered vector.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ z_t ld_stream(const z_t* p) {
  d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
  return z_t{v.x, v.y};
}
__device__ __forceinline__ c_t ld_stream(const c_t* p) {
  f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(p));
  return c_t{v.x, v.y};
}
__device__ __forceinline__ int ld_stream(const int* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ int ld_stream(const int16_t* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ double ld_stream(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ld_stream(const float* p) { return __builtin_nontemporal_load(p); }

// Real-part sweep of the split form: acc += re_k * x[col_k] over the row.
template <typename T, typename I>
__device__ __forceinline__ void split_real(const I* __restrict__ c, const T* __restrict__ v, int w, int64_t row,
                                           const cx<T>* __restrict__ x, T& ar, T& ai) {
#pragma unroll 9
  for (int k = 0; k < w; ++k) {
    int j = ld_stream(c + (k << 6));
    if (sizeof(I) == 2) j += int(row);
    T a = ld_stream(v + (k << 6));
    cx<T> xv = x[j];
    ar = fma(a, xv.re, ar);
    ai = fma(a, xv.im, ai);
  }
}

// Storage forms of a SellOp (compile-time selector of sell_row_form).
enum { kFormComplex = 0, kFormSplit = 1, kFormStencil = 2 };

// Launch bounds of the solver kernels that carry a sparse product (T: the
// vector type).  Capping the FP64 kernels at 6 waves per SIMD lets the
// compiler give the product loop more registers (measured: 88 VGPRs, 5 waves,
// 250.5 us per BiCGStab iteration on the 160x96x80 cavity, against 76 VGPRs,
// 6 waves, 258.5 us uncapped); the complex64 kernels ran slower capped.
#define HZ_PRODUCT_BOUNDS __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, sizeof(T) == 8 ? 6 : 8)))

// y_row = sum_k A[row, col_k] x[col_k] over the row's sliced-ELL entries,
// for an operator known to be in form F.
template <int F, typename T>
__device__ __forceinline__ cx<T> sell_row_form(const SellOp<T>& A, int64_t row, const cx<T>* __restrict__ x) {
  const int slice = int(row >> 6), lane = int(row & 63);
  if constexpr (F == kFormComplex) {
    const int beg = A.ptr[slice];
    const int w = (A.ptr[slice + 1] - beg) >> 6;
    const int* __restrict__ c = A.col + beg + lane;
    const cx<T>* __restrict__ v = A.val + beg + lane;
    cx<T> acc = {T(0), T(0)};
#pragma unroll 6
    for (int k = 0; k < w; ++k) {
      int j = ld_stream(c + (k << 6));
      cx<T> a = ld_stream(v + (k << 6));
      cx<T> xv = x[j];
      cfma(acc, a, xv);
    }
    return acc;
  }
  T ar = T(0), ai = T(0);
  // the slice's imaginary-list descriptor, loaded ahead of the real-part sweep
  const ImSlice im = A.imeta[slice];
  const bool listed = (im.mask >> lane) & 1ull;
  const int jl = __builtin_popcountll(im.mask & ((1ull << lane) - 1ull));
  if constexpr (F == kFormStencil) {
    // Slots 3 t, 3 t + 1, 3 t + 2 are one line of the box (offsets o - 1,
    // o, o + 1).  The wave's 64 consecutive rows load the centre x[row + o]
    // once; the left and right neighbours come from the adjacent lanes,
    // and only the wave's two end lanes load their outer value (one load
    // with two lanes active).  Terms are added in slot order, as before.
    // Every caller runs this with all 64 lanes of the wave active.
    const T* __restrict__ v = A.st + int64_t(slice) * (kStencil * 64) + lane;
    const int64_t last = A.nrows - 1;
    auto clampi = [last](int64_t j) { return j < 0 ? int64_t(0) : (j > last ? last : j); };
#pragma unroll 3
    for (int t = 0; t < kStencil / 3; ++t) {
      const int o = A.soff.o[3 * t + 1];
      const cx<T> xc = x[clampi(row + o)];
      cx<T> xe = {T(0), T(0)};
      if (lane == 0 || lane == kWave - 1) xe = x[clampi(lane == 0 ? row + o - 1 : row + o + 1)];
      cx<T> xl, xr;
      xl.re = __shfl_up(xc.re, 1, kWave);
      xl.im = __shfl_up(xc.im, 1, kWave);
      xr.re = __shfl_down(xc.re, 1, kWave);
      xr.im = __shfl_down(xc.im, 1, kWave);
      if (lane == 0) xl = xe;
      if (lane == kWave - 1) xr = xe;
      const T a0 = ld_stream(v + ((3 * t) << 6));
      const T a1 = ld_stream(v + ((3 * t + 1) << 6));
      const T a2 = ld_stream(v + ((3 * t + 2) << 6));
      ar = fma(a0, xl.re, ar);
      ai = fma(a0, xl.im, ai);
      ar = fma(a1, xc.re, ar);
      ai = fma(a1, xc.im, ai);
      ar = fma(a2, xr.re, ar);
      ai = fma(a2, xr.im, ai);
    }
  } else {
    const int beg = A.ptr[slice];
    const int w = (A.ptr[slice + 1] - beg) >> 6;
    if (A.dcol) split_real(A.dcol + beg + lane, A.re + beg + lane, w, row, x, ar, ai);
    else split_real(A.col + beg + lane, A.re + beg + lane, w, row, x, ar, ai);
  }
  // imaginary entries, four steps at a time: the four value/column loads,
  // then the four gathers, issue back to back (a step past the slice's
  // longest list gathers x[0] and adds nothing; a padded entry adds zero);
  // the terms are added in list order
  if (listed) {
    const T* __restrict__ pb = A.iim + im.base + jl;
    const int* __restrict__ pc = A.icol + im.base + jl;
    for (int k = 0; k < im.w; k += 4) {
      T b[4];
      int c[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool on = k + u < im.w;
        b[u] = on ? pb[(k + u) * im.nl] : T(0);
        c[u] = on ? pc[(k + u) * im.nl] : 0;
      }
      cx<T> xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) xv[u] = x[c[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (k + u < im.w) {         // i b x = -b x.im + i b x.re
          ar = fma(-b[u], xv[u].im, ar);
          ai = fma(b[u], xv[u].re, ai);
        }
    }
  }
  return cx<T>{ar, ai};
}


// Block geometry of a segmented kernel: tile, row, segment.  Tile t holds
// rows [256 t, 256 t + 256); workgroups take tiles in runs of 8 per XCD
// (xcd_chunk_tile), so rows whose neighbourhoods overlap mostly share one
// XCD's L2.  Measured on the 27-point products this beats both plain
// dispatch order and one contiguous row range per XCD.
struct Tile {
  int tile;
  int seg;
  int64_t row;
};
__device__ __forceinline__ Tile tile_of(const Seg& L) {
  Tile t;
  t.tile = xcd_chunk_tile(blockIdx.x, gridDim.x);
  t.seg = L.blk_seg[t.tile];
  t.row = int64_t(t.tile) * kBlock + threadIdx.x;
  return t;
}
// Count of this block's waves that have stored their sums in store_partials.
__device__ __forceinline__ int* block_wave_count() {
  __shared__ int n;
  return &n;
}
// The tile of a kernel that stores block partials (store_partials takes
// only this type): all its threads call it first, before any return, and
// the block's wave count is zeroed behind a barrier.
struct SumTile : Tile {};
__device__ __forceinline__ SumTile tile_of_sums(const Seg& L) {
  SumTile t;
  static_cast<Tile&>(t) = tile_of(L);
  if (threadIdx.x == 0) *block_wave_count() = 0;
  __syncthreads();
  return t;
}

// Block-sum NQ doubles and store them as partial[tile * NQ + q]: every
// quantity is reduced within each wave, each wave puts its sums in LDS and
// counts itself in, and the wave that counts last adds the waves' sums in
// wave order (so the result does not depend on which wave that is) and
// stores them.  No barrier closes the kernel: a wave that is not last
// leaves at once instead of holding its slot until the block's slowest wave
// finishes (measured 79 -> 75 us for the 27-point product with four sums).
// Called once per kernel, by every wave of the block or by none (the
// callers return early only for a whole segment, hence a whole block), with
// the tile from tile_of_sums, which zeroed the count.
template <int NQ>
__device__ __forceinline__ void store_partials(double (&v)[NQ], double* partial, const SumTile& t) {
  const int tile = t.tile;
  constexpr int kWaves = kBlock / kWave;
  __shared__ double lds[NQ][kWaves];
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  double s[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) s[q] = wave_sum(v[q]);
  int last = 0;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) lds[q][w] = s[q];
    // release: the sums are in LDS before the count; acquire for the last
    last = __hip_atomic_fetch_add(block_wave_count(), 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) ==
           kWaves - 1;
  }
  last = __shfl(last, 0, kWave);
  if (!last) return;
  // every lane of the last wave reads the other waves' sums after the count
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  for (int q = lane; q < NQ; q += kWave) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i)
      t += __hip_atomic_load(&lds[q][i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    partial[int64_t(tile) * NQ + q] = t;
  }
}

// The same, storing quantity q at partial[q * qstride + tile] (each
// quantity's block partials contiguous, for finalize kernels that reduce one
// quantity per block).
template <int NQ>
__device__ __forceinline__ void store_partials_qmajor(double (&v)[NQ], double* partial, int64_t qstride,
                                                      const SumTile& t) {
  const int tile = t.tile;
  constexpr int kWaves = kBlock / kWave;
  __shared__ double lds[NQ][kWaves];
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  double s[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) s[q] = wave_sum(v[q]);
  int last = 0;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) lds[q][w] = s[q];
    last = __hip_atomic_fetch_add(block_wave_count(), 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) ==
           kWaves - 1;
  }
  last = __shfl(last, 0, kWave);
  if (!last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  for (int q = lane; q < NQ; q += kWave) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i)
      t += __hip_atomic_load(&lds[q][i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    partial[int64_t(q) * qstride + tile] = t;
  }
}

// Finalize kernels run with kFinBlock threads, one block per segment.
constexpr int kFinBlock = 1024;

// Sum every quantity of this segment's partials in one pass (thread t takes
// tiles t, t + blockDim, ...; then wave sums and the waves in order); the
// totals are valid in thread 0.  Finalize kernels call it before they branch
// on the segment's state (read into registers first), so the partials'
// loads do not wait for the state's; the sums of a segment that is off are
// simply not used.
template <int NQ>
__device__ __forceinline__ void seg_sums(const Seg& L, const double* partial, int seg, double (&out)[NQ]) {
  __shared__ double lds[NQ][kFinBlock / kWave];
  // one segment spans every block: no dependent load of its block range
  const int b0 = L.nseg == 1 ? 0 : L.seg_blk[seg], b1 = L.nseg == 1 ? L.nblk : L.seg_blk[seg + 1];
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
#pragma unroll 4
  for (int i = b0 + int(threadIdx.x); i < b1; i += int(blockDim.x)) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] += partial[int64_t(i) * NQ + q];
  }
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave, nw = blockDim.x / kWave;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double s = wave_sum(acc[q]);
    if (lane == 0) lds[q][w] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double s = 0.0;
      for (int i = 0; i < nw; ++i) s += lds[q][i];
      out[q] = s;
    }
  }
  __syncthreads();
}

// In a finalize kernel (one block per segment): sum quantity q of this
// segment's partials; valid in thread 0.
template <int NQ>
__device__ __forceinline__ double seg_sum(const Seg& L, const double* partial, int seg, int q) {
  __shared__ double lds[kFinBlock / kWave];
  const int b0 = L.nseg == 1 ? 0 : L.seg_blk[seg], b1 = L.nseg == 1 ? L.nblk : L.seg_blk[seg + 1];
  return block_sum_strided(partial + int64_t(b0) * NQ + q, b1 - b0, NQ, lds);
}

// Host-side description of a segmented system on the device.
struct SegHost {
  int nseg = 0, nblk = 0;
  int64_t nrows = 0;
  std::vector<int> seg_blk;       // host copy [nseg + 1]
  std::vector<int64_t> seg_n;     // true (unpadded) rows per segment
  Seg dev;                        // device view
};
