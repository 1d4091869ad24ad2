// Shared definitions of the gfx950 Helmholtz library: the complex type,
// error reporting, launch geometry and wave64/block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>

#include "hz.h"

#define HD __host__ __device__ __forceinline__

// Complex number as a pair of reals (paper Sec. 4 defines its own complex
// class template in place of the vendor type; this is the same idea, laid out
// so that complex<double> loads as one 16-byte and complex<float> as one
// 8-byte vector access).
template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};
using z_t = cx<double>;
using c_t = cx<float>;

template <typename T> HD cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T> HD cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> HD cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> HD cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> HD cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> HD cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
template <typename T> HD T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }
// acc += a * b
template <typename T> HD void cfma(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
template <typename T> HD void cfma_conj(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}
// Complex division by Smith's method (R. L. Smith, "Algorithm 116: Complex
// division", CACM 5(8), 1962): scale by the larger component to avoid
// overflow in |d|^2.
template <typename T> HD cx<T> cdiv(cx<T> a, cx<T> d) {
  if (fabs(d.re) >= fabs(d.im)) {
    if (d.re == T(0)) return {T(NAN), T(NAN)};
    T r = d.im / d.re, den = d.re + d.im * r;
    return {(a.re + a.im * r) / den, (a.im - a.re * r) / den};
  }
  T r = d.re / d.im, den = d.re * r + d.im;
  return {(a.re * r + a.im) / den, (a.im * r - a.re) / den};
}
template <typename T> HD cx<T> crecip(cx<T> d) { return cdiv(cx<T>{T(1), T(0)}, d); }
template <typename To, typename Ti> HD cx<To> ccast(cx<Ti> a) { return {To(a.re), To(a.im)}; }

// ---------------------------------------------------------------- errors
void hz_set_error(const char* fmt, ...);
int hz_fail(int code, const char* fmt, ...);

#define HZ_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return hz_fail(e_ == hipErrorOutOfMemory ? HZ_ERR_OOM : HZ_ERR_HIP, "%s: %s (%s:%d)", \
                     #call, hipGetErrorString(e_), __FILE__, __LINE__);                \
  } while (0)

#define HZ_TRY(expr)            \
  do {                          \
    int rc_ = (expr);           \
    if (rc_ < 0) return rc_;    \
  } while (0)

// ---------------------------------------------------------------- launch geometry
constexpr int kBlock = 256;      // 4 waves of 64
constexpr int kWave = 64;
constexpr int kNumXcd = 8;       // MI355X: 8 accelerator complex dies, round-robin dispatch

inline int ceil_div(int64_t a, int64_t b) { return int((a + b - 1) / b); }

// Blocks of a grid-stride reduction over n entries: a pure function of n so
// that the summation order (and result) is reproducible run to run.
inline int reduce_grid(int64_t n) {
  int g = ceil_div(n, int64_t(kBlock) * 4);
  return g < 1 ? 1 : (g > 1024 ? 1024 : g);
}

// The hardware hands workgroup b to XCD b % 8.  Give each XCD a contiguous
// range of logical tiles so neighbouring rows (which gather the same x
// entries) share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  int q = nblocks / kNumXcd, r = nblocks % kNumXcd;
  int x = b % kNumXcd, idx = b / kNumXcd;
  return x * q + (x < r ? x : r) + idx;
}

// Chunked variant: each XCD takes runs of kXcdChunk consecutive tiles, the
// XCDs' runs interleaved (tiles [8 C g + C x, 8 C g + C x + C) on XCD x);
// the tail past the last whole round of 8 C tiles keeps dispatch order.
constexpr int kXcdChunk = 8;
__device__ __forceinline__ int xcd_chunk_tile(int b, int nblocks) {
  constexpr int span = kNumXcd * kXcdChunk;
  const int full = nblocks / span * span;
  if (b >= full) return b;
  const int x = b % kNumXcd, i = b / kNumXcd;
  return ((i / kXcdChunk) * kNumXcd + x) * kXcdChunk + i % kXcdChunk;
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum of v over the block (blockDim.x threads, a multiple of 64, at most
// 1024); the result is valid in thread 0.  Fixed order: wave butterflies,
// then the waves in order.
__device__ __forceinline__ double block_sum(double v, double* lds /*[blockDim.x/kWave]*/) {
  v = wave_sum(v);
  int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < int(blockDim.x) / kWave; ++i) s += lds[i];
  }
  __syncthreads();
  return s;
}

// Sum of `cnt` values `part[i*stride]` by one block, fixed order; valid in thread 0.
__device__ __forceinline__ double block_sum_strided(const double* part, int cnt, int stride,
                                                    double* lds) {
  double s = 0.0;
  for (int i = threadIdx.x; i < cnt; i += int(blockDim.x)) s += part[int64_t(i) * stride];
  return block_sum(s, lds);
}
