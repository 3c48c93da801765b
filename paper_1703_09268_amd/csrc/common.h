// Internal definitions shared by the HIP kernels and the host runtime.
// Complex numbers are plain {re, im} pairs with the natural alignment so a
// complex<float> is one 8-byte load (global_load_dwordx2) and a
// complex<double> one 16-byte load.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdint>
#include <cstdlib>
#include <string>

namespace helm {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) {
  cx<T> z;
  z.re = r;
  z.im = i;
  return z;
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return mk(a.re + b.re, a.im + b.im);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return mk(a.re - b.re, a.im - b.im);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) {
  return mk(s * a.re, s * a.im);
}
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
// acc + a * b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> acc) {
  return mk(acc.re + a.re * b.re - a.im * b.im, acc.im + a.re * b.im + a.im * b.re);
}
template <typename To, typename Ti>
__host__ __device__ __forceinline__ cx<To> cast(cx<Ti> a) {
  return mk<To>(static_cast<To>(a.re), static_cast<To>(a.im));
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> czero() {
  return mk<T>(T(0), T(0));
}

using c32 = cx<float>;

constexpr int KMAX = 32;                // largest Krylov dimension per restart cycle
constexpr int PSTRIDE = 2 * (KMAX + 1);  // doubles per workgroup in partial-sum buffers
using c64d = cx<double>;

// ---------------------------------------------------------------------------
// wavefront / block reductions (wave64), FP64 accumulation
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of `v` over the block (blockDim.x*blockDim.y*blockDim.z threads, a
// multiple of 64, at most 1024).  Result valid in every thread.  `smem` must
// hold 16 doubles.  Fixed order -> deterministic.
__device__ __forceinline__ double block_sum(double v, double* smem) {
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nthreads = blockDim.x * blockDim.y * blockDim.z;
  v = wave_sum(v);
  const int wid = tid >> 6, lane = tid & 63;
  __syncthreads();
  if (lane == 0) smem[wid] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = nthreads >> 6;
  for (int w = 0; w < nw; ++w) s += smem[w];
  return s;
}

// ---------------------------------------------------------------------------
// host-side error plumbing
// ---------------------------------------------------------------------------
struct Error {
  int code;
  std::string msg;
};

#define HELM_HIP_CHECK(expr)                                                  \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      throw ::helm::Error{-3, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define HELM_REQUIRE(cond, text)                       \
  do {                                                 \
    if (!(cond)) throw ::helm::Error{-1, (text)};      \
  } while (0)

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// A roctx range over a scope (host time from the first enqueue to the
// synchronisation that ends the phase), shown by rocprofv3 --marker-trace.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

// HELM_LOG=1: one line per outer cycle of every solve on stderr (active
// right-hand sides, largest and smallest FP64 relative residual); 2: also
// every right-hand side's residual.
inline int log_level() {
  const char* e = std::getenv("HELM_LOG");
  return e ? std::atoi(e) : 0;
}

}  // namespace helm
