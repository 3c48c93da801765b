// Vector kernels of the box-constrained L-BFGS that drives the inversion
// (arXiv:1703.09268, the 2D inversion example and the stochastic inversion
// section: a bound-constrained quasi-Newton method on m_LB <= m <= m_UB).
// Every vector is FP64 and N long; the free set F (variables not held at a
// bound by the gradient: not (x <= lo and g > 0) and not (x >= hi and
// g < 0)) is evaluated inline from the current iterate x and gradient g, so
// restricted vectors are never stored.  Reductions leave one partial sum per
// workgroup (fixed order); the host adds the partials in workgroup order, so
// every dot product is deterministic.
#pragma once

#include "common.h"

namespace helm {

constexpr int LB_BLOCKS = 1024;  // workgroups of every L-BFGS vector kernel (at most)
constexpr int LB_MAXMEM = 16;    // stored pairs (at most)

// Bounds: per-point arrays, or the scalars where an array is null.
struct Box {
  const double* lo;
  const double* hi;
  double slo, shi;
};

__device__ __forceinline__ double box_lo(const Box& b, int64_t i) { return b.lo ? b.lo[i] : b.slo; }
__device__ __forceinline__ double box_hi(const Box& b, int64_t i) { return b.hi ? b.hi[i] : b.shi; }
__device__ __forceinline__ bool is_free(double x, double g, double lo, double hi) {
  return !((x <= lo && g > 0.0) || (x >= hi && g < 0.0));
}

__device__ __forceinline__ double block_max(double v, double* smem) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) smem[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s = fmax(s, smem[w]);
  return s;
}

// x = clamp(m0, lo, hi) in FP64; part[b] = number of points with lo > hi
template <typename T>
__global__ __launch_bounds__(256) void k_lb_init(const T* __restrict__ m0, Box bx, double* __restrict__ x, int64_t N,
                                                 double* __restrict__ part) {
  __shared__ double sm[16];
  double bad = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
    const double lo = box_lo(bx, i), hi = box_hi(bx, i);
    bad += (lo > hi || !(lo == lo) || !(hi == hi)) ? 1.0 : 0.0;
    x[i] = fmin(fmax((double)m0[i], lo), hi);
  }
  bad = block_sum(bad, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = bad;
}

// q = g restricted to F; part[b] = max |q| over the workgroup's points
__global__ __launch_bounds__(256) void k_lb_start(const double* __restrict__ x, const double* __restrict__ g, Box bx,
                                                  double* __restrict__ q, int64_t N, double* __restrict__ part) {
  __shared__ double sm[16];
  double mx = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
    const double gi = g[i];
    const double v = is_free(x[i], gi, box_lo(bx, i), box_hi(bx, i)) ? gi : 0.0;
    q[i] = v;
    mx = fmax(mx, fabs(v));
  }
  mx = block_max(mx, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = mx;
}

// Restricted products of the stored pairs: for k < npair,
//   part[b][2k] = sum_F s_k y_k,  part[b][2k+1] = sum_F y_k y_k
// (S[k], Y[k] the pair pointers in newest-first order).
struct PairPtrs {
  const double* s[LB_MAXMEM];
  const double* y[LB_MAXMEM];
};

__global__ __launch_bounds__(256) void k_lb_pair_dots(PairPtrs P, int npair, const double* __restrict__ x,
                                                      const double* __restrict__ g, Box bx, int64_t N,
                                                      double* __restrict__ part) {
  __shared__ double sm[16];
  for (int k = 0; k < npair; ++k) {
    const double* __restrict__ s = P.s[k];
    const double* __restrict__ y = P.y[k];
    double sy = 0.0, yy = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
      if (!is_free(x[i], g[i], box_lo(bx, i), box_hi(bx, i))) continue;
      const double yi = y[i];
      sy += s[i] * yi;
      yy += yi * yi;
    }
    sy = block_sum(sy, sm);
    yy = block_sum(yy, sm);
    if (threadIdx.x == 0) {
      part[(size_t)blockIdx.x * 2 * LB_MAXMEM + 2 * k] = sy;
      part[(size_t)blockIdx.x * 2 * LB_MAXMEM + 2 * k + 1] = yy;
    }
  }
}

// One step of the two-loop recursion (and its end):
//   v = scale * (v + c * u restricted to F)     (u may be null: v = scale v)
//   part[b] = sum w * v                          (w may be null: no sum)
// v is zero off F on entry (it starts as the restricted gradient), so the
// sum of w * v equals the restricted product.
__global__ __launch_bounds__(256) void k_lb_update(double* __restrict__ v, double c, const double* __restrict__ u,
                                                   double scale, const double* __restrict__ w,
                                                   const double* __restrict__ x, const double* __restrict__ g, Box bx,
                                                   int64_t N, double* __restrict__ part) {
  __shared__ double sm[16];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
    double vi = v[i];
    if (u && is_free(x[i], g[i], box_lo(bx, i), box_hi(bx, i))) vi += c * u[i];
    vi *= scale;
    v[i] = vi;
    if (w) acc += w[i] * vi;
  }
  if (w) {
    acc = block_sum(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
  }
}

// Trial point xt = clamp(x + t d, lo, hi) (d null: clamp(x)), its copy in
// the solver's real type (mt, null when the solver reads xt itself), and
// part[b] = sum g (xt - x) (g null: no sum).
template <typename T>
__global__ __launch_bounds__(256) void k_lb_trial(const double* __restrict__ x, const double* __restrict__ d, double t,
                                                  Box bx, double* __restrict__ xt, T* __restrict__ mt,
                                                  const double* __restrict__ g, int64_t N, double* __restrict__ part) {
  __shared__ double sm[16];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
    const double xi = x[i];
    const double v = fmin(fmax(d ? xi + t * d[i] : xi, box_lo(bx, i)), box_hi(bx, i));
    xt[i] = v;
    if (mt) mt[i] = (T)v;
    if (g) acc += g[i] * (v - xi);
  }
  if (g) {
    acc = block_sum(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
  }
}

// Accept the trial: s = xt - x, y = gt - g (gt = the trial's gradient in the
// solver's real type), x = xt, g = gt; part[b][0..2] = s.y, s.s, y.y.  With
// s null only x and g are replaced (the start of a subproblem).
template <typename T>
__global__ __launch_bounds__(256) void k_lb_accept(double* __restrict__ x, double* __restrict__ g,
                                                   const double* __restrict__ xt, const T* __restrict__ gt,
                                                   double* __restrict__ s, double* __restrict__ y, int64_t N,
                                                   double* __restrict__ part) {
  __shared__ double sm[16];
  double sy = 0.0, ss = 0.0, yy = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
    const double xn = xt[i], gn = (double)gt[i];
    if (s) {
      const double si = xn - x[i], yi = gn - g[i];
      s[i] = si;
      y[i] = yi;
      sy += si * yi;
      ss += si * si;
      yy += yi * yi;
    }
    x[i] = xn;
    g[i] = gn;
  }
  if (s) {
    sy = block_sum(sy, sm);
    ss = block_sum(ss, sm);
    yy = block_sum(yy, sm);
    if (threadIdx.x == 0) {
      part[3 * blockIdx.x] = sy;
      part[3 * blockIdx.x + 1] = ss;
      part[3 * blockIdx.x + 2] = yy;
    }
  }
}

// m = x in the caller's real type
template <typename T>
__global__ __launch_bounds__(256) void k_lb_store(const double* __restrict__ x, T* __restrict__ m, int64_t N) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) m[i] = (T)x[i];
}

}  // namespace helm
