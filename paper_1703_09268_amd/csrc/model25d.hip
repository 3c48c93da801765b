// Kernels of 2.5D modelling (arXiv:1703.09268, the 2.5D subsection): for a
// model invariant along y, the 3D field is the cosine synthesis
//   u(x, y, z) = sum_i w_i u~_{k_i}(x, z) cos(k_i (y - y_s))
// of 2D fields u~_k solving (d_xx + d_zz + omega^2 m - k^2) u~ = delta_s, one
// per Gauss-Legendre node k_i of the k_y integral (weights w_i with 1/pi).
// Each (frequency, source, k_i) triple is one "pair" p of a batched 2D solve
// (pairs contiguous, p = row * nky + i with row a selected (frequency,
// source)); its model is m - k_i^2 / omega^2 and its receivers' values carry
// the weight c_{p,r} = w_i cos(k_i (y_r - y_s)).
#pragma once

#include "common.h"

namespace helm {

// out_j = m - shift_j (model j of the shifted set), j = blockIdx.y
template <typename T>
__global__ __launch_bounds__(256) void k_shift_models(const T* __restrict__ m, int64_t N,
                                                      const double* __restrict__ shift, T* __restrict__ out) {
  const int j = blockIdx.y;
  const double sh = shift[j];
  T* o = out + (int64_t)j * N;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256)
    o[i] = (T)((double)m[i] - sh);
}

// Per-pair quadrature data: node k, weight w (1/pi included), source y.
struct Quad25 {
  const double* k;
  const double* w;
  const double* ys;
};

// Receiver synthesis of row r (a selected (frequency, source)):
//   dp_r[e] = sum_i c_{p,e} (P u~_p)_e,  p = r * nky + i,
// u FP64 (pair p at u + p N); res = dp - d[drow_r] (stored in T), pred (if
// not null) = dp at [drow_r]; part[r * gridDim.x + blk] = sum |res|^2.
template <typename T>
__global__ __launch_bounds__(256) void k_synth25d(const cx<double>* __restrict__ u, int64_t N, int nky, Quad25 q,
                                                  const int* __restrict__ rptr, const int64_t* __restrict__ rlin,
                                                  const double* __restrict__ rw, const double* __restrict__ rec_y,
                                                  int nrec, const cx<T>* __restrict__ d,
                                                  const int64_t* __restrict__ drow, cx<T>* __restrict__ res,
                                                  cx<T>* __restrict__ pred, double* __restrict__ part) {
  __shared__ double red[16];
  const int r = blockIdx.y;
  const int e = blockIdx.x * 256 + threadIdx.x;
  double acc = 0.0;
  if (e < nrec) {
    cx<double> dp = czero<double>();
    for (int i = 0; i < nky; ++i) {
      const int64_t p = (int64_t)r * nky + i;
      const double c = q.w[p] * cos(q.k[p] * (rec_y[e] - q.ys[p]));
      const cx<double>* up = u + p * N;
      cx<double> v = czero<double>();
      for (int t = rptr[e]; t < rptr[e + 1]; ++t) v = v + rw[t] * up[rlin[t]];
      dp = dp + c * v;
    }
    if (pred) pred[drow[r] * nrec + e] = cast<T>(dp);
    cx<double> rr = dp;
    if (d) {
      const cx<T> dv = d[drow[r] * nrec + e];
      rr = mk<double>(dp.re - (double)dv.re, dp.im - (double)dv.im);
    }
    res[(int64_t)r * nrec + e] = cast<T>(rr);
    acc = rr.re * rr.re + rr.im * rr.im;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[(int64_t)r * gridDim.x + blockIdx.x] = t;
}

// Adjoint sources b_p = -P_r^T (c_p * res_{row p}) at the nodes the receivers
// touch (b zero elsewhere beforehand); node lists as k_adjoint_source (fixed
// summation order).  Grid (node blocks, pairs).
template <typename T>
__global__ __launch_bounds__(256) void k_adjoint25d(cx<T>* __restrict__ b, int64_t N, int nky, Quad25 q,
                                                    const int64_t* __restrict__ node_lin,
                                                    const int* __restrict__ node_ptr,
                                                    const int* __restrict__ node_rec,
                                                    const double* __restrict__ node_w, int nnode,
                                                    const double* __restrict__ rec_y,
                                                    const cx<T>* __restrict__ res, int nrec) {
  const int p = blockIdx.y;
  const int nd = blockIdx.x * 256 + threadIdx.x;
  if (nd >= nnode) return;
  const int row = p / nky;
  const double k = q.k[p], w = q.w[p], ys = q.ys[p];
  cx<double> acc = czero<double>();
  for (int t = node_ptr[nd]; t < node_ptr[nd + 1]; ++t) {
    const int e = node_rec[t];
    const double c = node_w[t] * w * cos(k * (rec_y[e] - ys));
    acc = acc + c * cast<double>(res[(int64_t)row * nrec + e]);
  }
  b[(int64_t)p * N + node_lin[nd]] = cast<T>(mk<double>(-acc.re, -acc.im));
}

}  // namespace helm
