// Receiver-space kernels of the WRI field solve (arXiv:1703.09268, Penalty
// Method subsection, eqs. wri and wrifieldeq; Appendix B).  The field
// u = argmin 1/2 ||P_r u - d||^2 + lambda^2/2 ||H u - q||^2 is written as
// u = H^{-1}(q + e) with e = H^{-H} P_r^T y, where y solves the receiver-space
// system (K + lambda^2 I) y = d - P_r H^{-1} q, K = P_r H^{-1} H^{-H} P_r^T
// (Hermitian positive semidefinite); y is found by conjugate gradients and u
// is accumulated as u0 + sum_k alpha_k z_k with z_k = H^{-1} H^{-H} P_r^T p_k,
// so y itself is never stored.  Receiver-space vectors are FP64, one row of
// nrec values per (frequency, source) pair; per-workgroup partial sums go to
// part[s * gridDim.x + blk] and are added on the host in workgroup order.
#pragma once

#include "common.h"

namespace helm {

// rho_s = d[drow_s] - P_r u_s (u FP64), p_s = rho_s; part = |rho|^2
template <typename T>
__global__ __launch_bounds__(256) void k_wri_start(const cx<double>* __restrict__ u, const int64_t* __restrict__ uoff,
                                                   const int* __restrict__ rptr, const int64_t* __restrict__ rlin,
                                                   const double* __restrict__ rw, int nrec,
                                                   const cx<T>* __restrict__ d, const int64_t* __restrict__ drow,
                                                   cx<double>* __restrict__ rho, cx<double>* __restrict__ p,
                                                   double* __restrict__ part) {
  __shared__ double red[16];
  const int s = blockIdx.y;
  const int k = blockIdx.x * 256 + threadIdx.x;
  double acc = 0.0;
  if (k < nrec) {
    cx<double> uv = czero<double>();
    const cx<double>* us = u + uoff[s];
    for (int e = rptr[k]; e < rptr[k + 1]; ++e) uv = uv + rw[e] * us[rlin[e]];
    const cx<T> dv = d[drow[s] * nrec + k];
    const cx<double> r = mk<double>((double)dv.re - uv.re, (double)dv.im - uv.im);
    rho[(int64_t)s * nrec + k] = r;
    p[(int64_t)s * nrec + k] = r;
    acc = r.re * r.re + r.im * r.im;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[(int64_t)s * gridDim.x + blockIdx.x] = t;
}

// b_s = +P_r^T p_s at the nodes the receivers touch (b zero elsewhere
// beforehand); node lists as k_adjoint_source (fixed summation order)
template <typename T>
__global__ __launch_bounds__(256) void k_wri_spread(cx<T>* __restrict__ b, int64_t N,
                                                    const int64_t* __restrict__ node_lin,
                                                    const int* __restrict__ node_ptr,
                                                    const int* __restrict__ node_rec,
                                                    const double* __restrict__ node_w, int nnode,
                                                    const cx<double>* __restrict__ p, int nrec) {
  const int s = blockIdx.y;
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= nnode) return;
  cx<double> acc = czero<double>();
  for (int e = node_ptr[q]; e < node_ptr[q + 1]; ++e) acc = acc + node_w[e] * p[(int64_t)s * nrec + node_rec[e]];
  b[s * N + node_lin[q]] = cast<T>(acc);
}

// ap_s = P_r z_s + lambda^2 p_s (z FP64, pair s at z + s N); part =
// Re(conj(p) ap)
__global__ __launch_bounds__(256) void k_wri_apply(const cx<double>* __restrict__ z, int64_t N,
                                                   const int* __restrict__ rptr, const int64_t* __restrict__ rlin,
                                                   const double* __restrict__ rw, int nrec, double lam2,
                                                   const cx<double>* __restrict__ p, cx<double>* __restrict__ ap,
                                                   double* __restrict__ part) {
  __shared__ double red[16];
  const int s = blockIdx.y;
  const int k = blockIdx.x * 256 + threadIdx.x;
  double acc = 0.0;
  if (k < nrec) {
    cx<double> zv = czero<double>();
    const cx<double>* zs = z + s * N;
    for (int e = rptr[k]; e < rptr[k + 1]; ++e) zv = zv + rw[e] * zs[rlin[e]];
    const cx<double> pv = p[(int64_t)s * nrec + k];
    const cx<double> a = mk<double>(zv.re + lam2 * pv.re, zv.im + lam2 * pv.im);
    ap[(int64_t)s * nrec + k] = a;
    acc = pv.re * a.re + pv.im * a.im;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[(int64_t)s * gridDim.x + blockIdx.x] = t;
}

// rho_s -= alpha_s ap_s; part = |rho|^2
__global__ __launch_bounds__(256) void k_wri_residual(cx<double>* __restrict__ rho, const cx<double>* __restrict__ ap,
                                                      const double* __restrict__ alpha, int nrec,
                                                      double* __restrict__ part) {
  __shared__ double red[16];
  const int s = blockIdx.y;
  const int k = blockIdx.x * 256 + threadIdx.x;
  double acc = 0.0;
  if (k < nrec) {
    const int64_t i = (int64_t)s * nrec + k;
    const double a = alpha[s];
    cx<double> r = rho[i];
    const cx<double> v = ap[i];
    r = mk<double>(r.re - a * v.re, r.im - a * v.im);
    rho[i] = r;
    acc = r.re * r.re + r.im * r.im;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[(int64_t)s * gridDim.x + blockIdx.x] = t;
}

// p_s = rho_s + beta_s p_s (beta_s < 0: the pair has stopped, p_s = 0)
__global__ __launch_bounds__(256) void k_wri_direction(cx<double>* __restrict__ p, const cx<double>* __restrict__ rho,
                                                       const double* __restrict__ beta, int nrec) {
  const int s = blockIdx.y;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= nrec) return;
  const int64_t i = (int64_t)s * nrec + k;
  const double b = beta[s];
  if (b < 0.0) {
    p[i] = czero<double>();
  } else {
    const cx<double> r = rho[i], v = p[i];
    p[i] = mk<double>(r.re + b * v.re, r.im + b * v.im);
  }
}

// u_s += alpha_s z_s over the N points of every pair (FP64)
__global__ __launch_bounds__(256) void k_wri_field(cx<double>* __restrict__ u, const cx<double>* __restrict__ z,
                                                   const double* __restrict__ alpha, int64_t N) {
  const int s = blockIdx.y;
  const double a = alpha[s];
  if (a == 0.0) return;
  cx<double>* us = u + s * N;
  const cx<double>* zs = z + s * N;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
    const cx<double> v = zs[i];
    cx<double> w = us[i];
    us[i] = mk<double>(w.re + a * v.re, w.im + a * v.im);
  }
}

}  // namespace helm
