// Adjoint-state misfit / gradient kernels (arXiv:1703.09268, Listing of
// PDEfunc cases OBJ, JACOB_FORW, JACOB_ADJ, HESS_GN, HESS; Table derivstuff;
// Appendix A eqs. dH, dHadj, DTadj), over a list of (frequency, source)
// pairs solved together:
//   q_p = amp_p P_s^T 1 / h^3                     (point source: on a node, or
//                                                   the windowed sinc around it)
//   r_p = P_r u_p - d_p,  f = 1/2 sum_p ||r_p||^2  (FP64 accumulation)
//   b_p = -P_r^T r_p                               (adjoint source)
//   g   = sum_p Re(w_p conj(u_p) (A^H v_p))        (gradient w.r.t. real m,
//                                                   w_p = omega_p^2 [/ #pairs])
// Pair p's forward field starts at element uoff[p] of its array (the fields
// may live in a caller's [frequency][source] store); right-hand sides,
// adjoint fields and receiver residuals are contiguous per pair.  Receivers
// that share a node are summed in a fixed order (node-sorted receiver
// lists), so the adjoint source is deterministic.
#pragma once

#include "common.h"

namespace helm {

// Sources and receivers are weighted node lists (CSR): entry e of point k is
// node lin[e] with weight w[e], e in [ptr[k], ptr[k+1]).  An on-node point is
// one entry of weight 1; an off-grid point the windowed-sinc stencil around
// it (nodes inside the grid only).

// q[s] += amp_s w_e / h^3 at the nodes of pair s's source (q zeroed before;
// the nodes of one source are distinct).  Grid: (entry blocks, pairs).
template <typename T>
__global__ __launch_bounds__(256) void k_point_sources(cx<T>* __restrict__ q, int64_t N,
                                                       const int* __restrict__ src_of_pair,
                                                       const int* __restrict__ ptr, const int64_t* __restrict__ lin,
                                                       const double* __restrict__ w,
                                                       const double2* __restrict__ amp, double inv_h3) {
  const int s = blockIdx.y;
  const int k = src_of_pair[s];
  const double2 a = amp[s];
  for (int e = ptr[k] + blockIdx.x * 256 + threadIdx.x; e < ptr[k + 1]; e += gridDim.x * 256) {
    const double c = w[e] * inv_h3;
    q[s * N + lin[e]] = mk<T>((T)(a.x * c), (T)(a.y * c));
  }
}

// r[s][k] = (P_r u_s)_k - d[drow_s][k] (s: pair); per-workgroup
// partial sum of |r|^2 in part[s * gridDim.x + blk] (FP64).  u may be the
// FP64 outer iterate of the solve (TU = double): the residual is a small
// difference of two fields, so it is formed before the fields are rounded to
// the storage precision.
template <typename TU, typename T>
__global__ __launch_bounds__(256) void k_sample_residual(const cx<TU>* __restrict__ u,
                                                         const int64_t* __restrict__ uoff,
                                                         const int* __restrict__ rptr,
                                                         const int64_t* __restrict__ rlin,
                                                         const double* __restrict__ rw, int nrec,
                                                         const cx<T>* __restrict__ d,
                                                         const int64_t* __restrict__ drow,
                                                         cx<T>* __restrict__ res, double* __restrict__ part) {
  __shared__ double red[16];
  const int s = blockIdx.y;
  const int k = blockIdx.x * 256 + threadIdx.x;
  double acc = 0.0;
  if (k < nrec) {
    cx<double> uv = czero<double>();
    const cx<TU>* us = u + uoff[s];
    for (int e = rptr[k]; e < rptr[k + 1]; ++e) uv = uv + rw[e] * cast<double>(us[rlin[e]]);
    const cx<T> dv = d[drow[s] * nrec + k];
    const cx<double> rr = mk<double>(uv.re - (double)dv.re, uv.im - (double)dv.im);
    res[(int64_t)s * nrec + k] = cast<T>(rr);
    acc = rr.re * rr.re + rr.im * rr.im;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[(int64_t)s * gridDim.x + blockIdx.x] = t;
}

// b[s] (+)= -P_r^T r[rrow_s]: one lane per distinct node any receiver
// touches, summing that node's (receiver, weight) entries in a fixed order
// (node_ptr / node_rec / node_w: CSR over distinct nodes, ascending).  rrow (row of pair s in r; null: row s).  Without ADD, b must
// be zero beforehand.
template <typename T, bool ADD = false>
__global__ __launch_bounds__(256) void k_adjoint_source(cx<T>* __restrict__ b, int64_t N,
                                                        const int64_t* __restrict__ node_lin,
                                                        const int* __restrict__ node_ptr,
                                                        const int* __restrict__ node_rec,
                                                        const double* __restrict__ node_w, int nnode,
                                                        const cx<T>* __restrict__ res, int nrec,
                                                        const int64_t* __restrict__ rrow = nullptr) {
  const int s = blockIdx.y;
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= nnode) return;
  const int64_t row = rrow ? rrow[s] : s;
  cx<double> acc = czero<double>();
  for (int e = node_ptr[q]; e < node_ptr[q + 1]; ++e)
    acc = acc + node_w[e] * cast<double>(res[row * nrec + node_rec[e]]);
  cx<T>* dst = b + s * N + node_lin[q];
  if (ADD) acc = mk<double>(acc.re - (double)dst->re, acc.im - (double)dst->im);
  *dst = cast<T>(mk<double>(-acc.re, -acc.im));
}

// out[orow_s][k] = (P_r u_s)_k: receiver sampling of pair s's field (u may be
// an FP64 outer iterate).
template <typename TU, typename T>
__global__ __launch_bounds__(256) void k_sample(const cx<TU>* __restrict__ u, const int64_t* __restrict__ uoff,
                                                const int* __restrict__ rptr, const int64_t* __restrict__ rlin,
                                                const double* __restrict__ rw, int nrec,
                                                cx<T>* __restrict__ out, const int64_t* __restrict__ orow) {
  const int s = blockIdx.y;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= nrec) return;
  cx<double> uv = czero<double>();
  const cx<TU>* us = u + uoff[s];
  for (int e = rptr[k]; e < rptr[k + 1]; ++e) uv = uv + rw[e] * cast<double>(us[rlin[e]]);
  out[orow[s] * nrec + k] = cast<T>(uv);
}

// Right-hand sides of the linearised problems (Appendix A, eqs. dH and the
// derivative of the adjoint equation), pair s, w_s = omega_s^2:
//   DHADJ = false:  out_s = -w_s A (x_s * dm)     (-T dm, x = the forward field)
//   DHADJ = true:   out_s = -w_s dm * (A x_s)     (-DH[dm]^H x, x = an adjoint field)
// A = I (7-point) or the 27-point mass distribution (real symmetric, zero
// outside the grid).  x_s starts at x + xoff[s]; out is contiguous per pair.
template <typename TX, typename T, bool MASS27, bool DHADJ>
__global__ __launch_bounds__(256) void k_born_source(const cx<TX>* __restrict__ x, const int64_t* __restrict__ xoff,
                                                     const T* __restrict__ dm, int npair, int nx, int ny, int nz,
                                                     const double* __restrict__ w, double mw0, double mw1,
                                                     double mw2, double mw3, cx<T>* __restrict__ out) {
  const int64_t N = (int64_t)nx * ny * nz;
  const int64_t stride = (int64_t)gridDim.x * 256;
  const int s = blockIdx.y;
  const cx<TX>* xs = x + xoff[s];
  const double ws = w[s];
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < N; p += stride) {
    cx<double> acc;
    if (!MASS27) {
      acc = (double)dm[p] * cast<double>(xs[p]);
    } else {
      const int k = (int)(p % nz);
      const int j = (int)((p / nz) % ny);
      const int i = (int)(p / ((int64_t)ny * nz));
      const double mw[4] = {mw0, mw1, mw2, mw3};
      acc = czero<double>();
      for (int di = -1; di <= 1; ++di) {
        if (i + di < 0 || i + di >= nx) continue;
        for (int dj = -1; dj <= 1; ++dj) {
          if (j + dj < 0 || j + dj >= ny) continue;
          for (int dk = -1; dk <= 1; ++dk) {
            if (k + dk < 0 || k + dk >= nz) continue;
            const int cls = (di != 0) + (dj != 0) + (dk != 0);
            const int64_t q = p + (int64_t)di * ny * nz + (int64_t)dj * nz + dk;
            const double f = DHADJ ? mw[cls] : mw[cls] * (double)dm[q];
            acc = acc + f * cast<double>(xs[q]);
          }
        }
      }
      if (DHADJ) acc = (double)dm[p] * acc;
    }
    out[s * N + p] = cast<T>(mk<double>(-ws * acc.re, -ws * acc.im));
  }
}

// x[0..n) = 0 (real)
template <typename T>
__global__ __launch_bounds__(256) void k_fill_zero_real(T* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) x[i] = T(0);
}

// g[p] (+)= sum_s Re(w_s conj(u_s[p]) (A v_s)[p]) over the pairs s, with
// A = I (7-point) or the 27-point mass distribution (real symmetric,
// A^H = A); u_s starts at u + uoff[s], v_s at v + s N.
template <typename TU, typename T, typename TG, bool MASS27>
__global__ __launch_bounds__(256) void k_gradient(const cx<TU>* __restrict__ u, const int64_t* __restrict__ uoff,
                                                  const cx<T>* __restrict__ v, int npair, int nx, int ny, int nz,
                                                  const double* __restrict__ w, double mw0, double mw1, double mw2,
                                                  double mw3, TG* __restrict__ g, bool accumulate) {
  const int64_t N = (int64_t)nx * ny * nz;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < N; p += stride) {
    double acc = 0.0;
    int i = 0, j = 0, k = 0;
    if (MASS27) {
      k = (int)(p % nz);
      j = (int)((p / nz) % ny);
      i = (int)(p / ((int64_t)ny * nz));
    }
    for (int s = 0; s < npair; ++s) {
      const cx<TU> us = u[uoff[s] + p];
      cx<double> av;
      if (!MASS27) {
        av = cast<double>(v[s * N + p]);
      } else {
        const double mw[4] = {mw0, mw1, mw2, mw3};
        av = czero<double>();
        for (int di = -1; di <= 1; ++di) {
          if (i + di < 0 || i + di >= nx) continue;
          for (int dj = -1; dj <= 1; ++dj) {
            if (j + dj < 0 || j + dj >= ny) continue;
            for (int dk = -1; dk <= 1; ++dk) {
              if (k + dk < 0 || k + dk >= nz) continue;
              const int cls = (di != 0) + (dj != 0) + (dk != 0);
              const cx<double> vq = cast<double>(v[s * N + p + (int64_t)di * ny * nz + (int64_t)dj * nz + dk]);
              av = av + mw[cls] * vq;
            }
          }
        }
      }
      // w Re(conj(u) * av)
      acc += w[s] * ((double)us.re * av.re + (double)us.im * av.im);
    }
    g[p] = accumulate ? (TG)((double)g[p] + acc) : (TG)acc;
  }
}

}  // namespace helm
