// Grid-transfer kernels of the multilevel V-cycle (arXiv:1703.09268, ML-GMRES
// section: linear interpolation as prolongation, its adjoint as restriction).
//
// Coarse grid: n_c = floor(n_f/2) + 1 nodes per axis, coarse node I at fine
// node 2I.  P is the tensor product of 1D linear interpolation (even fine node
// 2I <- coarse I; odd fine node 2I+1 <- (coarse I + coarse I+1)/2).  The
// restriction is R = P^T / 8, the adjoint of P in the h^3-weighted inner
// product, i.e. full weighting
//   (R r)_I = (1/8) sum_{d in {-1,0,1}^3} prod_a (1 - |d_a|/2) r_{2I+d}.
// The coarse model is injected: m_c(I) = m_f(min(2I, n_f - 1)).
#pragma once

#include "common.h"

namespace helm {

// rc = R (s_r * rf)  with per-rhs scale s_r (may be null)
template <typename T>
__global__ __launch_bounds__(256) void k_restrict(const cx<T>* __restrict__ rf, const double* __restrict__ rs,
                                                  int nfx, int nfy, int nfz, cx<T>* __restrict__ rc,
                                                  int ncx, int ncy, int ncz,
                                                  const int* __restrict__ active) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int64_t Nc = (int64_t)ncx * ncy * ncz;
  const int64_t Nf = (int64_t)nfx * nfy * nfz;
  const int64_t pc = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (pc >= Nc) return;
  const int K = (int)(pc % ncz);
  const int J = (int)((pc / ncz) % ncy);
  const int I = (int)(pc / ((int64_t)ncy * ncz));
  const cx<T>* f = rf + r * Nf;
  cx<T> acc = czero<T>();
  for (int di = -1; di <= 1; ++di) {
    const int i = 2 * I + di;
    if (i < 0 || i >= nfx) continue;
    const T wi = di ? T(0.5) : T(1);
    for (int dj = -1; dj <= 1; ++dj) {
      const int j = 2 * J + dj;
      if (j < 0 || j >= nfy) continue;
      const T wj = dj ? T(0.5) : T(1);
      for (int dk = -1; dk <= 1; ++dk) {
        const int k = 2 * K + dk;
        if (k < 0 || k >= nfz) continue;
        const T wk = dk ? T(0.5) : T(1);
        acc = acc + (wi * wj * wk) * f[((int64_t)i * nfy + j) * nfz + k];
      }
    }
  }
  const T s = rs ? (T)rs[r] : T(1);
  rc[r * Nc + pc] = (s * T(0.125)) * acc;
}

// xf += P xc
template <typename T>
__global__ __launch_bounds__(256) void k_prolong_add(const cx<T>* __restrict__ xc, int ncx, int ncy,
                                                     int ncz, cx<T>* __restrict__ xf, int nfx, int nfy,
                                                     int nfz, const int* __restrict__ active) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int64_t Nc = (int64_t)ncx * ncy * ncz;
  const int64_t Nf = (int64_t)nfx * nfy * nfz;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= Nf) return;
  const int k = (int)(p % nfz);
  const int j = (int)((p / nfz) % nfy);
  const int i = (int)(p / ((int64_t)nfy * nfz));
  // 1D stencils: (index, weight) pairs, second entry weight 0 for even nodes
  const int i0 = i >> 1, i1 = (i + 1) >> 1;
  const int j0 = j >> 1, j1 = (j + 1) >> 1;
  const int k0 = k >> 1, k1 = (k + 1) >> 1;
  const T wi = (i & 1) ? T(0.5) : T(1), wj = (j & 1) ? T(0.5) : T(1), wk = (k & 1) ? T(0.5) : T(1);
  const cx<T>* c = xc + r * Nc;
  auto at = [&](int a, int b, int d) { return c[((int64_t)a * ncy + b) * ncz + d]; };
  cx<T> acc = at(i0, j0, k0);
  if (k & 1) acc = acc + at(i0, j0, k1);
  cx<T> s2 = acc;
  if (j & 1) {
    cx<T> t = at(i0, j1, k0);
    if (k & 1) t = t + at(i0, j1, k1);
    s2 = s2 + t;
  }
  cx<T> s3 = s2;
  if (i & 1) {
    cx<T> t = at(i1, j0, k0);
    if (k & 1) t = t + at(i1, j0, k1);
    if (j & 1) {
      cx<T> u = at(i1, j1, k0);
      if (k & 1) u = u + at(i1, j1, k1);
      t = t + u;
    }
    s3 = s3 + t;
  }
  xf[r * Nf + p] = xf[r * Nf + p] + (wi * wj * wk) * s3;
}

template <typename TM>
__global__ __launch_bounds__(256) void k_inject_model(const TM* __restrict__ mf, int nfx, int nfy, int nfz,
                                                      TM* __restrict__ mc, int ncx, int ncy, int ncz) {
  const int64_t Nc = (int64_t)ncx * ncy * ncz;
  const int64_t pc = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (pc >= Nc) return;
  const int K = (int)(pc % ncz);
  const int J = (int)((pc / ncz) % ncy);
  const int I = (int)(pc / ((int64_t)ncy * ncz));
  const int i = min(2 * I, nfx - 1), j = min(2 * J, nfy - 1), k = min(2 * K, nfz - 1);
  mc[pc] = mf[((int64_t)i * nfy + j) * nfz + k];
}

}  // namespace helm
