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
// All kernels are point-wise over the segments of one level (tmap of the
// level whose points the lanes own); fine and coarse descriptors of a
// segment share its index.  Vectors use each level's z pitch; pad entries of
// the coarse outputs are written as zero, fine pads are left untouched.
#pragma once

#include "common.h"
#include "segment.h"

namespace helm {

// rc = R (s_r * rf); lanes own coarse points
template <typename T>
__global__ __launch_bounds__(256) void k_restrict(const Seg* __restrict__ fsegs, const Seg* __restrict__ csegs,
                                                  const int* __restrict__ ctmap, const cx<T>* __restrict__ rf,
                                                  const double* __restrict__ rs, cx<T>* __restrict__ rc,
                                                  const int* __restrict__ active) {
  const int wg = blockIdx.x;
  const int sid = ctmap[wg];
  if (active && !active[sid]) return;
  const Seg& C = csegs[sid];
  const Seg& F = fsegs[sid];
  const int64_t pc = (int64_t)(wg - C.tblk0) * 256 + threadIdx.x;
  if (pc >= C.N) return;
  const int ncy = C.n[1], ncz = C.n[2], cpz = C.pz;
  const int nfx = F.n[0], nfy = F.n[1], nfz = F.n[2], fpz = F.pz;
  const int K = (int)(pc % cpz);
  const int J = (int)((pc / cpz) % ncy);
  const int I = (int)(pc / ((int64_t)ncy * cpz));
  if (K >= ncz) {
    rc[C.off + pc] = czero<T>();
    return;
  }
  const cx<T>* f = rf + F.off;
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
        acc = acc + (wi * wj * wk) * f[((int64_t)i * nfy + j) * fpz + k];
      }
    }
  }
  const T s = rs ? (T)rs[sid] : T(1);
  // 1/2 per coarsened axis: 1/8, or 1/4 on a 2D grid (an axis of one node)
  const T w = (nfx > 1 ? T(0.5) : T(1)) * (nfy > 1 ? T(0.5) : T(1)) * (nfz > 1 ? T(0.5) : T(1));
  rc[C.off + pc] = (s * w) * acc;
}

// xf += P xc; lanes own fine points
template <typename T>
__global__ __launch_bounds__(256) void k_prolong_add(const Seg* __restrict__ fsegs, const Seg* __restrict__ csegs,
                                                     const int* __restrict__ ftmap, const cx<T>* __restrict__ xc,
                                                     cx<T>* __restrict__ xf, const int* __restrict__ active) {
  const int wg = blockIdx.x;
  const int sid = ftmap[wg];
  if (active && !active[sid]) return;
  const Seg& F = fsegs[sid];
  const Seg& C = csegs[sid];
  const int64_t p = (int64_t)(wg - F.tblk0) * 256 + threadIdx.x;
  if (p >= F.N) return;
  const int nfy = F.n[1], nfz = F.n[2], fpz = F.pz;
  const int ncy = C.n[1], cpz = C.pz;
  const int k = (int)(p % fpz);
  const int j = (int)((p / fpz) % nfy);
  const int i = (int)(p / ((int64_t)nfy * fpz));
  if (k >= nfz) return;
  // even node: one coarse node (weight 1); odd node: two (weight 1/2 each)
  const int i0 = i >> 1, i1 = (i + 1) >> 1;
  const int j0 = j >> 1, j1 = (j + 1) >> 1;
  const int k0 = k >> 1, k1 = (k + 1) >> 1;
  const T wi = (i & 1) ? T(0.5) : T(1), wj = (j & 1) ? T(0.5) : T(1), wk = (k & 1) ? T(0.5) : T(1);
  const cx<T>* c = xc + C.off;
  auto at = [&](int a, int b, int d) { return c[((int64_t)a * ncy + b) * cpz + d]; };
  cx<T> s2 = at(i0, j0, k0);
  if (k & 1) s2 = s2 + at(i0, j0, k1);
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
  xf[F.off + p] = xf[F.off + p] + (wi * wj * wk) * s3;
}

// coarse model by injection, one lane per coarse point of the segments that
// own their model buffer (own[sid] != 0)
template <typename TM>
__global__ __launch_bounds__(256) void k_inject_model(const Seg* __restrict__ fsegs, const Seg* __restrict__ csegs,
                                                      const int* __restrict__ ctmap,
                                                      const int* __restrict__ own) {
  const int wg = blockIdx.x;
  const int sid = ctmap[wg];
  if (!own[sid]) return;
  const Seg& C = csegs[sid];
  const Seg& F = fsegs[sid];
  const int64_t pc = (int64_t)(wg - C.tblk0) * 256 + threadIdx.x;
  if (pc >= C.N) return;
  const int ncy = C.n[1], ncz = C.n[2], cpz = C.pz;
  const int K = (int)(pc % cpz);
  const int J = (int)((pc / cpz) % ncy);
  const int I = (int)(pc / ((int64_t)ncy * cpz));
  TM* mc = reinterpret_cast<TM*>(const_cast<void*>(C.m));
  if (K >= ncz) {
    mc[pc] = TM(0);
    return;
  }
  const int i = min(2 * I, F.n[0] - 1), j = min(2 * J, F.n[1] - 1), k = min(2 * K, F.n[2] - 1);
  const TM* mf = reinterpret_cast<const TM*>(F.m);
  mc[pc] = mf[((int64_t)i * F.n[1] + j) * F.pz + k];
}

}  // namespace helm
