// Matrix-free Helmholtz stencils for gfx950.
//
// H = L + omega^2 A diag(m) on a [nx][ny][nz] grid, z fastest (Appendix A of
// arXiv:1703.09268, the system L u + omega^2 A diag(m) u = q; the layer of
// the Preamble's extended domain enters L through per-axis complex
// stretches).
//
// 7-point rows are evaluated in difference form from three per-axis
// coefficient tables (alpha, beta, delta), one entry per node index:
//
//   (Hx)_p = (omega^2 m_p + sum_a delta_a) x_p
//            + sum_a alpha_a (x_{p+e_a} - x_p) + beta_a (x_{p-e_a} - x_p)
//
// The forward operator uses alpha = cp, beta = cm, delta = 0; the adjoint
// H^H uses alpha(i) = conj(cm(i+1)), beta(i) = conj(cp(i-1)) and delta =
// conj(diag) + alpha + beta, so both directions run the same kernel with a
// different table.  The difference form keeps complex64 rounding relative to
// the local variation of x instead of to |x| / h^2.
//
// Kernel shape: a workgroup owns a TZ x TY tile of the (z, y) plane and marches
// along x over `xchunk` planes, holding x[i-1], x[i], x[i+1] of its own column
// in registers; y and z neighbours come from the vector cache (they are the
// neighbouring lanes' own loads).  z is the lane index, so every load and
// store is a contiguous 64-lane access; the x-axis coefficients are
// workgroup-uniform (scalar loads).
#pragma once

#include "common.h"

namespace helm {

template <typename T>
struct Tab7 {
  const cx<T>* al[3];
  const cx<T>* be[3];
  const cx<T>* de[3];
};

// 27-point interior description (compact stencil away from the layer).
struct Int27 {
  int lo[3], hi[3];  // rows i with lo <= i <= hi on every axis are interior
  double lw[4];      // Laplacian weights: centre, face, edge, corner
  double mw[4];      // mass weights: centre, face, edge, corner
};

template <typename TX, typename TC>
__device__ __forceinline__ cx<TC> ld(const cx<TX>* p) {
  return cast<TC>(*p);
}

// out = s_x * H x            (RESID = false)
// out = s_b * b - s_x * H x  (RESID = true)
// optional per-workgroup partial sum of |out|^2 (in TC precision -> double)
// written to part[(r * nblk + blk) * PSTRIDE].
template <typename TC, typename TX, typename TM, typename TB, typename TO,
          bool RESID, bool NORM, int TZ, int TY>
__global__ __launch_bounds__(TZ* TY) void k_h7(
    const cx<TX>* __restrict__ x, const double* __restrict__ xs,
    const TM* __restrict__ m, TC w2, Tab7<TC> tab,
    const cx<TB>* __restrict__ b, const double* __restrict__ bs,
    cx<TO>* __restrict__ out, double* __restrict__ part,
    const int* __restrict__ active, int nx, int ny, int nz, int xchunk,
    int nxc) {
  __shared__ double red[16];
  const int k = blockIdx.x * TZ + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int xc = blockIdx.z % nxc;
  const int r = blockIdx.z / nxc;
  const int nblk = gridDim.x * gridDim.y * nxc;
  const int blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * xc);
  if (active && !active[r]) {
    if (NORM && threadIdx.x == 0 && threadIdx.y == 0) part[((int64_t)r * nblk + blk) * PSTRIDE] = 0.0;
    return;  // uniform across the workgroup
  }
  const bool in = (k < nz) && (j < ny);
  const int64_t N = (int64_t)nx * ny * nz;
  const int64_t plane = (int64_t)ny * nz;
  const cx<TX>* xr = x + r * N;
  const TC sx = xs ? (TC)xs[r] : TC(1);
  const int i0 = xc * xchunk;
  const int i1 = min(nx, i0 + xchunk);
  cx<TC> az = czero<TC>(), bz = az, dz = az, ay = az, by = az, dy = az;
  if (in) {
    az = tab.al[2][k]; bz = tab.be[2][k]; dz = tab.de[2][k];
    ay = tab.al[1][j]; by = tab.be[1][j]; dy = tab.de[1][j];
  }
  int64_t p = (int64_t)i0 * plane + (int64_t)j * nz + k;
  cx<TC> xm = czero<TC>(), xcur = czero<TC>();
  if (in) {
    if (i0 > 0) xm = ld<TX, TC>(xr + p - plane);
    xcur = ld<TX, TC>(xr + p);
  }
  double nrm = 0.0;
  TC sb = TC(1);
  if (RESID) sb = bs ? (TC)bs[r] : TC(1);
  for (int i = i0; i < i1; ++i, p += plane) {
    cx<TC> xp = czero<TC>();
    if (in && i + 1 < nx) xp = ld<TX, TC>(xr + p + plane);
    if (in) {
      const cx<TC> ym = j > 0 ? ld<TX, TC>(xr + p - nz) : czero<TC>();
      const cx<TC> yp = j + 1 < ny ? ld<TX, TC>(xr + p + nz) : czero<TC>();
      const cx<TC> zm = k > 0 ? ld<TX, TC>(xr + p - 1) : czero<TC>();
      const cx<TC> zp = k + 1 < nz ? ld<TX, TC>(xr + p + 1) : czero<TC>();
      const cx<TC> ax = tab.al[0][i], bx = tab.be[0][i], dx = tab.de[0][i];
      const TC wm = w2 * (TC)m[p];
      cx<TC> acc = mk<TC>(wm + dx.re + dy.re + dz.re, dx.im + dy.im + dz.im) * xcur;
      acc = cfma(ax, xp - xcur, acc);
      acc = cfma(bx, xm - xcur, acc);
      acc = cfma(ay, yp - xcur, acc);
      acc = cfma(by, ym - xcur, acc);
      acc = cfma(az, zp - xcur, acc);
      acc = cfma(bz, zm - xcur, acc);
      acc = sx * acc;
      if (RESID) acc = sb * ld<TB, TC>(b + r * N + p) - acc;
      out[r * N + p] = cast<TO>(acc);
      if (NORM) nrm += (double)acc.re * (double)acc.re + (double)acc.im * (double)acc.im;
    }
    xm = xcur;
    xcur = xp;
  }
  if (NORM) {
    const double s = block_sum(nrm, red);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[((int64_t)r * nblk + blk) * PSTRIDE] = s;
  }
}

// ---------------------------------------------------------------------------
// compact 27-point operator (one output point per lane, neighbours through
// the vector cache).  Interior rows: L27 = sum over the 27 offsets of the
// class weight; layer rows: the 7-point stretched row from the tables.  Mass
// term on every row: omega^2 sum_d wm(class d) m_{p+d} x_{p+d}.
// Adjoint: L27 (mask . x) + L7^H ((1 - mask) . x) + omega^2 m_p (A x)_p.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool interior27(const Int27& in27, int i, int j, int k) {
  return i >= in27.lo[0] && i <= in27.hi[0] && j >= in27.lo[1] && j <= in27.hi[1] &&
         k >= in27.lo[2] && k <= in27.hi[2];
}

template <typename TC, typename TX, typename TM, typename TB, typename TO,
          bool ADJ, bool RESID, bool NORM>
__global__ __launch_bounds__(256) void k_h27(
    const cx<TX>* __restrict__ x, const double* __restrict__ xs,
    const TM* __restrict__ m, TC w2, Tab7<TC> tab, Int27 in27,
    const cx<TB>* __restrict__ b, const double* __restrict__ bs,
    cx<TO>* __restrict__ out, double* __restrict__ part,
    const int* __restrict__ active, int nx, int ny, int nz) {
  __shared__ double red[16];
  const int r = blockIdx.y;
  const int nblk = gridDim.x;
  const int64_t N = (int64_t)nx * ny * nz;
  if (active && !active[r]) {
    if (NORM && threadIdx.x == 0) part[((int64_t)r * nblk + blockIdx.x) * PSTRIDE] = 0.0;
    return;
  }
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool in = p < N;
  double nrm = 0.0;
  if (in) {
    const int k = (int)(p % nz);
    const int j = (int)((p / nz) % ny);
    const int i = (int)(p / ((int64_t)ny * nz));
    const cx<TX>* xr = x + r * N;
    const TC sx = xs ? (TC)xs[r] : TC(1);
    const TC lw[4] = {(TC)in27.lw[0], (TC)in27.lw[1], (TC)in27.lw[2], (TC)in27.lw[3]};
    const TC mw[4] = {(TC)in27.mw[0], (TC)in27.mw[1], (TC)in27.mw[2], (TC)in27.mw[3]};
    cx<TC> lap = czero<TC>(), mass = czero<TC>();
    const bool own_int = interior27(in27, i, j, k);
    const cx<TC> xcur = ld<TX, TC>(xr + p);
    cx<TC> nb7[6];  // 7-point neighbours (with the adjoint mask applied)
#pragma unroll
    for (int q = 0; q < 6; ++q) nb7[q] = czero<TC>();
    for (int di = -1; di <= 1; ++di) {
      const int ii = i + di;
      if (ii < 0 || ii >= nx) continue;
      for (int dj = -1; dj <= 1; ++dj) {
        const int jj = j + dj;
        if (jj < 0 || jj >= ny) continue;
        for (int dk = -1; dk <= 1; ++dk) {
          const int kk = k + dk;
          if (kk < 0 || kk >= nz) continue;
          const int cls = (di != 0) + (dj != 0) + (dk != 0);
          const int64_t q = p + (int64_t)di * ny * nz + (int64_t)dj * nz + dk;
          const cx<TC> xq = (cls == 0) ? xcur : ld<TX, TC>(xr + q);
          if (!ADJ) {
            if (own_int) lap = cfma(mk<TC>(lw[cls], 0), xq, lap);
            mass = cfma(mk<TC>(mw[cls] * (TC)m[q], 0), xq, mass);
          } else {
            const bool qint = interior27(in27, ii, jj, kk);
            if (qint) lap = cfma(mk<TC>(lw[cls], 0), xq, lap);
            mass = cfma(mk<TC>(mw[cls], 0), xq, mass);
            if (cls == 1 && !qint) {
              const int slot = di ? (di < 0 ? 0 : 1) : dj ? (dj < 0 ? 2 : 3) : (dk < 0 ? 4 : 5);
              nb7[slot] = xq;
            }
          }
        }
      }
    }
    if (!ADJ) {
      if (!own_int) {
        const cx<TC> xmx = i > 0 ? ld<TX, TC>(xr + p - (int64_t)ny * nz) : czero<TC>();
        const cx<TC> xpx = i + 1 < nx ? ld<TX, TC>(xr + p + (int64_t)ny * nz) : czero<TC>();
        const cx<TC> xmy = j > 0 ? ld<TX, TC>(xr + p - nz) : czero<TC>();
        const cx<TC> xpy = j + 1 < ny ? ld<TX, TC>(xr + p + nz) : czero<TC>();
        const cx<TC> xmz = k > 0 ? ld<TX, TC>(xr + p - 1) : czero<TC>();
        const cx<TC> xpz = k + 1 < nz ? ld<TX, TC>(xr + p + 1) : czero<TC>();
        cx<TC> d = tab.de[0][i] + tab.de[1][j] + tab.de[2][k];
        lap = d * xcur;
        lap = cfma(tab.al[0][i], xpx - xcur, lap);
        lap = cfma(tab.be[0][i], xmx - xcur, lap);
        lap = cfma(tab.al[1][j], xpy - xcur, lap);
        lap = cfma(tab.be[1][j], xmy - xcur, lap);
        lap = cfma(tab.al[2][k], xpz - xcur, lap);
        lap = cfma(tab.be[2][k], xmz - xcur, lap);
      }
      lap = lap + w2 * mass;
    } else {
      // L7^H applied to x' = (1 - mask) . x: own value masked too
      const cx<TC> xo = own_int ? czero<TC>() : xcur;
      cx<TC> l7 = (tab.de[0][i] + tab.de[1][j] + tab.de[2][k]) * xo;
      l7 = cfma(tab.be[0][i], nb7[0] - xo, l7);
      l7 = cfma(tab.al[0][i], nb7[1] - xo, l7);
      l7 = cfma(tab.be[1][j], nb7[2] - xo, l7);
      l7 = cfma(tab.al[1][j], nb7[3] - xo, l7);
      l7 = cfma(tab.be[2][k], nb7[4] - xo, l7);
      l7 = cfma(tab.al[2][k], nb7[5] - xo, l7);
      lap = lap + l7 + (w2 * (TC)m[p]) * mass;
    }
    cx<TC> acc = sx * lap;
    if (RESID) {
      const TC sb = bs ? (TC)bs[r] : TC(1);
      acc = sb * ld<TB, TC>(b + r * N + p) - acc;
    }
    out[r * N + p] = cast<TO>(acc);
    if (NORM) nrm = (double)acc.re * (double)acc.re + (double)acc.im * (double)acc.im;
  }
  if (NORM) {
    const double s = block_sum(nrm, red);
    if (threadIdx.x == 0) part[((int64_t)r * nblk + blockIdx.x) * PSTRIDE] = s;
  }
}

}  // namespace helm
