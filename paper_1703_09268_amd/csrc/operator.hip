// Host-side description of one discrete Helmholtz operator (one grid level)
// and the launch wrappers of the stencil kernels.
//
// Level l of the multigrid hierarchy has n_l = floor(n_{l-1}/2) + 1 nodes per
// axis, spacing 2^l h, the same omega, and the absorbing-layer profile of the
// fine grid evaluated at fine coordinates 2^l I and 2^l (I +- 1/2)
// (re-discretisation of the same problem on the coarser grid; arXiv:1703.09268,
// ML-GMRES section, where the coarse problem is "an instance of the original
// problem").
#pragma once

#include <cmath>
#include <complex>
#include <vector>

#include "common.h"
#include "stencil.hip"

namespace helm {

// Simple owning device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void ensure(size_t b) {
    if (b <= bytes) return;
    release();
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error{-2, "hipMalloc of " + std::to_string(b) + " bytes failed"};
    }
    bytes = b;
  }
};

struct GridSpec {
  int n[3];
  double h;
  int npml;
  double R;
  double vref;
  int stencil;  // 0 7-pt, 1 27-pt
  double w27[7];
};

// Damping profile of the layer at fine coordinate tf (fine-grid node units).
inline double layer_sigma(const GridSpec& g, int axis, double tf) {
  if (g.npml == 0) return 0.0;
  const double nf = g.n[axis];
  const double d = std::max(0.0, std::max(g.npml - tf, tf - (nf - 1 - g.npml)));
  const double smax = 3.0 * g.vref * std::log(1.0 / g.R) / (2.0 * g.npml * g.h);
  return smax * (d / g.npml) * (d / g.npml);
}

struct Level {
  int n[3];
  int64_t N;
  double h;
  int stride;
  int stencil;
  Int27 in27;
  double omega;
  // layer tables, [dir][axis][kind][n_axis], kinds alpha, beta, delta
  DevBuf tabf, tabd;
  Tab7<float> tf[2];
  Tab7<double> td[2];
  std::vector<std::complex<double>> host[2][3][3];
  // model on this level (level 0 borrows the caller's pointer)
  const void* m = nullptr;
  DevBuf m_own;
};

// Fill the host tables of level L for grid g at this level's stride.
inline void build_tables(const GridSpec& g, Level& L) {
  typedef std::complex<double> C;
  const double w = L.omega;
  for (int a = 0; a < 3; ++a) {
    const int n = L.n[a];
    auto s_at = [&](double t) { return C(1.0, layer_sigma(g, a, t * L.stride) / w); };
    std::vector<C> cp(n), cm(n);
    for (int i = 0; i < n; ++i) {
      const C s0 = s_at(i), sp = s_at(i + 0.5), sm = s_at(i - 0.5);
      cp[i] = 1.0 / (L.h * L.h * s0 * sp);
      cm[i] = 1.0 / (L.h * L.h * s0 * sm);
    }
    for (int d = 0; d < 3; ++d) L.host[0][a][d].assign(n, C(0, 0));
    for (int d = 0; d < 3; ++d) L.host[1][a][d].assign(n, C(0, 0));
    for (int i = 0; i < n; ++i) {
      // forward: alpha = cp, beta = cm, delta = 0
      L.host[0][a][0][i] = cp[i];
      L.host[0][a][1][i] = cm[i];
      // adjoint: conj of the transposed couplings
      const C al = (i + 1 < n) ? std::conj(cm[i + 1]) : C(0, 0);
      const C be = (i > 0) ? std::conj(cp[i - 1]) : C(0, 0);
      const C ga = -std::conj(cp[i] + cm[i]);
      L.host[1][a][0][i] = al;
      L.host[1][a][1][i] = be;
      L.host[1][a][2][i] = ga + al + be;
    }
  }
  // 27-point interior range per axis: rows whose +-1 neighbours are damping-free
  for (int a = 0; a < 3; ++a) {
    int lo = 1, hi = 0;
    bool found = false;
    for (int i = 0; i < L.n[a]; ++i) {
      const bool ok = layer_sigma(g, a, (double)(i - 1) * L.stride) == 0.0 &&
                      layer_sigma(g, a, (double)(i + 1) * L.stride) == 0.0;
      if (ok && !found) { lo = i; found = true; }
      if (ok) hi = i;
    }
    L.in27.lo[a] = lo;
    L.in27.hi[a] = found ? hi : lo - 1;
  }
  const double w1 = g.w27[0], w2 = g.w27[1], w3 = g.w27[2];
  const double h2 = L.h * L.h;
  L.in27.lw[0] = (w1 * -6.0 + w2 * (-6.0 / 3.0 - 12.0 / 6.0) + w3 * (-8.0 / 4.0)) / h2;
  L.in27.lw[1] = (w1 * 1.0 + w2 * (1.0 / 3.0)) / h2;
  L.in27.lw[2] = (w2 * (1.0 / 6.0)) / h2;
  L.in27.lw[3] = (w3 * (1.0 / 4.0)) / h2;
  for (int c = 0; c < 4; ++c) L.in27.mw[c] = g.w27[3 + c];
  if (g.stencil == 0) {
    L.in27.lw[0] = L.in27.lw[1] = L.in27.lw[2] = L.in27.lw[3] = 0.0;
    L.in27.mw[0] = 1.0;
    L.in27.mw[1] = L.in27.mw[2] = L.in27.mw[3] = 0.0;
  }
}

// Upload the tables in both precisions (the mixed-precision residual uses
// the double tables on the complex64 path).
inline void upload_tables(Level& L, hipStream_t st) {
  const size_t tot = (size_t)2 * 3 * (L.n[0] + L.n[1] + L.n[2]);
  L.tabd.ensure(tot * sizeof(cx<double>));
  L.tabf.ensure(tot * sizeof(cx<float>));
  std::vector<cx<double>> hd(tot);
  std::vector<cx<float>> hf(tot);
  size_t off = 0;
  for (int dir = 0; dir < 2; ++dir)
    for (int a = 0; a < 3; ++a)
      for (int kind = 0; kind < 3; ++kind) {
        cx<double>* pd = reinterpret_cast<cx<double>*>(L.tabd.p) + off;
        cx<float>* pf = reinterpret_cast<cx<float>*>(L.tabf.p) + off;
        if (kind == 0) { L.td[dir].al[a] = pd; L.tf[dir].al[a] = pf; }
        if (kind == 1) { L.td[dir].be[a] = pd; L.tf[dir].be[a] = pf; }
        if (kind == 2) { L.td[dir].de[a] = pd; L.tf[dir].de[a] = pf; }
        const auto& v = L.host[dir][a][kind];
        for (size_t i = 0; i < v.size(); ++i) {
          hd[off + i] = mk<double>(v[i].real(), v[i].imag());
          hf[off + i] = mk<float>((float)v[i].real(), (float)v[i].imag());
        }
        off += v.size();
      }
  HELM_HIP_CHECK(hipMemcpyAsync(L.tabd.p, hd.data(), tot * sizeof(cx<double>), hipMemcpyHostToDevice, st));
  HELM_HIP_CHECK(hipMemcpyAsync(L.tabf.p, hf.data(), tot * sizeof(cx<float>), hipMemcpyHostToDevice, st));
  HELM_HIP_CHECK(hipStreamSynchronize(st));
}

inline void init_level(const GridSpec& g, Level& L, const int n[3], double h, int stride, double omega,
                       hipStream_t st) {
  for (int a = 0; a < 3; ++a) L.n[a] = n[a];
  L.N = (int64_t)n[0] * n[1] * n[2];
  L.h = h;
  L.stride = stride;
  L.stencil = g.stencil;
  L.omega = omega;
  build_tables(g, L);
  upload_tables(L, st);
}

template <typename T> inline const Tab7<T>& tab_of(const Level& L, int dir);
template <> inline const Tab7<float>& tab_of<float>(const Level& L, int dir) { return L.tf[dir]; }
template <> inline const Tab7<double>& tab_of<double>(const Level& L, int dir) { return L.td[dir]; }

// Launch geometry of the 7-point x-marching kernel.
struct Tile7 {
  int tz, ty, xchunk, nxc;
  dim3 grid;
};

inline Tile7 plan7(const Level& L, int nrhs) {
  Tile7 t;
  const int nz = L.n[2], ny = L.n[1], nx = L.n[0];
  if (nz >= 48) { t.tz = 64; t.ty = 4; }
  else if (nz >= 24) { t.tz = 32; t.ty = 8; }
  else { t.tz = 16; t.ty = 16; }
  const int gx = (int)ceil_div(nz, t.tz), gy = (int)ceil_div(ny, t.ty);
  const int64_t per_plane = (int64_t)gx * gy * nrhs;
  int nxc = (int)std::max<int64_t>(1, std::min<int64_t>(nx, (4096 + per_plane - 1) / per_plane));
  int xchunk = (nx + nxc - 1) / nxc;
  if (xchunk < 4) xchunk = std::min(nx, 4);
  nxc = (nx + xchunk - 1) / xchunk;
  t.xchunk = xchunk;
  t.nxc = nxc;
  t.grid = dim3(gx, gy, nxc * nrhs);
  return t;
}

inline int nblk_stencil(const Level& L, int nrhs) {
  if (L.stencil == 1) return (int)ceil_div(L.N, 256);
  const Tile7 t = plan7(L, nrhs);
  return (int)(t.grid.x * t.grid.y * t.nxc);
}

// out = [s_b b -] s_x H x  on nrhs right-hand sides.  Returns the number of
// partial-norm workgroups per right-hand side when NORM.
template <typename TC, typename TX, typename TM, typename TB, typename TO, bool RESID, bool NORM>
int launch_h(const Level& L, int adj, int nrhs, const cx<TX>* x, const double* xs, const TM* m,
             const cx<TB>* b, const double* bs, cx<TO>* out, double* part, const int* active,
             hipStream_t st) {
  const TC w2 = (TC)(L.omega * L.omega);
  const Tab7<TC>& tab = tab_of<TC>(L, adj);
  if (L.stencil == 1) {
    dim3 grid(ceil_div(L.N, 256), nrhs);
    if (adj)
      hipLaunchKernelGGL((k_h27<TC, TX, TM, TB, TO, true, RESID, NORM>), grid, dim3(256), 0, st, x, xs, m,
                         w2, tab, L.in27, b, bs, out, part, active, L.n[0], L.n[1], L.n[2]);
    else
      hipLaunchKernelGGL((k_h27<TC, TX, TM, TB, TO, false, RESID, NORM>), grid, dim3(256), 0, st, x, xs,
                         m, w2, tab, L.in27, b, bs, out, part, active, L.n[0], L.n[1], L.n[2]);
    return (int)grid.x;
  }
  const Tile7 t = plan7(L, nrhs);
#define HELM_L7(TZ, TY)                                                                        \
  hipLaunchKernelGGL((k_h7<TC, TX, TM, TB, TO, RESID, NORM, TZ, TY>), t.grid, dim3(TZ, TY), 0, st, \
                     x, xs, m, w2, tab, b, bs, out, part, active, L.n[0], L.n[1], L.n[2], t.xchunk, \
                     t.nxc)
  if (t.tz == 64) HELM_L7(64, 4);
  else if (t.tz == 32) HELM_L7(32, 8);
  else HELM_L7(16, 16);
#undef HELM_L7
  return (int)(t.grid.x * t.grid.y * t.nxc);
}

}  // namespace helm
