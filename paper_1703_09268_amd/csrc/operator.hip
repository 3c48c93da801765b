// Host-side setup of the discrete operators of a solve: layer tables per
// distinct (grid, omega, level), the segments of every level with their
// workgroup maps, the coarse models, and the stencil launch wrapper.
//
// Level l of the multigrid hierarchy has n_l = floor(n_{l-1}/2) + 1 nodes per
// axis, spacing 2^l h, the same omega, and the absorbing-layer profile of the
// fine grid evaluated at fine coordinates 2^l I and 2^l (I +- 1/2)
// (re-discretisation of the same problem on the coarser grid; arXiv:1703.09268,
// ML-GMRES section, where the coarse problem is an instance of the original
// one).  The coarse model is injected from the next finer level.
#pragma once

#include <cmath>
#include <complex>
#include <cstdlib>
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <sys/stat.h>
#include <map>
#include <mutex>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "common.h"
#include "krylov.hip"
#include "segment.h"
#include "stencil.hip"
#include "transfer.hip"

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
      (void)hipGetLastError();
      p = nullptr;
      throw Error{-2, "hipMalloc of " + std::to_string(b) + " bytes failed"};
    }
    bytes = b;
  }
  template <typename T>
  T* as() const { return reinterpret_cast<T*>(p); }
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

// One problem of a solve (fine level).
struct ProblemSpec {
  GridSpec g;
  double omega;
  int dir;         // 0: H, 1: H^H
  const void* m;   // fine model (device)
};

// Damping profile of the layer at fine coordinate tf (fine-grid node units).
inline double layer_sigma(const GridSpec& g, int axis, double tf) {
  if (g.npml == 0) return 0.0;
  const double nf = g.n[axis];
  const double d = std::max(0.0, std::max(g.npml - tf, tf - (nf - 1 - g.npml)));
  const double smax = 3.0 * g.vref * std::log(1.0 / g.R) / (2.0 * g.npml * g.h);
  return smax * (d / g.npml) * (d / g.npml);
}

// Layer tables and 27-point description of one operator on one level.
struct OpTables {
  int n[3];
  DevBuf tabf, tabd;  // [dir][axis][alpha, beta, delta][n_axis]
  int tpre[3], tdir;
  Int27 in27;
};

// 27-point description of one operator on one level: the interior range per
// axis (rows whose +-1 neighbours are damping-free) and the class weights of
// the compact Laplacian and of the mass distribution (7-point: no interior
// rows used, mass = identity).
inline Int27 interior27_desc(const GridSpec& g, const int n[3], double h, int stride) {
  Int27 in27;
  for (int a = 0; a < 3; ++a) {
    int lo = 1, hi = 0;
    bool found = false;
    for (int i = 0; i < n[a]; ++i) {
      const bool ok = layer_sigma(g, a, (double)(i - 1) * stride) == 0.0 &&
                      layer_sigma(g, a, (double)(i + 1) * stride) == 0.0;
      if (ok && !found) { lo = i; found = true; }
      if (ok) hi = i;
    }
    in27.lo[a] = lo;
    in27.hi[a] = found ? hi : lo - 1;
  }
  const double w1 = g.w27[0], w2 = g.w27[1], w3 = g.w27[2];
  const double h2 = h * h;
  if (g.stencil == 1) {
    // L1 = h^-2 sum of axis second differences; L2 = L1/3 + (6h^2)^-1 sum
    // over face diagonals; L3 = (4h^2)^-1 sum over body diagonals
    in27.lw[0] = (w1 * -6.0 + w2 * (-6.0 / 3.0 - 12.0 / 6.0) + w3 * (-8.0 / 4.0)) / h2;
    in27.lw[1] = (w1 * 1.0 + w2 * (1.0 / 3.0)) / h2;
    in27.lw[2] = (w2 * (1.0 / 6.0)) / h2;
    in27.lw[3] = (w3 * (1.0 / 4.0)) / h2;
    for (int c = 0; c < 4; ++c) in27.mw[c] = g.w27[3 + c];
  } else {
    for (int c = 0; c < 4; ++c) in27.lw[c] = 0.0;
    in27.mw[0] = 1.0;
    in27.mw[1] = in27.mw[2] = in27.mw[3] = 0.0;
  }
  return in27;
}

// Layer-table arithmetic shared by every path that builds tables (one
// device kernel, so the tables of every entry point are bitwise identical).
// sigma at fine coordinate tf of an axis with nf fine nodes.
__device__ __forceinline__ double table_sigma(double smax, int npml, int nf, double tf) {
  if (npml == 0) return 0.0;
  const double d = fmax(0.0, fmax(npml - tf, tf - (nf - 1 - npml)));
  return smax * (d / npml) * (d / npml);
}
// 1 / (h^2 s(t) s(t + dt)) with s(t) = 1 + i sigma(t) / omega, level
// coordinates t (fine coordinate t * stride).
__device__ __forceinline__ cx<double> table_coef(double h, double smax, int npml, int nf, int stride,
                                                 double omega, double t, double dt) {
  const cx<double> s0 = mk(1.0, table_sigma(smax, npml, nf, t * stride) / omega);
  const cx<double> s1 = mk(1.0, table_sigma(smax, npml, nf, (t + dt) * stride) / omega);
  const cx<double> z = (h * h) * (s0 * s1);
  const double den = z.re * z.re + z.im * z.im;
  return mk(z.re / den, -z.im / den);
}

// Layer tables of one operator on one level, [dir][axis][alpha, beta,
// delta][n_axis] in complex<double> (tabd) and complex<float> (tabf).  Per
// axis, cp(i) = 1/(h^2 s(i) s(i+1/2)) and cm(i) = 1/(h^2 s(i) s(i-1/2)).
// Forward row: alpha = cp, beta = cm, delta = 0; a coupling to a node outside
// the grid (zero Dirichlet value) is folded into delta and the coupling itself
// set to zero, so a kernel may read any finite value in place of the missing
// neighbour.  Adjoint row: the conjugates of the transposed couplings
// (already zero towards nodes outside the grid).  One thread per (axis, node).
__global__ void k_layer_tables(cx<double>* tabd, cx<float>* tabf, int n0, int n1, int n2, int f0, int f1, int f2,
                               double h, double smax, int npml, int stride, double omega) {
  const int n[3] = {n0, n1, n2}, nfine[3] = {f0, f1, f2};
  const int tdir = 3 * (n0 + n1 + n2);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n0 + n1 + n2; t += gridDim.x * blockDim.x) {
    const int a = t < n0 ? 0 : t < n0 + n1 ? 1 : 2;
    const int i = t - (a > 0 ? n0 : 0) - (a > 1 ? n1 : 0);
    const int na = n[a], nf = nfine[a];
    const int pre = a == 0 ? 0 : a == 1 ? 3 * n0 : 3 * (n0 + n1);
    auto cp = [&](int k) { return table_coef(h, smax, npml, nf, stride, omega, (double)k, 0.5); };
    auto cm = [&](int k) { return table_coef(h, smax, npml, nf, stride, omega, (double)k, -0.5); };
    const cx<double> z = czero<double>();
    if (na == 1) {  // the absent axis of a 2D grid: no coupling, no diagonal term
      for (int r = 0; r < 6; ++r) {
        const int64_t o = (r >= 3 ? tdir : 0) + pre + (r % 3) * na + i;
        tabd[o] = z;
        tabf[o] = cast<float>(z);
      }
      continue;
    }
    const cx<double> cpi = cp(i), cmi = cm(i);
    const cx<double> al = (i + 1 < na) ? cpi : z;
    const cx<double> be = (i > 0) ? cmi : z;
    const cx<double> de = (i + 1 < na ? z : mk(-cpi.re, -cpi.im)) + (i > 0 ? z : mk(-cmi.re, -cmi.im));
    const cx<double> cmn = cm(i + 1), cpp = cp(i - 1);
    const cx<double> aal = (i + 1 < na) ? mk(cmn.re, -cmn.im) : z;
    const cx<double> abe = (i > 0) ? mk(cpp.re, -cpp.im) : z;
    const cx<double> sum = cpi + cmi;
    const cx<double> ade = mk(-sum.re, sum.im) + aal + abe;
    const cx<double> v[6] = {al, be, de, aal, abe, ade};
    for (int r = 0; r < 6; ++r) {
      const int64_t o = (r >= 3 ? tdir : 0) + pre + (r % 3) * na + i;
      tabd[o] = v[r];
      tabf[o] = cast<float>(v[r]);
    }
  }
}

// sigma_max of the layer profile (fine-grid units)
inline double layer_smax(const GridSpec& g) {
  if (g.npml == 0) return 0.0;
  return 3.0 * g.vref * std::log(1.0 / g.R) / (2.0 * g.npml * g.h);
}

inline void launch_layer_tables(const GridSpec& g, double omega, const int n[3], double h, int stride,
                                cx<double>* tabd, cx<float>* tabf, hipStream_t st) {
  const int nt = n[0] + n[1] + n[2];
  hipLaunchKernelGGL(k_layer_tables, dim3(ceil_div(nt, 256)), dim3(256), 0, st, tabd, tabf, n[0], n[1], n[2],
                     g.n[0], g.n[1], g.n[2], h, layer_smax(g), g.npml, stride, omega);
  HELM_HIP_CHECK(hipGetLastError());
}

inline std::unique_ptr<OpTables> build_tables(const GridSpec& g, double omega, const int n[3], double h,
                                              int stride, hipStream_t st) {
  std::unique_ptr<OpTables> T(new OpTables());
  for (int a = 0; a < 3; ++a) T->n[a] = n[a];
  T->tdir = 3 * (n[0] + n[1] + n[2]);
  T->tpre[0] = 0;
  T->tpre[1] = 3 * n[0];
  T->tpre[2] = 3 * (n[0] + n[1]);
  T->tabd.ensure(2 * (size_t)T->tdir * sizeof(cx<double>));
  T->tabf.ensure(2 * (size_t)T->tdir * sizeof(cx<float>));
  launch_layer_tables(g, omega, n, h, stride, T->tabd.as<cx<double>>(), T->tabf.as<cx<float>>(), st);
  T->in27 = interior27_desc(g, n, h, stride);
  return T;
}

// What a stencil launch needs of a level: device descriptors and maps, and
// the launch shape.
struct LevelView {
  const Seg* segs;
  const int* smap;
  const int* slocal;
  const int* tmap;
  int nsblk, ntblk;
  int stencil;  // 0 7-point, 1 27-point
  int dir;      // 0 H, 1 H^H (one direction per level)
  bool pair;
  int stage27;
};

// All segments of one level with their workgroup maps.
struct LevelSet {
  int stencil = 0;
  std::vector<Seg> host;
  DevBuf segs, smap, slocal, vmap, tmap, own;
  int nsblk = 0, nvblk = 0, ntblk = 0;
  int sblk_bound = 1;  // stencil workgroups at the smallest x chunk
  int xchunk = 0;      // current x chunk of the stencil tiles
  int group = 1;       // segments per tile group (1: segment-major; see layout_stencil)
  bool pair = false;   // every segment uses pair stencil tiles
  int stage27 = 0;     // LDS bytes per workgroup of the staged 27-point pass (0: register path)
  int64_t total = 0;  // vector length (sum of N)
  std::vector<std::unique_ptr<DevBuf>> models;  // owned coarse models
  const Seg* d() const { return segs.as<const Seg>(); }
  LevelView view() const {
    return LevelView{d(), smap.as<const int>(), slocal.as<const int>(), tmap.as<const int>(), nsblk, ntblk,
                     stencil, host.empty() ? 0 : host[0].dir, pair, stage27};
  }
};

constexpr int kMinXchunk = 4;  // smallest x chunk of a stencil tile

// LDS bytes per workgroup of the staged 27-point pair pass: two plane tiles
// of (512 + 2 pz + 4) complex64 and (up to 4 more) float values plus 16
// zero bytes each, for the widest z pitch of the level; 0 (register path)
// when that exceeds 40 KiB (four workgroups per CU must still fit) or with
// HELM_STAGE27=0.
inline int stage27_bytes_pz(int pzm) {
  if (const char* e = std::getenv("HELM_STAGE27"))
    if (e[0] == '0') return 0;
  const int64_t tl = 512 + 2 * (int64_t)pzm + 4;
  const int64_t buf = ((tl * 8 + (tl + 4) * 4 + 15) / 16) * 16 + 16;
  return 2 * buf <= 40 * 1024 ? (int)(2 * buf) : 0;
}
inline int stage27_bytes(const std::vector<Seg>& segs) {
  int pzm = 0;
  for (const Seg& S : segs) pzm = std::max(pzm, S.pz);
  return stage27_bytes_pz(pzm);
}

// x-chunk (planes per stencil workgroup) for a level: about `target`
// workgroups over the level (a few per wave slot of the chip), at least 4
// planes per workgroup.  The HELM_XCHUNK / HELM_STENCIL_WG environment
// variables override the chunk / the target (tile experiments).
// plane_blocks: workgroups of one x plane summed over the segments; nxmax:
// the longest x extent.
inline int choose_xchunk_for(int64_t plane_blocks, int nxmax, bool pair) {
  if (const char* e = std::getenv("HELM_XCHUNK")) {
    const int v = std::atoi(e);
    if (v >= kMinXchunk) return v;
  }
  // measured on 128^3 and 65x65x66 with 16 right-hand sides: pair tiles
  // prefer longer marches (2048 workgroups), one-point tiles 8192
  int64_t target = pair ? 2048 : 8192;
  if (const char* e = std::getenv("HELM_STENCIL_WG")) {
    const int v = std::atoi(e);
    if (v >= 1) target = v;
  }
  nxmax = std::max(nxmax, 1);
  const int64_t nxc = std::max<int64_t>(1, (target + plane_blocks - 1) / std::max<int64_t>(plane_blocks, 1));
  int xchunk = (int)((nxmax + nxc - 1) / nxc);
  return std::max(kMinXchunk, std::min(xchunk, nxmax));
}
inline int choose_xchunk(const std::vector<Seg>& segs) {
  int64_t plane = 0;
  int nxmax = 1;
  for (const Seg& s : segs) {
    plane += s.plane_blocks;
    nxmax = std::max(nxmax, s.n[0]);
  }
  return choose_xchunk_for(plane, nxmax, !segs.empty() && segs[0].pair);
}

// Largest number of vector-kernel workgroups per segment (grid-stride over
// the segment).  HELM_VEC_WG overrides it (tile experiments).
inline int vector_blocks_cap() {
  if (const char* e = std::getenv("HELM_VEC_WG")) {
    const int v = std::atoi(e);
    if (v >= 1 && v <= DOT_BLOCKS_MAX) return v;
  }
  return DOT_BLOCKS;
}

// The operator hierarchy of a list of problems: tables, segments, maps,
// coarse models.
class Hierarchy {
 public:
  // model_bytes: size of one model value (4 for the complex64 path, 8 for complex128)
  // pad_fine: the fine level uses the even z pitch too (the caller then
  // passes right-hand sides and fields in that layout, and the fine models
  // are copied into it by refresh_fine_models).
  Hierarchy(const std::vector<ProblemSpec>& probs, int nlev, size_t model_bytes, hipStream_t st,
            bool pad_fine = false)
      : nlev_(nlev), st_(st), model_bytes_(model_bytes) {
    const int ns = (int)probs.size();
    HELM_REQUIRE(ns >= 1, "no problems");
    stencil_ = probs[0].g.stencil;
    for (const auto& p : probs) HELM_REQUIRE(p.g.stencil == stencil_, "a batch must use one stencil type");
    pair_path_ = uses_pairs(stencil_, model_bytes_);
    pad_fine_ = pad_fine && pair_path_;
    lev_.resize(nlev);
    // segment -> table index per level, deduplicated by (grid, omega)
    std::vector<int> tab_of(ns);
    std::map<std::string, int> tkey;
    std::vector<const ProblemSpec*> tprob;
    for (int s = 0; s < ns; ++s) {
      std::string key((const char*)&probs[s].g, sizeof(GridSpec));
      key.append((const char*)&probs[s].omega, sizeof(double));
      auto it = tkey.find(key);
      if (it == tkey.end()) {
        tab_of[s] = (int)tprob.size();
        tkey[key] = tab_of[s];
        tprob.push_back(&probs[s]);
      } else {
        tab_of[s] = it->second;
      }
    }
    // coarse model owners: one per distinct (model pointer, grid)
    std::vector<int> mown(ns, -1);
    {
      std::map<std::string, int> mkey;
      for (int s = 0; s < ns; ++s) {
        std::string key((const char*)&probs[s].m, sizeof(void*));
        key.append((const char*)&probs[s].g, sizeof(GridSpec));
        auto it = mkey.find(key);
        if (it == mkey.end()) { mkey[key] = s; mown[s] = s; }
        else mown[s] = it->second;
      }
    }
    for (int l = 0; l < nlev; ++l) {
      lev_[l].reset(new LevelSet());
      LevelSet& L = *lev_[l];
      L.stencil = stencil_;
      L.host.resize(ns);
      // tables of this level
      std::vector<OpTables*> tl(tprob.size());
      for (size_t t = 0; t < tprob.size(); ++t) {
        int n[3];
        coarse_dims(tprob[t]->g.n, l, n);
        tables_.push_back(build_tables(tprob[t]->g, tprob[t]->omega, n, tprob[t]->g.h * (1 << l), 1 << l, st));
        tl[t] = tables_.back().get();
      }
      int64_t off = 0;
      bool pair = pair_path_;
      for (int s = 0; s < ns; ++s) {
        Seg& S = L.host[s];
        std::memset(&S, 0, sizeof(Seg));
        coarse_dims(probs[s].g.n, l, S.n);
        S.dir = probs[s].dir;
        S.pz = z_pitch(S.n[2], l, pair_path_, pad_fine_);
        S.N = (int64_t)S.n[0] * S.n[1] * S.pz;
        S.off = off;
        off += S.N;
        pair = pair && (S.pz % 2 == 0) && (int64_t)S.n[1] * S.pz < ((int64_t)1 << 28);  // 32-bit plane offsets
        S.w2 = probs[s].omega * probs[s].omega;
        const OpTables& T = *tl[tab_of[s]];
        S.tabf = T.tabf.p;
        S.tabd = T.tabd.p;
        for (int a = 0; a < 3; ++a) S.tpre[a] = T.tpre[a];
        S.tdir = T.tdir;
        S.in27 = T.in27;
      }
      for (int s = 0; s < ns; ++s) {
        Seg& S = L.host[s];
        S.pair = pair ? 1 : 0;
        S.plane_blocks = (int)ceil_div((int64_t)S.n[1] * S.pz, pair ? 512 : 256);
      }
      L.pair = pair;
      L.stage27 = pair && stencil_ == 1 ? stage27_bytes(L.host) : 0;
      L.total = off;
      // models: level 0 borrows the caller's; coarse levels own one per distinct model
      std::vector<int> own(ns, 0);
      for (int s = 0; s < ns; ++s) {
        if (l == 0 && L.host[s].pz == L.host[s].n[2]) {
          L.host[s].m = probs[s].m;
        } else if (l == 0) {
          // fine model in the padded layout, copied from the caller's
          if (mown[s] == s) {
            L.models.emplace_back(new DevBuf());
            L.models.back()->ensure((size_t)L.host[s].N * model_bytes_);
            HELM_HIP_CHECK(hipMemsetAsync(L.models.back()->p, 0, (size_t)L.host[s].N * model_bytes_, st));
            L.host[s].m = L.models.back()->p;
            fine_copies_.push_back({s, probs[s].m});
          } else {
            L.host[s].m = L.host[mown[s]].m;
          }
        } else if (mown[s] == s) {
          L.models.emplace_back(new DevBuf());
          L.models.back()->ensure((size_t)L.host[s].N * model_bytes_);
          L.host[s].m = L.models.back()->p;
          own[s] = 1;
        } else {
          L.host[s].m = L.host[mown[s]].m;
        }
      }
      // workgroup ranges of the vector and point-wise kernels
      const int vcap = vector_blocks_cap();
      int vb = 0, tb = 0;
      for (int s = 0; s < ns; ++s) {
        Seg& S = L.host[s];
        S.vblk0 = vb;
        S.vnblk = (int)std::min<int64_t>(vcap, ceil_div(S.N, 256));
        vb += S.vnblk;
        S.tblk0 = tb;
        S.tnblk = (int)ceil_div(S.N, 256);
        tb += S.tnblk;
      }
      L.nvblk = vb;
      L.ntblk = tb;
      std::vector<int> vmap(std::max(vb, 1)), tmap(std::max(tb, 1));
      for (int s = 0; s < ns; ++s) {
        const Seg& S = L.host[s];
        for (int b = 0; b < S.vnblk; ++b) vmap[S.vblk0 + b] = s;
        for (int b = 0; b < S.tnblk; ++b) tmap[S.tblk0 + b] = s;
      }
      upload(L.vmap, vmap);
      upload(L.tmap, tmap);
      upload(L.own, own);
      L.segs.ensure(ns * sizeof(Seg));
      // stencil tiles (the x chunk may be re-chosen by the tile tuner)
      int64_t bound = 0;
      for (const Seg& S : L.host) bound += (int64_t)S.plane_blocks * ceil_div(S.n[0], kMinXchunk);
      L.sblk_bound = (int)std::max<int64_t>(bound, 1);
      L.smap.ensure(L.sblk_bound * sizeof(int));
      L.slocal.ensure(L.sblk_bound * sizeof(int));
      layout_stencil(l, choose_xchunk(L.host));
    }
  }

  // Whether level l's stencil tiles may interleave the segments: several
  // segments of one grid and one model, on a tiled stencil path.
  bool can_interleave(int l) const {
    const LevelSet& L = *lev_[l];
    const int ns = (int)L.host.size();
    bool ok = (stencil_ == 0 || L.pair) && ns > 1;
    for (int s = 1; s < ns && ok; ++s)
      ok = L.host[s].m == L.host[0].m && L.host[s].n[0] == L.host[0].n[0] &&
           L.host[s].n[1] == L.host[0].n[1] && L.host[s].n[2] == L.host[0].n[2];
    return ok;
  }

  // Stencil workgroup layout of level l for x chunk `xchunk`: segment ranges,
  // workgroup -> (segment, tile) maps, uploaded.  When every segment of a
  // level has the same geometry and model (the sources of one frequency), the
  // segments may be taken in groups of `group`: inside a group the segments
  // of one tile get consecutive workgroup ids (segment fastest), so they run
  // together on one XCD and read that tile of the model once into its L2;
  // the groups follow one another.  group 1 is segment-major order (one
  // right-hand side's neighbouring tiles together, the model read once per
  // XCD and segment), group >= the segment count interleaves all of them.
  // group: -1 chooses (the size rule below, or HELM_INTERLEAVE /
  // HELM_TILE_GROUP); segment-major wherever the segments do not share grid
  // and model.
  void layout_stencil(int l, int xchunk, int group = -1) {
    LevelSet& L = *lev_[l];
    const int ns = (int)L.host.size();
    xchunk = std::max(xchunk, kMinXchunk);
    int sb = 0;
    for (int s = 0; s < ns; ++s) {
      Seg& S = L.host[s];
      S.xchunk = xchunk;
      S.nxc = (S.n[0] + xchunk - 1) / xchunk;
      S.sblk0 = sb;
      S.snblk = (stencil_ == 0 || L.pair) ? S.plane_blocks * S.nxc : 0;
      sb += S.snblk;
    }
    HELM_REQUIRE(sb <= L.sblk_bound, "internal: stencil workgroup bound exceeded");
    L.nsblk = sb;
    L.xchunk = xchunk;
    std::vector<int> smap(std::max(sb, 1)), slocal(std::max(sb, 1));
    // (measured: on small levels, where the model tile is most of a tile's
    // distinct data, groups of 4 pay -- the 128^3 16-source solve is 2 %
    // faster with its 65^3 level in groups of 4 than with all 16 interleaved
    // (groups of 2 / 8: 1.7 / 1.4 %); on 128^3 and larger, keeping one
    // right-hand side's neighbouring tiles on one XCD is worth more)
    if (group < 0) {
      group = L.host[0].N <= ((int64_t)1 << 20) ? std::min(ns, 4) : 1;
      if (const char* il = std::getenv("HELM_INTERLEAVE"))  // 1 / 0: all / none (tile experiments)
        group = il[0] == '1' ? ns : 1;
      // segments per group, one value per level ("4" or "4,16,16"; the last
      // value holds for deeper levels) -- tile experiments
      if (const char* tg = std::getenv("HELM_TILE_GROUP")) {
        int v = 0;
        const char* c = tg;
        for (int k = 0; k <= l && *c; ++k) {
          v = std::atoi(c);
          const char* comma = std::strchr(c, ',');
          if (!comma) break;
          c = comma + 1;
        }
        if (v >= 1) group = v;
      }
    }
    group = can_interleave(l) ? std::max(1, std::min(group, ns)) : 1;
    L.group = group;
    for (int s = 0; s < ns; ++s) {
      const Seg& S = L.host[s];
      // group g = s / group holds segments [s0, s0 + gs), all with snblk tiles
      const int s0 = s - s % group, gs = std::min(group, ns - s0);
      for (int b = 0; b < S.snblk; ++b) {
        const int wg = group == 1 ? S.sblk0 + b : S.sblk0 - (s - s0) * S.snblk + b * gs + (s - s0);
        smap[wg] = s;
        slocal[wg] = b;
      }
    }
    HELM_HIP_CHECK(hipMemcpyAsync(L.smap.p, smap.data(), smap.size() * sizeof(int), hipMemcpyHostToDevice, st_));
    HELM_HIP_CHECK(
        hipMemcpyAsync(L.slocal.p, slocal.data(), slocal.size() * sizeof(int), hipMemcpyHostToDevice, st_));
    HELM_HIP_CHECK(hipMemcpyAsync(L.segs.p, L.host.data(), ns * sizeof(Seg), hipMemcpyHostToDevice, st_));
    HELM_HIP_CHECK(hipStreamSynchronize(st_));
  }

  // Key of level l's tile choice: stencil kind, value size and the sorted
  // list of segment shapes (independent of the order of a batch).
  std::string tile_key(int l) const {
    const LevelSet& L = *lev_[l];
    std::vector<std::string> shapes;
    for (const Seg& S : L.host)
      shapes.push_back(std::to_string(S.n[0]) + "x" + std::to_string(S.n[1]) + "x" + std::to_string(S.n[2]) +
                       "p" + std::to_string(S.pz));
    std::sort(shapes.begin(), shapes.end());
    std::string k = std::to_string(stencil_) + ":" + std::to_string(model_bytes_) + ":" + std::to_string(L.pair);
    for (const auto& x : shapes) k += "," + x;
    return k;
  }

  int nlev() const { return nlev_; }
  int nseg() const { return (int)lev_[0]->host.size(); }
  const LevelSet& level(int l) const { return *lev_[l]; }
  int stencil() const { return stencil_; }

  // Set the direction (H or H^H) of every segment on every level.
  void set_dir(int dir) {
    for (auto& L : lev_) {
      bool changed = false;
      for (auto& S : L->host)
        if (S.dir != dir) { S.dir = dir; changed = true; }
      if (changed) {
        HELM_HIP_CHECK(hipMemcpyAsync(L->segs.p, L->host.data(), L->host.size() * sizeof(Seg),
                                      hipMemcpyHostToDevice, st_));
        HELM_HIP_CHECK(hipStreamSynchronize(st_));
      }
    }
  }

  // Coarse models from the (current contents of the) fine models.
  template <typename TM>
  void inject_models() {
    for (int l = 1; l < nlev_; ++l) {
      const LevelSet& F = *lev_[l - 1];
      const LevelSet& C = *lev_[l];
      hipLaunchKernelGGL((k_inject_model<TM>), dim3(C.ntblk), dim3(256), 0, st_, F.d(), C.d(),
                         C.tmap.as<const int>(), C.own.as<const int>());
    }
    HELM_HIP_CHECK(hipGetLastError());
  }

  size_t max_partials() const {
    size_t mx = 1;
    for (const auto& L : lev_) {
      mx = std::max<size_t>(mx, L->sblk_bound);
      mx = std::max<size_t>(mx, L->nvblk);
      if (stencil_ == 1) mx = std::max<size_t>(mx, L->ntblk);
    }
    return mx;
  }

  // The complex64 7-point path tiles its stencil in z-pairs (16-byte
  // accesses); its coarse levels get an even z pitch.  The fine level keeps
  // the caller's layout (pairs there need an even n2).
  static bool uses_pairs(int stencil, size_t model_bytes) { (void)stencil; return model_bytes == 4; }
  static int z_pitch(int nz, int level, bool pairs, bool pad_fine) {
    return (pairs && (level > 0 || pad_fine)) ? nz + (nz & 1) : nz;
  }
  // vector length of one problem on level l
  static int64_t level_points(const int n0[3], int l, bool pairs, bool pad_fine) {
    int n[3];
    coarse_dims(n0, l, n);
    return (int64_t)n[0] * n[1] * z_pitch(n[2], l, pairs, pad_fine);
  }
  bool pad_fine() const { return pad_fine_; }

  // Copy the callers' fine models into the padded fine layout (before every
  // solve: the caller may have changed them in place).
  void refresh_fine_models() {
    const LevelSet& L = *lev_[0];
    for (const auto& fc : fine_copies_) {
      const Seg& S = L.host[fc.first];
      HELM_HIP_CHECK(hipMemcpy2DAsync(const_cast<void*>(S.m), (size_t)S.pz * model_bytes_, fc.second,
                                      (size_t)S.n[2] * model_bytes_, (size_t)S.n[2] * model_bytes_,
                                      (size_t)S.n[0] * S.n[1], hipMemcpyDeviceToDevice, st_));
    }
  }

  static void coarse_dims(const int n0[3], int l, int n[3]) {
    for (int a = 0; a < 3; ++a) {
      n[a] = n0[a];
      for (int k = 0; k < l; ++k) n[a] = n[a] / 2 + 1;
    }
  }

 private:
  template <typename V>
  void upload(DevBuf& buf, const std::vector<V>& v) {
    buf.ensure(v.size() * sizeof(V));
    HELM_HIP_CHECK(hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, st_));
  }

  int nlev_;
  hipStream_t st_;
  size_t model_bytes_;
  int stencil_ = 0;
  bool pair_path_ = false;
  bool pad_fine_ = false;
  std::vector<std::pair<int, const void*>> fine_copies_;  // (segment, caller's model)
  std::vector<std::unique_ptr<LevelSet>> lev_;
  std::vector<std::unique_ptr<OpTables>> tables_;
};

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// out = [s_b b -] s_x H x over all segments of level L.  The complex64
// 7-point operator runs pair tiles when the level and the buffers allow it.
// Returns the partial-sum range a NORM launch wrote (PR_STENCIL: stencil
// tiles; PR_POINT: point-wise workgroups).
template <typename TC, typename TX, typename TM, typename TB, typename TO, bool RESID, bool NORM>
int launch_h(const LevelView& L, const cx<TX>* x, const double* xs, const cx<TB>* b, const double* bs,
             cx<TO>* out, double* part, const int* active, hipStream_t st) {
  constexpr bool all_f32 = std::is_same<TC, float>::value && std::is_same<TX, float>::value &&
                           std::is_same<TM, float>::value && std::is_same<TB, float>::value &&
                           std::is_same<TO, float>::value;
  const bool pair_ok = all_f32 && L.pair && aligned16(x) && aligned16(out) && (!RESID || aligned16(b));
  if (L.stencil == 1 && pair_ok) {
    if (L.dir)
      hipLaunchKernelGGL((k_h27p<true, RESID, NORM>), dim3(L.nsblk), dim3(256), L.stage27, st, L.segs, L.smap,
                         L.slocal, reinterpret_cast<const c32*>(x), xs, reinterpret_cast<const c32*>(b), bs,
                         reinterpret_cast<c32*>(out), part, active, VecPtrs{}, (const double*)nullptr,
                         L.stage27 > 0 ? 1 : 0);
    else
      hipLaunchKernelGGL((k_h27p<false, RESID, NORM>), dim3(L.nsblk), dim3(256), L.stage27, st, L.segs, L.smap,
                         L.slocal, reinterpret_cast<const c32*>(x), xs, reinterpret_cast<const c32*>(b), bs,
                         reinterpret_cast<c32*>(out), part, active, VecPtrs{}, (const double*)nullptr,
                         L.stage27 > 0 ? 1 : 0);
    return PR_STENCIL;
  } else if (L.stencil == 1) {
    hipLaunchKernelGGL((k_h27<TC, TX, TM, TB, TO, RESID, NORM>), dim3(L.ntblk), dim3(256), 0, st, L.segs, L.tmap, x,
                       xs, b, bs, out, part, active);
    return PR_POINT;
  } else if (pair_ok) {
    hipLaunchKernelGGL((k_h7p<RESID, NORM, 0, false>), dim3(L.nsblk), dim3(256), 0, st, L.segs, L.smap, L.slocal,
                       reinterpret_cast<const c32*>(x), xs, reinterpret_cast<const c32*>(b), bs,
                       reinterpret_cast<c32*>(out), part, active, VecPtrs{}, (const double*)nullptr);
    return PR_STENCIL;
  } else {
    hipLaunchKernelGGL((k_h7<TC, TX, TM, TB, TO, RESID, NORM>), dim3(L.nsblk), dim3(256), 0, st, L.segs, L.smap,
                       L.slocal, x, xs, b, bs, out, part, active);
  }
  return PR_STENCIL;
}

template <typename TC, typename TX, typename TM, typename TB, typename TO, bool RESID, bool NORM>
int launch_h(const LevelSet& L, const cx<TX>* x, const double* xs, const cx<TB>* b, const double* bs,
             cx<TO>* out, double* part, const int* active, hipStream_t st) {
  return launch_h<TC, TX, TM, TB, TO, RESID, NORM>(L.view(), x, xs, b, bs, out, part, active, st);
}

// Tile choice of one level: x chunk of the stencil march and segment group.
struct TileChoice {
  int xchunk = 0;
  int group = 1;
};

// On-disk record of tile choices, so that a problem set gets the same tiles
// (hence bitwise the same results) in every process on the same kind of GPU:
// one line "key<TAB>xchunk<TAB>group" per choice, in the file named by
// HELM_TUNE_CACHE (set but empty: no file), else
// $XDG_CACHE_HOME/helm/tiles.tsv or $HOME/.cache/helm/tiles.tsv.  Keys carry
// the record format and the device (architecture, compute units).  A file
// that cannot be read or written is ignored: choices then live for the
// process only.
inline std::string tune_cache_path() {
  if (const char* e = std::getenv("HELM_TUNE_CACHE")) return std::string(e);
  std::string dir;
  if (const char* x = std::getenv("XDG_CACHE_HOME")) dir = x;
  else if (const char* h = std::getenv("HOME")) dir = std::string(h) + "/.cache";
  if (dir.empty()) return std::string();
  return dir + "/helm/tiles.tsv";
}

inline void tune_cache_load(const std::string& path, std::map<std::string, TileChoice>& cache) {
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char line[4096];
  while (std::fgets(line, sizeof(line), f)) {
    char* t1 = std::strchr(line, '\t');
    if (!t1) continue;
    *t1 = '\0';
    TileChoice c;
    if (std::sscanf(t1 + 1, "%d\t%d", &c.xchunk, &c.group) == 2 && c.xchunk >= kMinXchunk && c.group >= 1)
      cache[line] = c;
  }
  std::fclose(f);
}

inline void tune_cache_store(const std::string& path, const std::string& key, const TileChoice& c) {
  if (path.empty()) return;
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0) {  // the directory and its parent, best effort
    const std::string dir = path.substr(0, slash);
    const size_t up = dir.rfind('/');
    if (up != std::string::npos && up > 0) (void)mkdir(dir.substr(0, up).c_str(), 0755);
    (void)mkdir(dir.c_str(), 0755);
  }
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%s\t%d\t%d\n", key.c_str(), c.xchunk, c.group);
  std::fclose(f);
}

inline std::string device_tag() {
  int dev = 0;
  HELM_HIP_CHECK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HELM_HIP_CHECK(hipGetDeviceProperties(&prop, dev));
  return std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount);
}

// Tile tuner: time a stencil launch for a few x chunks, each with the
// segment-major and, where the segments share grid and model, the
// segment-fastest order, and keep the fastest.  The choice is cached per tile
// key for the process and on disk (see above), so one problem set, in any
// order, always gets the same tiles and hence the same results.  Fixed tiles
// with HELM_XCHUNK / HELM_STENCIL_WG; off with HELM_AUTOTUNE=0 (heuristic
// tiles).  `run(L)` launches the kernel to time on level L (what the caller
// runs most there); `kind` names it in the cache key.
template <typename Run>
void tune_tiles(Hierarchy& H, const std::string& kind, Run run, hipStream_t st) {
  static std::mutex mu;
  static std::map<std::string, TileChoice> cache;
  static std::string loaded_from = "\x01";  // path the cache was last read from
  if (std::getenv("HELM_XCHUNK") || std::getenv("HELM_STENCIL_WG")) return;
  if (const char* e = std::getenv("HELM_AUTOTUNE"))
    if (e[0] == '0') return;
  std::lock_guard<std::mutex> guard(mu);
  const std::string path = tune_cache_path();
  if (path != loaded_from) {
    tune_cache_load(path, cache);
    loaded_from = path;
  }
  const std::string prefix = "tiles3|" + device_tag() + "|" + kind + "|";
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HELM_HIP_CHECK(hipEventCreate(&e0));
  HELM_HIP_CHECK(hipEventCreate(&e1));
  try {
    for (int l = 0; l < H.nlev(); ++l) {
      if (H.stencil() != 0 && !H.level(l).pair) continue;  // point-wise 27-point kernel: no tiles
      const std::string key = prefix + H.tile_key(l);
      auto it = cache.find(key);
      if (it != cache.end()) {
        if (it->second.xchunk != H.level(l).xchunk || it->second.group != H.level(l).group)
          H.layout_stencil(l, it->second.xchunk, it->second.group);
        continue;
      }
      int nxm = 0;
      for (const Seg& S : H.level(l).host) nxm = std::max(nxm, S.n[0]);
      const int reps = H.level(l).total < (int64_t)1 << 24 ? 10 : 3;  // short launches: more samples
      std::vector<int> cand = {H.level(l).xchunk, nxm, (nxm + 1) / 2, (nxm + 3) / 4, 32, 16, 8, kMinXchunk};
      std::sort(cand.begin(), cand.end());
      cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
      // segment orders: the heuristic's first, then segment-major, groups of
      // 2 and 4, all segments (where the segments share grid and model)
      const int ns = (int)H.level(l).host.size();
      std::vector<int> orders = {H.level(l).group};
      if (H.can_interleave(l))
        for (int gr : {1, 2, 4, ns})
          if (gr <= ns && std::find(orders.begin(), orders.end(), gr) == orders.end()) orders.push_back(gr);
      TileChoice best{H.level(l).xchunk, H.level(l).group};
      float best_ms = 1e30f;
      std::vector<std::pair<TileChoice, float>> timed;
      const bool verbose = std::getenv("HELM_VERBOSE") != nullptr;
      std::string trace;
      for (int order : orders) {
        for (int c : cand) {
          if (c < kMinXchunk || c > std::max(nxm, kMinXchunk)) continue;
          H.layout_stencil(l, c, order);
          const LevelSet& L = H.level(l);
          run(L);  // warm
          HELM_HIP_CHECK(hipEventRecord(e0, st));
          for (int r = 0; r < reps; ++r) run(L);
          HELM_HIP_CHECK(hipEventRecord(e1, st));
          HELM_HIP_CHECK(hipEventSynchronize(e1));
          float ms = 0.f;
          HELM_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
          if (verbose)
            trace += " " + std::to_string(c) + "g" + std::to_string(L.group) + ":" + std::to_string(ms / reps * 1e3f) +
                     "us";
          timed.push_back({TileChoice{c, L.group}, ms});
          if (ms < best_ms) {
            best_ms = ms;
            best = TileChoice{c, L.group};
          }
        }
      }
      // within 1.5 % of the fastest (about the run-to-run spread of these
      // timings) take the largest segment group, the one with the fewest
      // model copies in the L2 caches, so that the choice does not flip with
      // noise between runs and GPUs
      int gmax = best.group;
      for (const auto& t : timed)
        if (t.second <= 1.015f * best_ms) gmax = std::max(gmax, t.first.group);
      float gbest = 1e30f;
      for (const auto& t : timed)
        if (t.first.group == gmax && t.second <= 1.015f * best_ms && t.second < gbest) {
          gbest = t.second;
          best = t.first;
        }
      if (verbose)
        fprintf(stderr, "helm tiles %s level %d -> x chunk %d, segment group %d (%s)\n", kind.c_str(), l, best.xchunk,
                best.group, trace.c_str());
      H.layout_stencil(l, best.xchunk, best.group);
      cache[key] = best;
      tune_cache_store(path, key, best);
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// Tiles for the plain operator, timed on the caller's a -> b (each at least
// as long as the level's vectors).
template <typename T>
void tune_tiles_apply(Hierarchy& H, const cx<T>* a, cx<T>* b, hipStream_t st) {
  tune_tiles(H, "apply", [&](const LevelSet& L) {
    launch_h<T, T, T, T, T, false, false>(L, a, nullptr, (const cx<T>*)nullptr, nullptr, b, nullptr, nullptr, st);
  }, st);
}

// out = s_x H x together with the partial inner products of out with
// D[0..nmem) and, when self, with x itself (last); complex64 pair tiles only.
// Returns false (nothing launched) when the level or the buffers do not allow
// the fused pass; the caller then runs the separate inner-product kernel.
template <int NMEM, bool SELF>
void launch_h_dots_n(const LevelSet& L, const c32* x, const double* xs, const double* npart, c32* out,
                     const VecPtrs& D, double* part, const int* active, hipStream_t st) {
  const dim3 grid(L.nsblk), block(256);
  const int* sm = L.smap.as<const int>();
  const int* sl = L.slocal.as<const int>();
  if (L.stencil == 0)
    hipLaunchKernelGGL((k_h7p<false, false, NMEM, SELF>), grid, block, 0, st, L.d(), sm, sl, x, xs,
                       (const c32*)nullptr, (const double*)nullptr, out, part, active, D, npart);
  else if (L.host[0].dir)
    hipLaunchKernelGGL((k_h27p<true, false, false, NMEM, SELF>), grid, block, L.stage27, st, L.d(), sm, sl, x, xs,
                       (const c32*)nullptr, (const double*)nullptr, out, part, active, D, npart,
                       L.stage27 > 0 ? 1 : 0);
  else
    hipLaunchKernelGGL((k_h27p<false, false, false, NMEM, SELF>), grid, block, L.stage27, st, L.d(), sm, sl, x, xs,
                       (const c32*)nullptr, (const double*)nullptr, out, part, active, D, npart,
                       L.stage27 > 0 ? 1 : 0);
}

// whether launch_h_dots can run on this level with nmem memory vectors
inline bool can_fuse_dots(const LevelSet& L, int nmem, bool self) {
  return L.pair && nmem >= 0 && nmem <= 5 && nmem + (self ? 1 : 0) >= 1;
}

// npart (optional): the input scale is 1/||x|| from these vector-range
// partial norms instead of xs.
inline bool launch_h_dots(const LevelSet& L, const c32* x, const double* xs, const double* npart, c32* out,
                          const c32* const* D, int nmem, bool self, double* part, const int* active,
                          hipStream_t st) {
  if (!can_fuse_dots(L, nmem, self) || !aligned16(x) || !aligned16(out)) return false;
  VecPtrs v{};
  for (int t = 0; t < nmem; ++t) {
    if (!aligned16(D[t])) return false;
    v.v[t] = D[t];
  }
#define HELM_HD(NM)                                                                                   \
  case NM:                                                                                           \
    if (self) launch_h_dots_n<NM, true>(L, x, xs, npart, out, v, part, active, st);                 \
    else launch_h_dots_n<NM, false>(L, x, xs, npart, out, v, part, active, st);                     \
    return true;
  switch (nmem) {
    HELM_HD(1)
    HELM_HD(2)
    HELM_HD(3)
    HELM_HD(4)
    HELM_HD(5)
    case 0:
      launch_h_dots_n<0, true>(L, x, xs, npart, out, v, part, active, st);
      return true;
  }
#undef HELM_HD
  return false;
}

}  // namespace helm
