// Host orchestration of the preconditioned Krylov solve (arXiv:1703.09268,
// ML-GMRES section) on a list of segments (problems) at once.
//
// * Outer solver: FGMRES(k) (flexible, because the preconditioner is itself
//   an iteration) to a relative residual `tol`, or plain GMRES(k).  The outer
//   iterate x and its true residual q - H x are kept in FP64 (mixed-precision
//   iterative refinement); the residual is the start vector of each cycle.
// * Preconditioner: the V-cycle of the paper's algorithm "Standard multigrid
//   V-cycle" with GMRES(ks_o cycles, ks_i steps) smoothers, residual,
//   restriction R = P^T/8, coarse solve by FGMRES(kc_o, kc_i) preconditioned
//   by the next level's V-cycle (plain GMRES(kc_o, kc_i) on the coarsest
//   grid), prolongation-and-add, post-smoothing; the V-cycle starts from 0.
// * Inner solves run fixed iteration counts (no tolerance test), so the
//   whole preconditioner is a fixed sequence of kernels with every scalar on
//   the device.  The part of an outer cycle after the convergence test (k
//   Arnoldi steps with their V-cycles, then the update of x) is therefore
//   the same kernel sequence in every cycle: it is captured once in a
//   hipGraph and replayed.  The host synchronises once per outer cycle.
// * Segments that reach the tolerance (or turn non-finite) are switched off
//   through a device mask that every kernel reads; the others continue.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <vector>

#include "common.h"
#include "krylov.hip"
#include "operator.hip"
#include "transfer.hip"

namespace helm {

struct SolveOpts {
  int method;  // 0 GMRES, 1 FGMRES + multilevel V-cycle
  int restart, max_cycles;
  double tol;
  int ks_o, ks_i, kc_o, kc_i, levels;
  int warm_start;
};

struct SolveInfo {
  int status = 0, cycles = 0, inner_its = 0;
  int64_t matvecs = 0;
  double relres = 0.0;
};

template <typename T>
struct VRef {
  const cx<T>* p;
  const double* s;  // per-segment scale (null = 1)
};

// The complex64 7-point Arnoldi steps form their inner products inside the
// stencil pass; HELM_FUSED_DOTS=0 runs the separate pass instead (A/B
// measurements).
inline bool fused_dots_enabled() {
  const char* e = std::getenv("HELM_FUSED_DOTS");
  return !(e && e[0] == '0');
}

inline bool graphs_enabled() {
  const char* e = std::getenv("HELM_GRAPH");
  return !(e && e[0] == '0');
}

template <typename T>
class Solver {
 public:
  // Krylov space of one (F)GMRES instance
  struct Space {
    int lvl = 0, k = 0;
    bool flex = false;
    cx<T>* V[KMAX + 1] = {};
    cx<T>* Z[KMAX] = {};
    const cx<T>* v0 = nullptr;  // basis vector 0 (may alias the right-hand side)
    KState ks{};
  };

  // pad_fine: fine-level vectors (q, u of solve) use the even z pitch of the
  // pair-tiled path (see Hierarchy).
  Solver(const std::vector<ProblemSpec>& probs, const SolveOpts& o, hipStream_t st, bool pad_fine = false)
      : o_(o), st_(st), nseg_((int)probs.size()) {
    nlev_ = (o.method == 1) ? o.levels : 1;
    H_.reset(new Hierarchy(probs, nlev_, sizeof(T), st, pad_fine));
    allocate();
    tune();
  }
  ~Solver() { drop_graph(); }

  const Hierarchy& hierarchy() const { return *H_; }
  // per-call options (the structural ones are fixed at construction)
  void set_call_opts(const SolveOpts& o) {
    o_.tol = o.tol;
    o_.max_cycles = o.max_cycles;
    o_.warm_start = o.warm_start;
  }
  int nseg() const { return nseg_; }
  // FP64 outer iterates of the last solve (level-0 layout); valid until the next solve
  const cx<double>* iterate() const { return X_; }

  // Solve with every segment in direction `dir` (0: H, 1: H^H).  q, u:
  // level-0 vectors (segment s at offset Seg::off).  Returns the worst status.
  int solve(int dir, const cx<T>* q, cx<T>* u, SolveInfo* info) {
    HELM_REQUIRE(dir == 0 || dir == 1, "direction must be 0 (H) or 1 (H^H)");
    const Range range(dir ? "helm solve H^H" : "helm solve H");
    const int lg = log_level();
    const char* const dname = dir ? "H^H" : "H";
    dir_ = dir;
    H_->set_dir(dir);
    H_->refresh_fine_models();
    H_->template inject_models<T>();
    const LevelSet& L = H_->level(0);
    std::vector<int> act(nseg_, 1);
    std::vector<double> qn(nseg_), beta(nseg_);
    for (int s = 0; s < nseg_; ++s) info[s] = SolveInfo();
    // ||q||
    hipLaunchKernelGGL((k_norm2<T>), dim3(L.nvblk), dim3(256), 0, st_, L.d(), L.vmap.as<const int>(), q, part_,
                       (const int*)nullptr);
    hipLaunchKernelGGL(k_seg_norm, dim3(nseg_), dim3(256), 0, st_, L.d(), (const double*)part_, (int)PR_VECTOR,
                       beta_dev_);
    HELM_HIP_CHECK(hipMemcpyAsync(qn.data(), beta_dev_, nseg_ * sizeof(double), hipMemcpyDeviceToHost, st_));
    HELM_HIP_CHECK(hipStreamSynchronize(st_));
    // outer iterate in FP64
    if (o_.warm_start)
      hipLaunchKernelGGL((k_convert<double, T>), dim3(flat_blocks(L.total)), dim3(256), 0, st_, (const cx<T>*)u,
                         X_, L.total);
    else
      hipLaunchKernelGGL((k_zero<double>), dim3(L.nvblk), dim3(256), 0, st_, L.d(), L.vmap.as<const int>(), X_,
                         (const int*)nullptr);
    std::vector<int> zero_seg(nseg_, 0);
    for (int s = 0; s < nseg_; ++s) {
      if (!(qn[s] > 0.0)) {  // zero (or non-finite) right-hand side
        act[s] = 0;
        info[s].status = std::isfinite(qn[s]) ? 0 : 2;
        info[s].relres = std::isfinite(qn[s]) ? 0.0 : qn[s];
        zero_seg[s] = std::isfinite(qn[s]) ? 1 : 0;
      }
    }
    bool any_zero = false;
    for (int s = 0; s < nseg_; ++s) any_zero |= zero_seg[s] != 0;
    if (any_zero) {  // a zero right-hand side has the zero solution
      upload_active(zero_seg);
      hipLaunchKernelGGL((k_zero<double>), dim3(L.nvblk), dim3(256), 0, st_, L.d(), L.vmap.as<const int>(), X_,
                         (const int*)active_);
    }
    upload_active(act);
    fine_mv_ = 0;
    int last_cycle = 0;
    for (int cyc = 0;; ++cyc) {
      const Range rc("helm outer cycle");
      last_cycle = cyc;
      // true residual in FP64, stored (rounded) as the first basis vector
      const int rng = launch_h<double, double, T, T, T, true, true>(L, X_, nullptr, q, nullptr, outer_.V[0],
                                                                    part_, active_, st_);
      fine_mv_++;
      hipLaunchKernelGGL(k_start_cycle, dim3(nseg_), dim3(256), 0, st_, L.d(), outer_.ks, rng,
                         (const double*)nullptr, beta_dev_, (const int*)active_);
      HELM_HIP_CHECK(hipMemcpyAsync(beta.data(), beta_dev_, nseg_ * sizeof(double), hipMemcpyDeviceToHost, st_));
      HELM_HIP_CHECK(hipStreamSynchronize(st_));
      int n_active = 0, n_seen = 0;
      double rmax = 0.0, rmin = HUGE_VAL;
      for (int s = 0; s < nseg_; ++s) {
        if (!act[s]) continue;
        const double rel = beta[s] / qn[s];
        ++n_seen;
        rmax = std::isnan(rel) ? rel : std::max(rmax, rel);
        rmin = std::min(rmin, rel);
        if (lg >= 2) std::fprintf(stderr, "helm:   rhs %d rel.res %.3e\n", s, rel);
        info[s].relres = rel;
        info[s].cycles = cyc;
        info[s].matvecs = fine_mv_;
        if (!std::isfinite(rel)) {
          act[s] = 0;
          info[s].status = 2;
        } else if (rel <= o_.tol) {
          act[s] = 0;
          info[s].status = 0;
        } else if (cyc >= o_.max_cycles) {
          act[s] = 0;
          info[s].status = 1;
        } else {
          ++n_active;
        }
      }
      if (lg >= 1)
        std::fprintf(stderr, "helm: solve %s cycle %d: %d of %d right-hand sides checked, rel.res max %.3e min %.3e, %d "
                     "continue\n", dname, cyc, n_seen, nseg_, rmax, n_seen ? rmin : 0.0, n_active);
      upload_active(act);
      if (n_active == 0) break;
      run_cycle_body();
      for (int s = 0; s < nseg_; ++s)
        if (act[s]) info[s].inner_its += outer_.k;
    }
    // result in the caller's precision
    hipLaunchKernelGGL((k_convert<T, double>), dim3(flat_blocks(L.total)), dim3(256), 0, st_,
                       (const cx<double>*)X_, u, L.total);
    HELM_HIP_CHECK(hipGetLastError());
    HELM_HIP_CHECK(hipStreamSynchronize(st_));
    int worst = 0, nst[3] = {0, 0, 0};
    for (int s = 0; s < nseg_; ++s) {
      worst = std::max(worst, info[s].status);
      nst[std::min(std::max(info[s].status, 0), 2)]++;
    }
    if (lg >= 1)
      std::fprintf(stderr, "helm: solve %s done after %d cycles: %d converged, %d not converged, %d breakdown\n",
                   dname, last_cycle, nst[0], nst[1], nst[2]);
    return worst;
  }

  // r = q - H x (dir 0) or q - H^H x (dir 1) for every segment, formed in
  // FP64 from an FP64 x (level-0 layout) and rounded to T; returns the FP64
  // norms ||r|| per segment.
  std::vector<double> residual(int dir, const cx<double>* x, const cx<T>* q, cx<T>* r) {
    HELM_REQUIRE(dir == 0 || dir == 1, "direction must be 0 (H) or 1 (H^H)");
    dir_ = dir;
    H_->set_dir(dir);
    const LevelSet& L = H_->level(0);
    const int rng = launch_h<double, double, T, T, T, true, true>(L, x, nullptr, q, nullptr, r, part_,
                                                                  (const int*)nullptr, st_);
    hipLaunchKernelGGL(k_seg_norm, dim3(nseg_), dim3(256), 0, st_, L.d(), (const double*)part_, rng, beta_dev_);
    HELM_HIP_CHECK(hipGetLastError());
    std::vector<double> out(nseg_);
    HELM_HIP_CHECK(hipMemcpyAsync(out.data(), beta_dev_, nseg_ * sizeof(double), hipMemcpyDeviceToHost, st_));
    HELM_HIP_CHECK(hipStreamSynchronize(st_));
    return out;
  }

  static size_t workspace_bytes(const std::vector<int64_t>& Nlev, const SolveOpts& o) {
    // Nlev[l] = total points of all segments on level l
    size_t total = 0;
    const int nlev = (int)Nlev.size();
    for (int l = 0; l < nlev; ++l) {
      total += (size_t)slots_at(o, l, nlev) * vec_bytes(Nlev[l]);
      if (l > 0) total += (size_t)Nlev[l] * sizeof(T);
    }
    total += round256((size_t)Nlev[0] * sizeof(cx<double>));  // FP64 outer iterate
    return total;
  }

  // every workspace vector starts on a 256-byte boundary (16-byte pair
  // accesses need at least 16)
  static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }
  static size_t vec_bytes(int64_t len) { return round256((size_t)len * sizeof(cx<T>)); }

 private:
  static unsigned flat_blocks(int64_t n) { return std::min<unsigned>(65536, ceil_div(n, 256)); }

  static int slots_at(const SolveOpts& o, int l, int nlev) {
    int s = 0;
    if (l == 0) {
      s += (o.restart + 1) + (o.method == 1 ? o.restart : 0);  // outer V, Z
      if (nlev > 1) s += (o.ks_i + 1) + 1;                      // smoother V, residual
    } else {
      const bool coarsest = (l == nlev - 1);
      s += (o.kc_i + 1) + (coarsest ? 0 : o.kc_i) + 2;  // coarse V, Z, b, x
      if (!coarsest) s += (o.ks_i + 1) + 1;             // smoother V, residual
    }
    return s;
  }

  void upload_active(const std::vector<int>& act) {
    HELM_HIP_CHECK(hipMemcpyAsync(active_, act.data(), nseg_ * sizeof(int), hipMemcpyHostToDevice, st_));
    HELM_HIP_CHECK(hipStreamSynchronize(st_));
  }

  void make_space(Space& S, int lvl, int k, bool flex, char*& cur) {
    S.lvl = lvl;
    S.k = k;
    S.flex = flex;
    const int64_t len = H_->level(lvl).total;
    for (int i = 0; i <= k; ++i) {
      S.V[i] = reinterpret_cast<cx<T>*>(cur);
      cur += vec_bytes(len);
    }
    if (flex)
      for (int i = 0; i < k; ++i) {
        S.Z[i] = reinterpret_cast<cx<T>*>(cur);
        cur += vec_bytes(len);
      }
  }

  void make_state(KState& ks, double*& cur) {
    const int R = nseg_;
    ks.nseg = R;
    ks.H = reinterpret_cast<double2*>(cur);
    cur += 2 * (KMAX + 1) * KMAX * R;
    ks.cs = cur;
    cur += KMAX * R;
    ks.sn = reinterpret_cast<double2*>(cur);
    cur += 2 * KMAX * R;
    ks.g = reinterpret_cast<double2*>(cur);
    cur += 2 * (KMAX + 1) * R;
    ks.scale = cur;
    cur += (KMAX + 1) * R;
    ks.coef = reinterpret_cast<double2*>(cur);
    cur += 2 * (KMAX + 1) * R;
    ks.part = part_;
  }

  void allocate() {
    HELM_REQUIRE(o_.restart >= 1 && o_.restart <= KMAX, "restart must be in 1..32");
    HELM_REQUIRE(o_.ks_i >= 1 && o_.ks_i <= KMAX && o_.kc_i >= 1 && o_.kc_i <= KMAX,
                 "inner Krylov dimensions must be in 1..32");
    size_t vbytes = 0;
    for (int l = 0; l < nlev_; ++l)
      vbytes += (size_t)slots_at(o_, l, nlev_) * vec_bytes(H_->level(l).total);
    const size_t xbytes = round256((size_t)H_->level(0).total * sizeof(cx<double>));
    vec_.ensure(vbytes + xbytes + 256);
    // two partial-sum areas: vector passes, and fused stencil passes (which
    // may read the former while writing)
    part_buf_.ensure(2 * H_->max_partials() * PSTRIDE * sizeof(double));
    part_ = part_buf_.as<double>();
    spart_ = part_ + H_->max_partials() * PSTRIDE;
    const int nstates = 1 + 2 * nlev_;
    const size_t per_state = (size_t)(2 * (KMAX + 1) * KMAX + KMAX + 2 * KMAX + 2 * (KMAX + 1) + (KMAX + 1) +
                                      2 * (KMAX + 1)) * nseg_;
    small_.ensure((nstates * per_state + 2 * (size_t)nseg_) * sizeof(double) + nseg_ * sizeof(int) + 256);
    double* sc = small_.as<double>();
    beta_dev_ = sc;
    sc += 2 * nseg_;
    char* cur = reinterpret_cast<char*>(vec_.p);
    X_ = reinterpret_cast<cx<double>*>(cur);
    cur += xbytes;
    make_space(outer_, 0, o_.restart, o_.method == 1, cur);
    make_state(outer_.ks, sc);
    smooth_.resize(nlev_);
    coarse_.resize(nlev_);
    R_.assign(nlev_, nullptr);
    B_.assign(nlev_, nullptr);
    Xc_.assign(nlev_, nullptr);
    for (int l = 0; l < nlev_; ++l) {
      const int64_t len = H_->level(l).total;
      const bool coarsest = (l == nlev_ - 1);
      if (l > 0) {
        make_space(coarse_[l], l, o_.kc_i, !coarsest, cur);
        make_state(coarse_[l].ks, sc);
        B_[l] = reinterpret_cast<cx<T>*>(cur);
        cur += vec_bytes(len);
        Xc_[l] = reinterpret_cast<cx<T>*>(cur);
        cur += vec_bytes(len);
      }
      if (!coarsest) {
        make_space(smooth_[l], l, o_.ks_i, false, cur);
        make_state(smooth_[l].ks, sc);
        R_[l] = reinterpret_cast<cx<T>*>(cur);
        cur += vec_bytes(len);
      }
    }
    active_ = reinterpret_cast<int*>(sc);
  }

  // Arnoldi steps + update of one outer cycle: replayed from a graph, one
  // per direction (the launches of H and of H^H may differ: the compact
  // 27-point passes are separate kernels for the two).
  void run_cycle_body() {
    if (!graphs_enabled()) {
      cycle_body();
      return;
    }
    const int d = dir_;
    if (!exec_[d]) {
      const int64_t mv0 = fine_mv_;
      HELM_HIP_CHECK(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
      try {
        cycle_body();
      } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(st_, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      HELM_HIP_CHECK(hipStreamEndCapture(st_, &graph_[d]));
      HELM_HIP_CHECK(hipGraphInstantiate(&exec_[d], graph_[d], nullptr, nullptr, 0));
      body_mv_[d] = fine_mv_ - mv0;
      fine_mv_ = mv0;
    }
    HELM_HIP_CHECK(hipGraphLaunch(exec_[d], st_));
    fine_mv_ += body_mv_[d];
  }

  void drop_graph() {
    for (int d = 0; d < 2; ++d) {
      if (exec_[d]) (void)hipGraphExecDestroy(exec_[d]);
      if (graph_[d]) (void)hipGraphDestroy(graph_[d]);
      exec_[d] = nullptr;
      graph_[d] = nullptr;
    }
  }

  void cycle_body() {
    const bool ml = (o_.method == 1);
    outer_.v0 = outer_.V[0];
    for (int j = 0; j < outer_.k; ++j) {
      VRef<T> vj{j == 0 ? outer_.v0 : outer_.V[j], outer_.ks.scale + (int64_t)j * nseg_};
      arnoldi_step(outer_, j, vj, ml);
    }
    update_x<double>(outer_, X_);
  }

  // Stencil tiles per level, timed on two level-0 workspace vectors (zeroed
  // first) with the launch the Arnoldi steps use most: the fused pass with
  // two basis vectors where the level allows it, else the plain operator.
  // By default only for batches of different grids (measured on the 64
  // uneven problems: +2 % solves/s); for the right-hand sides of one grid
  // the heuristic tiles measured about 1 % faster end to end on the 128^3
  // 16-source solve.  HELM_AUTOTUNE=1 tunes always, =0 never.
  void tune() {
    const char* e = std::getenv("HELM_AUTOTUNE");
    bool uneven = false;
    const auto& segs = H_->level(0).host;
    for (const Seg& g : segs)
      uneven = uneven || g.n[0] != segs[0].n[0] || g.n[1] != segs[0].n[1] || g.n[2] != segs[0].n[2];
    if (e && e[0] == '0') return;
    if (!(e && e[0] == '1') && !uneven) return;
    const size_t vb = (size_t)H_->level(0).total * sizeof(cx<T>);
    HELM_HIP_CHECK(hipMemsetAsync(outer_.V[0], 0, vb, st_));
    HELM_HIP_CHECK(hipMemsetAsync(outer_.V[1], 0, vb, st_));
    const cx<T>* a = outer_.V[0];
    cx<T>* b = outer_.V[1];
    const bool f32 = std::is_same<T, float>::value;
    tune_tiles(*H_, f32 && fused_dots_ ? "arnoldi" : "apply", [&](const LevelSet& L) {
      const c32* D[2] = {reinterpret_cast<const c32*>(a), reinterpret_cast<const c32*>(a)};
      if (!(f32 && fused_dots_ && launch_h_dots(L, reinterpret_cast<const c32*>(a), nullptr, nullptr,
                                                 reinterpret_cast<c32*>(b), D, 2, true, spart_, nullptr, st_)))
        launch_h<T, T, T, T, T, false, false>(L, a, nullptr, (const cx<T>*)nullptr, nullptr, b, nullptr, nullptr,
                                              st_);
    }, st_);
  }

  // Inner products of column j (unless the stencil pass formed them:
  // fused), then w -= sum coef_i V_i with ||w||^2, and the Givens step
  // (unless deferred into the next step).  gprev >= 0: the deferred Givens
  // step of column gprev runs first.  NV: exact vector count when EXACT, else
  // an upper bound of nv.
  template <int NV, bool EXACT>
  void dots_axpy(Space& S, int nv, int j, cx<T>* w, bool fused, int gprev, bool defer) {
    const LevelSet& L = H_->level(S.lvl);
    VecList<T> vl;
    vl.v[0] = S.v0;
    for (int i = 1; i < nv; ++i) vl.v[i] = S.V[i];
    if (!fused)
      hipLaunchKernelGGL((k_dots<T, NV, EXACT>), dim3(L.nvblk), dim3(256), 0, st_, L.d(), L.vmap.as<const int>(),
                         vl, nv, (const cx<T>*)w, part_, (const int*)active_);
    hipLaunchKernelGGL((k_reduce_dots<NV, EXACT>), dim3(nseg_), dim3(256), 0, st_, L.d(), S.ks, nv, j,
                       fused ? (int)PR_STENCIL : (int)PR_VECTOR, (const double*)(fused ? spart_ : part_), gprev,
                       (const int*)active_);
    hipLaunchKernelGGL((k_axpy_norm<T, NV, EXACT>), dim3(L.nvblk), dim3(256), 0, st_, L.d(),
                       L.vmap.as<const int>(), vl, nv, w, S.ks, (const int*)active_);
    if (!defer)
      hipLaunchKernelGGL(k_givens, dim3(nseg_), dim3(256), 0, st_, L.d(), S.ks, j, j + 1 == S.k ? S.k : 0,
                         S.flex ? 0 : 1, (const int*)active_);
  }

  // Whether step j of space S runs the fused stencil + inner-product pass.
  bool fuses(const Space& S, int j) const {
    if (!std::is_same<T, float>::value || !fused_dots_) return false;
    const bool self = !S.flex;
    return can_fuse_dots(H_->level(S.lvl), self ? j : j + 1, self);
  }

  // Whether the Givens step of column j moves into step j + 1: GMRES spaces
  // whose next step is fused (that pass derives its input scale from the
  // partial norms itself, and its reduction kernel runs the Givens step).
  bool defers_givens(const Space& S, int j) const { return !S.flex && j + 1 < S.k && fuses(S, j + 1); }

  // w = s_x H x with, where the level allows it, the inner products of w
  // with the basis V_0..V_j in the same pass (x itself is V_j for GMRES).
  // npart: derive s_x from these partial norms instead of xs.
  bool apply_arnoldi(Space& S, int j, const cx<T>* x, const double* xs, const double* npart, cx<T>* w) {
    const LevelSet& L = H_->level(S.lvl);
    bool fused = false;
    if (fuses(S, j)) {
      const c32* D[6];
      const bool self = !S.flex;  // GMRES: x is the basis vector V_j
      const int nmem = self ? j : j + 1;
      for (int i = 0; i < nmem; ++i) D[i] = reinterpret_cast<const c32*>(i == 0 ? S.v0 : S.V[i]);
      fused = launch_h_dots(L, reinterpret_cast<const c32*>(x), xs, npart, reinterpret_cast<c32*>(w), D, nmem,
                            self, spart_, active_, st_);
    }
    HELM_REQUIRE(fused || !npart, "internal: deferred Givens step without the fused stencil pass");
    if (!fused)
      launch_h<T, T, T, T, T, false, false>(L, x, xs, (const cx<T>*)nullptr, nullptr, w, nullptr, active_, st_);
    return fused;
  }

  // Arnoldi column j of space S from basis vector vj (with scale).
  void arnoldi_step(Space& S, int j, VRef<T> vj, bool precond) {
    cx<T>* w = S.V[j + 1];
    const bool defer_prev = j > 0 && defers_givens(S, j - 1);
    bool fused;
    if (S.flex) {
      HELM_REQUIRE(precond, "flexible space without preconditioner");
      vcycle(S.lvl, vj, S.Z[j]);
      fused = apply_arnoldi(S, j, S.Z[j], nullptr, nullptr, w);
    } else {
      fused = apply_arnoldi(S, j, vj.p, defer_prev ? nullptr : vj.s, defer_prev ? part_ : nullptr, w);
    }
    if (S.lvl == 0) fine_mv_++;
    const int nv = j + 1;
    const int gprev = defer_prev ? j - 1 : -1;
    const bool defer = defers_givens(S, j);
    switch (nv) {
      case 1: dots_axpy<1, true>(S, nv, j, w, fused, gprev, defer); break;
      case 2: dots_axpy<2, true>(S, nv, j, w, fused, gprev, defer); break;
      case 3: dots_axpy<3, true>(S, nv, j, w, fused, gprev, defer); break;
      case 4: dots_axpy<4, true>(S, nv, j, w, fused, gprev, defer); break;
      case 5: dots_axpy<5, true>(S, nv, j, w, fused, gprev, defer); break;
      case 6: dots_axpy<6, true>(S, nv, j, w, fused, gprev, defer); break;
      default:
        if (nv <= 11) dots_axpy<11, false>(S, nv, j, w, fused, gprev, defer);
        else if (nv <= 21) dots_axpy<21, false>(S, nv, j, w, fused, gprev, defer);
        else dots_axpy<33, false>(S, nv, j, w, fused, gprev, defer);
    }
  }

  template <typename TX>
  void update_x(Space& S, cx<TX>* x) {
    const LevelSet& L = H_->level(S.lvl);
    VecList<T> D;
    for (int j = 0; j < S.k; ++j) D.v[j] = S.flex ? S.Z[j] : (j == 0 ? S.v0 : S.V[j]);
    const dim3 grid(L.nvblk);
    const int* vm = L.vmap.as<const int>();
    const int* act = active_;
#define HELM_UPD(KM, EX) \
  hipLaunchKernelGGL((k_update_x<TX, T, KM, EX>), grid, dim3(256), 0, st_, L.d(), vm, D, S.k, S.ks, x, act)
    switch (S.k) {
      case 1: HELM_UPD(1, true); break;
      case 2: HELM_UPD(2, true); break;
      case 3: HELM_UPD(3, true); break;
      case 4: HELM_UPD(4, true); break;
      case 5: HELM_UPD(5, true); break;
      default:
        if (S.k <= 10) HELM_UPD(10, false);
        else if (S.k <= 20) HELM_UPD(20, false);
        else HELM_UPD(32, false);
    }
#undef HELM_UPD
  }

  // `cycles` restart cycles of the space's (F)GMRES on level S.lvl for
  // A x = b; x_zero: x starts at 0 (x is cleared here).
  void krylov(Space& S, VRef<T> b, cx<T>* x, bool x_zero, int cycles) {
    const LevelSet& L = H_->level(S.lvl);
    const int* vm = L.vmap.as<const int>();
    if (x_zero)
      hipLaunchKernelGGL((k_zero<T>), dim3(L.nvblk), dim3(256), 0, st_, L.d(), vm, x, (const int*)active_);
    for (int c = 0; c < cycles; ++c) {
      if (c == 0 && x_zero) {
        S.v0 = b.p;
        hipLaunchKernelGGL((k_norm2<T>), dim3(L.nvblk), dim3(256), 0, st_, L.d(), vm, b.p, part_,
                           (const int*)active_);
        hipLaunchKernelGGL(k_start_cycle, dim3(nseg_), dim3(256), 0, st_, L.d(), S.ks, (int)PR_VECTOR, b.s,
                           (double*)nullptr, (const int*)active_);
      } else {
        S.v0 = S.V[0];
        const int rng = launch_h<T, T, T, T, T, true, true>(L, x, nullptr, b.p, b.s, S.V[0], part_, active_, st_);
        if (S.lvl == 0) fine_mv_++;
        hipLaunchKernelGGL(k_start_cycle, dim3(nseg_), dim3(256), 0, st_, L.d(), S.ks, rng,
                           (const double*)nullptr, (double*)nullptr, (const int*)active_);
      }
      for (int j = 0; j < S.k; ++j) {
        VRef<T> vj{j == 0 ? S.v0 : S.V[j], S.ks.scale + (int64_t)j * nseg_};
        arnoldi_step(S, j, vj, S.flex);
      }
      update_x<T>(S, x);
    }
  }

  // x = V-cycle_l(b), x overwritten.
  void vcycle(int l, VRef<T> b, cx<T>* x) {
    const LevelSet& L = H_->level(l);
    const LevelSet& Lc = H_->level(l + 1);
    krylov(smooth_[l], b, x, true, o_.ks_o);  // pre-smooth from 0
    launch_h<T, T, T, T, T, true, false>(L, x, nullptr, b.p, b.s, R_[l], nullptr, active_, st_);  // r = b - H x
    if (l == 0) fine_mv_++;
    hipLaunchKernelGGL((k_restrict<T>), dim3(Lc.ntblk), dim3(256), 0, st_, L.d(), Lc.d(),
                       Lc.tmap.as<const int>(), (const cx<T>*)R_[l], (const double*)nullptr, B_[l + 1],
                       (const int*)active_);
    VRef<T> bc{B_[l + 1], nullptr};
    krylov(coarse_[l + 1], bc, Xc_[l + 1], true, o_.kc_o);  // coarse solve
    hipLaunchKernelGGL((k_prolong_add<T>), dim3(L.ntblk), dim3(256), 0, st_, L.d(), Lc.d(),
                       L.tmap.as<const int>(), (const cx<T>*)Xc_[l + 1], x, (const int*)active_);
    krylov(smooth_[l], b, x, false, o_.ks_o);  // post-smooth
  }

  SolveOpts o_;
  hipStream_t st_;
  int nseg_;
  int nlev_ = 1;
  std::unique_ptr<Hierarchy> H_;
  DevBuf vec_, part_buf_, small_;
  double* part_ = nullptr;
  double* spart_ = nullptr;
  double* beta_dev_ = nullptr;
  int* active_ = nullptr;
  cx<double>* X_ = nullptr;
  Space outer_;
  std::vector<Space> smooth_, coarse_;
  std::vector<cx<T>*> R_, B_, Xc_;
  int64_t fine_mv_ = 0, body_mv_[2] = {0, 0};
  int dir_ = 0;  // direction of the current solve (0: H, 1: H^H)
  bool fused_dots_ = fused_dots_enabled();
  hipGraph_t graph_[2] = {nullptr, nullptr};
  hipGraphExec_t exec_[2] = {nullptr, nullptr};
};

}  // namespace helm
