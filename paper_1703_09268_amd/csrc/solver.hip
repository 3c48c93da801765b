// Host orchestration of the preconditioned Krylov solve (arXiv:1703.09268,
// ML-GMRES section) on many right-hand sides at once.
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
//   the device; the host synchronises once per outer cycle for the
//   convergence test.
// * Right-hand sides that reach the tolerance (or turn non-finite) are
//   switched off through a device mask that every kernel reads.
#pragma once

#include <algorithm>
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
  const double* s;  // per right-hand-side scale (null = 1)
};

inline unsigned vec_blocks(int64_t N) { return std::min<unsigned>(DOT_BLOCKS, ceil_div(N, 256)); }

__global__ __launch_bounds__(64) void k_sqrt_sum(const double* __restrict__ part, int nblk,
                                                 double* __restrict__ out) {
  const int r = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) s += part[((int64_t)r * nblk + b) * PSTRIDE];
  s = wave_sum(s);
  if (threadIdx.x == 0) out[r] = sqrt(s);
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

  Solver(const GridSpec& g, const T* m, double omega, int nrhs, const SolveOpts& o, hipStream_t st)
      : g_(g), omega_(omega), nrhs_(nrhs), o_(o), st_(st) {
    nlev_ = (o.method == 1) ? o.levels : 1;
    levels_.resize(nlev_);
    int n[3] = {g.n[0], g.n[1], g.n[2]};
    double h = g.h;
    int stride = 1;
    for (int l = 0; l < nlev_; ++l) {
      levels_[l].reset(new Level());
      init_level(g, *levels_[l], n, h, stride, omega, st);
      if (l == 0) {
        levels_[l]->m = m;
      } else {
        Level& Lc = *levels_[l];
        const Level& Lf = *levels_[l - 1];
        Lc.m_own.ensure(Lc.N * sizeof(T));
        hipLaunchKernelGGL((k_inject_model<T>), dim3(ceil_div(Lc.N, 256)), dim3(256), 0, st,
                           (const T*)Lf.m, Lf.n[0], Lf.n[1], Lf.n[2], (T*)Lc.m_own.p, Lc.n[0], Lc.n[1],
                           Lc.n[2]);
        Lc.m = Lc.m_own.p;
      }
      for (int a = 0; a < 3; ++a) n[a] = n[a] / 2 + 1;
      h *= 2.0;
      stride *= 2;
    }
    allocate();
  }

  const Level& level(int l) const { return *levels_[l]; }
  // FP64 outer iterates of the last solve ([nrhs][N]); valid until the next solve
  const cx<double>* iterate() const { return X_; }
  int64_t fine_matvecs() const { return fine_mv_; }

  // ---- plain operator application -------------------------------------
  void apply(int adj, const cx<T>* x, cx<T>* y) {
    const Level& L = *levels_[0];
    launch_h<T, T, T, T, T, false, false>(L, adj, nrhs_, x, nullptr, (const T*)L.m, (const cx<T>*)nullptr,
                                          nullptr, y, nullptr, nullptr, st_);
    HELM_HIP_CHECK(hipGetLastError());
  }

  // ---- full solve ---------------------------------------------------------
  // q, u: nrhs blocks of N; info: nrhs entries.  Returns the worst status.
  int solve(int adj, const cx<T>* q, cx<T>* u, SolveInfo* info) {
    adj_ = adj;
    const Level& L = *levels_[0];
    const int64_t N = L.N;
    std::vector<int> act(nrhs_, 1);
    std::vector<double> qn(nrhs_), beta(nrhs_);
    for (int r = 0; r < nrhs_; ++r) info[r] = SolveInfo();
    // ||q||
    {
      dim3 grid(vec_blocks(N), nrhs_);
      hipLaunchKernelGGL((k_norm2<T>), grid, dim3(256), 0, st_, q, N, part_, (const int*)nullptr);
      hipLaunchKernelGGL(k_sqrt_sum, dim3(nrhs_), dim3(64), 0, st_, (const double*)part_, (int)grid.x,
                         beta_dev_);
      HELM_HIP_CHECK(hipMemcpyAsync(qn.data(), beta_dev_, nrhs_ * sizeof(double), hipMemcpyDeviceToHost, st_));
      HELM_HIP_CHECK(hipStreamSynchronize(st_));
    }
    // outer iterate in FP64
    {
      dim3 grid(vec_blocks(N) * 4, 1);
      if (o_.warm_start)
        hipLaunchKernelGGL((k_convert<double, T>), grid, dim3(256), 0, st_, (const cx<T>*)u, X_, N * nrhs_);
      else
        hipLaunchKernelGGL((k_zero<double>), dim3(vec_blocks(N) * 4, nrhs_), dim3(256), 0, st_, X_, N,
                           (const int*)nullptr);
    }
    for (int r = 0; r < nrhs_; ++r) {
      if (!(qn[r] > 0.0)) {  // zero (or non-finite) right-hand side
        act[r] = 0;
        info[r].status = std::isfinite(qn[r]) ? 0 : 2;
        info[r].relres = std::isfinite(qn[r]) ? 0.0 : qn[r];
        if (std::isfinite(qn[r]))
          HELM_HIP_CHECK(hipMemsetAsync(X_ + (int64_t)r * N, 0, N * sizeof(cx<double>), st_));
      }
    }
    upload_active(act);
    fine_mv_ = 0;
    const bool ml = (o_.method == 1);
    int cyc = 0;
    for (;; ++cyc) {
      // true residual in FP64, stored (rounded) as the first basis vector
      const int nb = launch_h<double, double, T, T, T, true, true>(L, adj_, nrhs_, X_, nullptr,
                                                                    (const T*)L.m, q, nullptr, outer_.V[0],
                                                                    part_, active_, st_);
      fine_mv_++;
      hipLaunchKernelGGL(k_start_cycle, dim3(nrhs_), dim3(64), 0, st_, outer_.ks, nb, (const double*)nullptr,
                         beta_dev_, (const int*)active_);
      HELM_HIP_CHECK(hipMemcpyAsync(beta.data(), beta_dev_, nrhs_ * sizeof(double), hipMemcpyDeviceToHost, st_));
      HELM_HIP_CHECK(hipStreamSynchronize(st_));
      int n_active = 0;
      for (int r = 0; r < nrhs_; ++r) {
        if (!act[r]) continue;
        const double rel = beta[r] / qn[r];
        info[r].relres = rel;
        info[r].cycles = cyc;
        info[r].matvecs = fine_mv_;
        if (!std::isfinite(rel)) {
          act[r] = 0;
          info[r].status = 2;
        } else if (rel <= o_.tol) {
          act[r] = 0;
          info[r].status = 0;
        } else if (cyc >= o_.max_cycles) {
          act[r] = 0;
          info[r].status = 1;
        } else {
          ++n_active;
        }
      }
      upload_active(act);
      if (n_active == 0) break;
      outer_.v0 = outer_.V[0];
      for (int j = 0; j < outer_.k; ++j) {
        VRef<T> vj{j == 0 ? outer_.v0 : outer_.V[j], outer_.ks.scale + (int64_t)j * nrhs_};
        arnoldi_step(outer_, j, vj, ml);
      }
      for (int r = 0; r < nrhs_; ++r)
        if (act[r]) info[r].inner_its += outer_.k;
      update_x<double>(outer_, X_);
    }
    // result in the caller's precision
    hipLaunchKernelGGL((k_convert<T, double>), dim3(vec_blocks(N) * 4), dim3(256), 0, st_,
                       (const cx<double>*)X_, u, N * nrhs_);
    HELM_HIP_CHECK(hipGetLastError());
    HELM_HIP_CHECK(hipStreamSynchronize(st_));
    int worst = 0;
    for (int r = 0; r < nrhs_; ++r) worst = std::max(worst, info[r].status);
    return worst;
  }

  static size_t workspace_bytes(const GridSpec& g, const SolveOpts& o, int nrhs) {
    size_t total = 0;
    int n[3] = {g.n[0], g.n[1], g.n[2]};
    const int nlev = (o.method == 1) ? o.levels : 1;
    for (int l = 0; l < nlev; ++l) {
      const int64_t N = (int64_t)n[0] * n[1] * n[2];
      total += (size_t)slots_at(o, l, nlev) * N * nrhs * sizeof(cx<T>);
      if (l > 0) total += (size_t)N * sizeof(T);
      for (int a = 0; a < 3; ++a) n[a] = n[a] / 2 + 1;
    }
    const int64_t N0 = (int64_t)g.n[0] * g.n[1] * g.n[2];
    total += (size_t)N0 * nrhs * sizeof(cx<double>);  // FP64 outer iterate
    return total;
  }

 private:
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
    HELM_HIP_CHECK(hipMemcpyAsync(active_, act.data(), nrhs_ * sizeof(int), hipMemcpyHostToDevice, st_));
    HELM_HIP_CHECK(hipStreamSynchronize(st_));
  }

  void make_space(Space& S, int lvl, int k, bool flex, char*& cur) {
    S.lvl = lvl;
    S.k = k;
    S.flex = flex;
    const int64_t N = levels_[lvl]->N;
    for (int i = 0; i <= k; ++i) {
      S.V[i] = reinterpret_cast<cx<T>*>(cur);
      cur += (size_t)N * nrhs_ * sizeof(cx<T>);
    }
    if (flex)
      for (int i = 0; i < k; ++i) {
        S.Z[i] = reinterpret_cast<cx<T>*>(cur);
        cur += (size_t)N * nrhs_ * sizeof(cx<T>);
      }
  }

  void make_state(KState& ks, double*& cur) {
    const int R = nrhs_;
    ks.nrhs = R;
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
    // vectors
    size_t vbytes = 0;
    for (int l = 0; l < nlev_; ++l)
      vbytes += (size_t)slots_at(o_, l, nlev_) * levels_[l]->N * nrhs_ * sizeof(cx<T>);
    const size_t xbytes = (size_t)levels_[0]->N * nrhs_ * sizeof(cx<double>);
    vec_.ensure(vbytes + xbytes + 256);
    // partial sums: the largest per-rhs workgroup count of any reduction
    int maxblk = (int)DOT_BLOCKS;
    for (int l = 0; l < nlev_; ++l) maxblk = std::max(maxblk, nblk_stencil(*levels_[l], nrhs_));
    part_buf_.ensure((size_t)maxblk * nrhs_ * PSTRIDE * sizeof(double));
    part_ = reinterpret_cast<double*>(part_buf_.p);
    // small per-rhs arrays
    const int nstates = 1 + 2 * nlev_;
    const size_t per_state = (size_t)(2 * (KMAX + 1) * KMAX + KMAX + 2 * KMAX + 2 * (KMAX + 1) + (KMAX + 1) +
                                      2 * (KMAX + 1)) * nrhs_;
    small_.ensure((nstates * per_state + 2 * nrhs_) * sizeof(double) + nrhs_ * sizeof(int) + 256);
    double* sc = reinterpret_cast<double*>(small_.p);
    beta_dev_ = sc;
    sc += nrhs_;
    sc += nrhs_;
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
      const int64_t N = levels_[l]->N;
      const bool coarsest = (l == nlev_ - 1);
      if (l > 0) {
        make_space(coarse_[l], l, o_.kc_i, !coarsest, cur);
        make_state(coarse_[l].ks, sc);
        B_[l] = reinterpret_cast<cx<T>*>(cur);
        cur += (size_t)N * nrhs_ * sizeof(cx<T>);
        Xc_[l] = reinterpret_cast<cx<T>*>(cur);
        cur += (size_t)N * nrhs_ * sizeof(cx<T>);
      }
      if (!coarsest || (l == 0 && nlev_ > 1)) {
        make_space(smooth_[l], l, o_.ks_i, false, cur);
        make_state(smooth_[l].ks, sc);
        R_[l] = reinterpret_cast<cx<T>*>(cur);
        cur += (size_t)N * nrhs_ * sizeof(cx<T>);
      }
    }
    active_ = reinterpret_cast<int*>(sc);
  }

  template <int NV>
  void dots_axpy(Space& S, int nv, int j, cx<T>* w) {
    const int64_t N = levels_[S.lvl]->N;
    VecList<T> vl;
    vl.v[0] = S.v0;
    for (int i = 1; i < nv; ++i) vl.v[i] = S.V[i];
    const dim3 grid(vec_blocks(N), nrhs_);
    hipLaunchKernelGGL((k_dots<T, NV>), grid, dim3(256), 0, st_, vl, nv, (const cx<T>*)w, N, part_,
                       (const int*)active_);
    hipLaunchKernelGGL(k_reduce_dots, dim3(nrhs_), dim3(64), 0, st_, S.ks, nv, j, (int)grid.x,
                       (const int*)active_);
    hipLaunchKernelGGL((k_axpy_norm<T, NV>), grid, dim3(256), 0, st_, vl, nv, w, N, S.ks,
                       (const int*)active_);
    hipLaunchKernelGGL(k_givens, dim3(nrhs_), dim3(64), 0, st_, S.ks, j, (int)grid.x, (const int*)active_);
  }

  // Arnoldi column j of space S from basis vector vj (with scale).
  void arnoldi_step(Space& S, int j, VRef<T> vj, bool precond) {
    const Level& L = *levels_[S.lvl];
    cx<T>* w = S.V[j + 1];
    if (S.flex) {
      if (precond)
        vcycle(S.lvl, vj, S.Z[j]);
      else
        HELM_REQUIRE(false, "flexible space without preconditioner");
      launch_h<T, T, T, T, T, false, false>(L, adj_, nrhs_, S.Z[j], nullptr, (const T*)L.m,
                                            (const cx<T>*)nullptr, nullptr, w, nullptr, active_, st_);
    } else {
      launch_h<T, T, T, T, T, false, false>(L, adj_, nrhs_, vj.p, vj.s, (const T*)L.m, (const cx<T>*)nullptr,
                                            nullptr, w, nullptr, active_, st_);
    }
    if (S.lvl == 0) fine_mv_++;
    const int nv = j + 1;
    if (nv <= 6) dots_axpy<6>(S, nv, j, w);
    else if (nv <= 11) dots_axpy<11>(S, nv, j, w);
    else if (nv <= 21) dots_axpy<21>(S, nv, j, w);
    else dots_axpy<33>(S, nv, j, w);
  }

  template <typename TX>
  void update_x(Space& S, cx<TX>* x) {
    const int64_t N = levels_[S.lvl]->N;
    VecList<T> D;
    for (int j = 0; j < S.k; ++j) D.v[j] = S.flex ? S.Z[j] : (j == 0 ? S.v0 : S.V[j]);
    const dim3 grid(vec_blocks(N), nrhs_);
    if (S.k <= 5)
      hipLaunchKernelGGL((k_update_x<TX, T, 5>), grid, dim3(256), 0, st_, D, S.k, !S.flex, S.ks, x, N,
                         (const int*)active_);
    else if (S.k <= 10)
      hipLaunchKernelGGL((k_update_x<TX, T, 10>), grid, dim3(256), 0, st_, D, S.k, !S.flex, S.ks, x, N,
                         (const int*)active_);
    else if (S.k <= 20)
      hipLaunchKernelGGL((k_update_x<TX, T, 20>), grid, dim3(256), 0, st_, D, S.k, !S.flex, S.ks, x, N,
                         (const int*)active_);
    else
      hipLaunchKernelGGL((k_update_x<TX, T, 32>), grid, dim3(256), 0, st_, D, S.k, !S.flex, S.ks, x, N,
                         (const int*)active_);
  }

  // `cycles` restart cycles of the space's (F)GMRES on level S.lvl for
  // A x = b; x_zero: x starts at 0 (x is cleared here).
  void krylov(Space& S, VRef<T> b, cx<T>* x, bool x_zero, int cycles) {
    const Level& L = *levels_[S.lvl];
    const int64_t N = L.N;
    if (x_zero)
      hipLaunchKernelGGL((k_zero<T>), dim3(vec_blocks(N), nrhs_), dim3(256), 0, st_, x, N,
                         (const int*)active_);
    for (int c = 0; c < cycles; ++c) {
      if (c == 0 && x_zero) {
        S.v0 = b.p;
        const dim3 grid(vec_blocks(N), nrhs_);
        hipLaunchKernelGGL((k_norm2<T>), grid, dim3(256), 0, st_, b.p, N, part_, (const int*)active_);
        hipLaunchKernelGGL(k_start_cycle, dim3(nrhs_), dim3(64), 0, st_, S.ks, (int)grid.x, b.s,
                           (double*)nullptr, (const int*)active_);
      } else {
        S.v0 = S.V[0];
        const int nb = launch_h<T, T, T, T, T, true, true>(L, adj_, nrhs_, x, nullptr, (const T*)L.m, b.p,
                                                           b.s, S.V[0], part_, active_, st_);
        if (S.lvl == 0) fine_mv_++;
        hipLaunchKernelGGL(k_start_cycle, dim3(nrhs_), dim3(64), 0, st_, S.ks, nb, (const double*)nullptr,
                           (double*)nullptr, (const int*)active_);
      }
      for (int j = 0; j < S.k; ++j) {
        VRef<T> vj{j == 0 ? S.v0 : S.V[j], S.ks.scale + (int64_t)j * nrhs_};
        arnoldi_step(S, j, vj, S.flex);
      }
      update_x<T>(S, x);
    }
  }

  // x = V-cycle_l(b), x overwritten.
  void vcycle(int l, VRef<T> b, cx<T>* x) {
    const Level& L = *levels_[l];
    const Level& Lc = *levels_[l + 1];
    krylov(smooth_[l], b, x, true, o_.ks_o);  // pre-smooth from 0
    launch_h<T, T, T, T, T, true, false>(L, adj_, nrhs_, x, nullptr, (const T*)L.m, b.p, b.s, R_[l], nullptr,
                                         active_, st_);  // r = b - H x
    if (l == 0) fine_mv_++;
    hipLaunchKernelGGL((k_restrict<T>), dim3(ceil_div(Lc.N, 256), nrhs_), dim3(256), 0, st_,
                       (const cx<T>*)R_[l], (const double*)nullptr, L.n[0], L.n[1], L.n[2], B_[l + 1], Lc.n[0],
                       Lc.n[1], Lc.n[2], (const int*)active_);
    VRef<T> bc{B_[l + 1], nullptr};
    krylov(coarse_[l + 1], bc, Xc_[l + 1], true, o_.kc_o);  // coarse solve
    hipLaunchKernelGGL((k_prolong_add<T>), dim3(ceil_div(L.N, 256), nrhs_), dim3(256), 0, st_,
                       (const cx<T>*)Xc_[l + 1], Lc.n[0], Lc.n[1], Lc.n[2], x, L.n[0], L.n[1], L.n[2],
                       (const int*)active_);
    krylov(smooth_[l], b, x, false, o_.ks_o);  // post-smooth
  }

  GridSpec g_;
  double omega_;
  int nrhs_;
  SolveOpts o_;
  hipStream_t st_;
  int adj_ = 0;
  int nlev_ = 1;
  std::vector<std::unique_ptr<Level>> levels_;
  DevBuf vec_, part_buf_, small_;
  double* part_ = nullptr;
  double* beta_dev_ = nullptr;
  int* active_ = nullptr;
  cx<double>* X_ = nullptr;
  Space outer_;
  std::vector<Space> smooth_, coarse_;
  std::vector<cx<T>*> R_, B_, Xc_;
  int64_t fine_mv_ = 0;
};

}  // namespace helm
