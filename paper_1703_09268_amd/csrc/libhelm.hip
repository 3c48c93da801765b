// C ABI of the Helmholtz library (declared in include/helm.h).  Everything
// below the ABI is C++/HIP; no exception crosses it.  This translation unit
// includes the kernel and runtime sources so the library builds as one
// gfx950 code object.
#include "../../include/helm.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "fwi.hip"
#include "lbfgs.hip"
#include "wri.hip"
#include "model25d.hip"
#include "noalloc.hip"
#include "solver.hip"

namespace {

// A solver kept by the context for the next call with the same problems and
// structural options (its workspace, tables and captured graph are reused;
// the coarse models are re-injected from the current model contents on
// every solve).
struct CachedSolver {
  std::string key;
  std::unique_ptr<helm::Solver<float>> s32;
  std::unique_ptr<helm::Solver<double>> s64;
};

}  // namespace

struct helm_ctx {
  int device = 0;
  std::string err;
  hipStream_t stream = nullptr;  // internal stream of the solves (capturable)
  hipEvent_t ev = nullptr;
  helm::DevBuf fwi_buf;          // sources / fields scratch of misfit_gradient
  helm::DevBuf fwi_small;
  helm::DevBuf batch_buf;        // concatenated q / u of a batched solve
  helm::DevBuf drv_buf;          // L-BFGS vectors of the inversion driver
  helm::DevBuf chk;              // flags of the input scan (HELM_CHECK=1)
  CachedSolver solver;
  std::unique_ptr<helm::Hierarchy> apply_h;  // operator of the last helm_apply
  std::string apply_key;
};

namespace {

std::string g_global_err;

helm_status fail(helm_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  else g_global_err = msg;
  return (helm_status)code;
}

template <typename F>
helm_status guarded(helm_ctx* ctx, F&& f) {
  if (!ctx) return fail(nullptr, HELM_E_INVAL, "null context");
  try {
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(ctx, HELM_E_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    ctx->err.clear();
    return f();
  } catch (const helm::Error& e) {
    (void)hipGetLastError();  // do not leave a sticky error for the caller's next HIP call
    return fail(ctx, e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(ctx, HELM_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(ctx, HELM_E_HIP, "unexpected C++ exception");
  }
}

void check_grid(const helm_grid* g) {
  HELM_REQUIRE(g != nullptr, "null grid");
  // n[0] == 1: the two-dimensional operator on the (n[1], n[2]) plane
  HELM_REQUIRE(g->n[0] == 1 || g->n[0] >= 3, "grid sizes must be >= 3 (or n[0] = 1 for a 2D grid)");
  for (int a = 1; a < 3; ++a) HELM_REQUIRE(g->n[a] >= 3, "grid sizes must be >= 3");
  HELM_REQUIRE((int64_t)g->n[0] * g->n[1] * g->n[2] < ((int64_t)1 << 40), "grid too large");
  HELM_REQUIRE(g->h > 0.0 && std::isfinite(g->h), "grid spacing must be positive");
  HELM_REQUIRE(g->npml >= 0, "npml must be >= 0");
  for (int a = 0; a < 3; ++a)
    HELM_REQUIRE(g->n[a] == 1 || 2 * g->npml < g->n[a], "npml must be < n/2 on every axis");
  if (g->npml > 0) {
    HELM_REQUIRE(g->pml_R > 0.0 && g->pml_R < 1.0, "pml_R must be in (0, 1)");
    HELM_REQUIRE(g->v_ref > 0.0 && std::isfinite(g->v_ref), "v_ref must be positive");
  }
  HELM_REQUIRE(g->stencil == HELM_7PT || g->stencil == HELM_27PT, "unknown stencil");
  HELM_REQUIRE(g->dtype == HELM_C64 || g->dtype == HELM_C128, "unknown dtype");
  if (g->stencil == HELM_27PT)
    for (int c = 0; c < 7; ++c) HELM_REQUIRE(std::isfinite(g->w27[c]), "27-point weights must be finite");
  HELM_REQUIRE(g->n[0] > 1 || g->stencil == HELM_7PT, "2D grids (n[0] = 1) use the 7-point stencil");
}

helm::GridSpec spec_of(const helm_grid* g) {
  helm::GridSpec s;
  std::memset(&s, 0, sizeof(s));
  for (int a = 0; a < 3; ++a) s.n[a] = g->n[a];
  s.h = g->h;
  s.npml = g->npml;
  s.R = g->npml > 0 ? g->pml_R : 0.5;
  s.vref = g->npml > 0 ? g->v_ref : 1.0;
  s.stencil = g->stencil;
  for (int c = 0; c < 7; ++c) s.w27[c] = g->stencil == HELM_27PT ? g->w27[c] : 0.0;
  return s;
}

helm::SolveOpts opts_of(const helm_solver_opts* o) {
  helm_solver_opts d;
  helm_default_opts(&d);
  if (!o) o = &d;
  helm::SolveOpts s;
  std::memset(&s, 0, sizeof(s));
  HELM_REQUIRE(o->method == HELM_GMRES || o->method == HELM_FGMRES_ML, "unknown solver method");
  HELM_REQUIRE(o->restart >= 1 && o->restart <= helm::KMAX, "restart must be in 1..32");
  HELM_REQUIRE(o->max_cycles >= 0, "max_cycles must be >= 0");
  HELM_REQUIRE(o->tol > 0.0, "tol must be > 0");
  const bool ml = o->method == HELM_FGMRES_ML;
  if (ml) {
    HELM_REQUIRE(o->levels >= 2 && o->levels <= 4, "levels must be in 2..4");
    HELM_REQUIRE(o->ks_o >= 1 && o->kc_o >= 1, "smoother / coarse cycles must be >= 1");
    HELM_REQUIRE(o->ks_i >= 1 && o->ks_i <= helm::KMAX && o->kc_i >= 1 && o->kc_i <= helm::KMAX,
                 "smoother / coarse Krylov dimensions must be in 1..32");
  }
  s.method = o->method;
  s.restart = o->restart;
  s.max_cycles = o->max_cycles;
  s.tol = o->tol;
  s.ks_o = ml ? o->ks_o : 1;
  s.ks_i = ml ? o->ks_i : 1;
  s.kc_o = ml ? o->kc_o : 1;
  s.kc_i = ml ? o->kc_i : 1;
  s.levels = ml ? o->levels : 1;
  s.warm_start = o->warm_start;
  return s;
}

void check_coarse_sizes(const helm_grid* g, const helm::SolveOpts& o) {
  if (o.method != HELM_FGMRES_ML) return;
  int n[3] = {g->n[0], g->n[1], g->n[2]};
  for (int l = 1; l < o.levels; ++l)
    for (int a = 0; a < 3; ++a) {
      if (n[a] == 1) continue;  // the absent axis of a 2D grid
      n[a] = n[a] / 2 + 1;
      HELM_REQUIRE(n[a] >= 3, "grid too small for the requested number of levels");
    }
}

void to_info(const helm::SolveInfo& s, helm_solve_info* o) {
  o->status = s.status;
  o->cycles = s.cycles;
  o->inner_its = s.inner_its;
  o->pad_ = 0;
  o->matvecs = s.matvecs;
  o->relres_fp64 = s.relres;
}

// The internal stream every solve runs on, ordered after the caller's
// pending work.  (A graph capture needs a stream of its own; the default
// stream cannot be captured.)
hipStream_t solve_stream(helm_ctx* ctx, void* caller) {
  if (!ctx->stream) {
    HELM_HIP_CHECK(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
    HELM_HIP_CHECK(hipEventCreateWithFlags(&ctx->ev, hipEventDisableTiming));
  }
  HELM_HIP_CHECK(hipEventRecord(ctx->ev, (hipStream_t)caller));
  HELM_HIP_CHECK(hipStreamWaitEvent(ctx->stream, ctx->ev, 0));
  return ctx->stream;
}

std::string key_of(const std::vector<helm::ProblemSpec>& probs, const helm::SolveOpts& o, int dtype) {
  std::string k((const char*)&o, sizeof(o));
  k.append((const char*)&dtype, sizeof(int));
  for (const auto& p : probs) {
    k.append((const char*)&p.g, sizeof(p.g));
    k.append((const char*)&p.omega, sizeof(double));
    k.append((const char*)&p.m, sizeof(void*));
  }
  return k;
}

template <typename T>
std::unique_ptr<helm::Solver<T>>& slot_of(CachedSolver& c);
template <>
std::unique_ptr<helm::Solver<float>>& slot_of<float>(CachedSolver& c) { return c.s32; }
template <>
std::unique_ptr<helm::Solver<double>>& slot_of<double>(CachedSolver& c) { return c.s64; }

// The cached solver for these problems (structure: grids, omegas, models,
// Krylov sizes), built on a miss.  Tolerance, cycle limit and warm start are
// per call.
template <typename T>
helm::Solver<T>& solver_for(helm_ctx* ctx, const std::vector<helm::ProblemSpec>& probs, const helm::SolveOpts& o,
                            hipStream_t st, bool pad_fine = false) {
  helm::SolveOpts ko = o;
  ko.warm_start = 0;
  ko.max_cycles = 0;
  ko.tol = 0.0;
  const std::string key = key_of(probs, ko, sizeof(T) == 4 ? HELM_C64 : HELM_C128) + (pad_fine ? "P" : "U");
  auto& slot = slot_of<T>(ctx->solver);
  if (!slot || ctx->solver.key != key) {
    ctx->solver.s32.reset();  // free the old workspace before allocating
    ctx->solver.s64.reset();
    slot.reset(new helm::Solver<T>(probs, o, st, pad_fine));
    ctx->solver.key = key;
  }
  slot->set_call_opts(o);
  return *slot;
}

// A complex64 solve of problems with an odd nz runs its fine level in
// the even-pitch layout of the pair-tiled kernels (right-hand sides and
// fields are copied in and out); everything else uses the caller's layout.
bool wants_pad(const std::vector<helm::ProblemSpec>& ps, bool f32) {
  if (!f32) return false;
  bool odd = false;
  for (const auto& p : ps) odd = odd || (p.g.n[2] & 1);
  return odd;
}

// dst (pitch dpz elements per z row) <- src (pitch spz), `rows` rows of nz
template <typename T>
void copy_rows(void* dst, int dpz, const void* src, int spz, int nz, size_t rows, hipStream_t st) {
  HELM_HIP_CHECK(hipMemcpy2DAsync(dst, (size_t)dpz * sizeof(helm::cx<T>), src, (size_t)spz * sizeof(helm::cx<T>),
                                  (size_t)nz * sizeof(helm::cx<T>), rows, hipMemcpyDeviceToDevice, st));
}

std::vector<helm::ProblemSpec> shared_problems(const helm_grid* g, const void* m, double omega, int dir, int n) {
  helm::ProblemSpec p;
  std::memset(&p, 0, sizeof(p));
  p.g = spec_of(g);
  p.omega = omega;
  p.dir = dir;
  p.m = m;
  return std::vector<helm::ProblemSpec>(n, p);
}

template <typename T>
helm_status solve_t(helm_ctx* ctx, const helm_grid* g, const void* m, double omega, int adjoint, int nrhs,
                    const void* q, void* u, const helm::SolveOpts& o, helm_solve_info* info, void* caller) {
  hipStream_t st = solve_stream(ctx, caller);
  const auto ps = shared_problems(g, m, omega, 0, nrhs);
  const bool pad = wants_pad(ps, sizeof(T) == 4);
  helm::Solver<T>& S = solver_for<T>(ctx, ps, o, st, pad);
  std::vector<helm::SolveInfo> inf(nrhs);
  int worst;
  if (!pad) {
    worst = S.solve(adjoint, (const helm::cx<T>*)q, (helm::cx<T>*)u, inf.data());
  } else {
    const helm::LevelSet& L0 = S.hierarchy().level(0);
    const int nz = g->n[2], pz = L0.host[0].pz;
    const size_t rows = (size_t)nrhs * g->n[0] * g->n[1];
    const size_t vb = (size_t)L0.total * sizeof(helm::cx<T>);
    ctx->batch_buf.ensure(2 * vb);
    helm::cx<T>* Q = ctx->batch_buf.as<helm::cx<T>>();
    helm::cx<T>* U = Q + L0.total;
    HELM_HIP_CHECK(hipMemsetAsync(Q, 0, 2 * vb, st));  // pads stay zero
    copy_rows<T>(Q, pz, q, nz, nz, rows, st);
    if (o.warm_start) copy_rows<T>(U, pz, u, nz, nz, rows, st);
    worst = S.solve(adjoint, Q, U, inf.data());
    copy_rows<T>(u, nz, U, pz, nz, rows, st);
    HELM_HIP_CHECK(hipStreamSynchronize(st));
  }
  if (info)
    for (int r = 0; r < nrhs; ++r) to_info(inf[r], info + r);
  return (helm_status)worst;
}

template <typename T>
helm_status solve_batched_t(helm_ctx* ctx, int nprob, const helm_problem* probs, int adjoint,
                            const helm::SolveOpts& o, helm_solve_info* info, void* caller) {
  using namespace helm;
  hipStream_t st = solve_stream(ctx, caller);
  std::vector<ProblemSpec> ps(nprob);
  int64_t total = 0;
  for (int i = 0; i < nprob; ++i) {
    std::memset(&ps[i], 0, sizeof(ProblemSpec));
    ps[i].g = spec_of(&probs[i].grid);
    ps[i].omega = probs[i].omega;
    ps[i].dir = 0;
    ps[i].m = probs[i].m;
    total += (int64_t)probs[i].grid.n[0] * probs[i].grid.n[1] * probs[i].grid.n[2];
  }
  const bool pad = wants_pad(ps, sizeof(T) == 4);
  Solver<T>& S = solver_for<T>(ctx, ps, o, st, pad);
  // gather the right-hand sides (and initial guesses) into the segment layout
  const auto& L0 = S.hierarchy().level(0);
  (void)total;
  ctx->batch_buf.ensure(2 * (size_t)L0.total * sizeof(cx<T>));
  cx<T>* Q = ctx->batch_buf.as<cx<T>>();
  cx<T>* U = Q + L0.total;
  if (pad) HELM_HIP_CHECK(hipMemsetAsync(Q, 0, 2 * (size_t)L0.total * sizeof(cx<T>), st));  // pads stay zero
  for (int i = 0; i < nprob; ++i) {
    const Seg& G = L0.host[i];
    const size_t rows = (size_t)G.n[0] * G.n[1];
    copy_rows<T>(Q + G.off, G.pz, probs[i].q, G.n[2], G.n[2], rows, st);
    if (o.warm_start) copy_rows<T>(U + G.off, G.pz, probs[i].u, G.n[2], G.n[2], rows, st);
  }
  std::vector<SolveInfo> inf(nprob);
  const int worst = S.solve(adjoint, Q, U, inf.data());
  for (int i = 0; i < nprob; ++i) {
    const Seg& G = L0.host[i];
    copy_rows<T>(probs[i].u, G.n[2], U + G.off, G.pz, G.n[2], (size_t)G.n[0] * G.n[1], st);
  }
  HELM_HIP_CHECK(hipStreamSynchronize(st));
  if (info)
    for (int i = 0; i < nprob; ++i) to_info(inf[i], info + i);
  return (helm_status)worst;
}

// Sources or receivers as weighted node lists (CSR over the points): point k
// is sum_e w[e] e_{lin[e]}, e in [ptr[k], ptr[k+1]).
struct PointSet {
  std::vector<int> ptr{0};
  std::vector<int64_t> lin;
  std::vector<double> w;
  int n() const { return (int)ptr.size() - 1; }
};

PointSet on_node_points(const helm_grid* g, int n, const int32_t* idx) {
  PointSet P;
  const int64_t plane = (int64_t)g->n[1] * g->n[2];
  for (int k = 0; k < n; ++k) {
    P.lin.push_back((int64_t)idx[3 * k] * plane + (int64_t)idx[3 * k + 1] * g->n[2] + idx[3 * k + 2]);
    P.w.push_back(1.0);
    P.ptr.push_back((int)P.lin.size());
  }
  return P;
}

// Modified Bessel function I0 by its power series sum_k ((x/2)^k / k!)^2.
double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double sum = 1.0, term = 1.0;
  for (int k = 1; k < 1000; ++k) {
    term *= q / ((double)k * (double)k);
    sum += term;
    if (term <= 1e-17 * sum) break;
  }
  return sum;
}

// sin(pi t) / (pi t), exactly zero at nonzero integers: sin(pi t) is taken
// as (-1)^n sin(pi (t - n)) with n the nearest integer.
double sinc_pi(double t) {
  if (t == 0.0) return 1.0;
  const double n = std::nearbyint(t);
  double sn = std::sin(M_PI * (t - n));
  if (std::fmod(n, 2.0) != 0.0) sn = -sn;
  return sn / (M_PI * t);
}

// Kaiser-windowed sinc interpolation (the paper's source and receiver
// operators, Software Design section): per axis, for position x in node
// units, w(i) = sinc(i - x) I0(b sqrt(1 - ((i - x)/r)^2)) / I0(b) over the 2r
// nodes floor(x) - r + 1 .. floor(x) + r inside the grid; the 3D weights
// are the tensor product.  Zero weights (all but one node of an on-node
// position) are left out.
PointSet sinc_points(const helm_grid* g, int n, const double* pos, int radius, double kb) {
  PointSet P;
  const double i0b = bessel_i0(kb);
  std::vector<int64_t> node[3];
  std::vector<double> wt[3];
  for (int k = 0; k < n; ++k) {
    for (int a = 0; a < 3; ++a) {
      node[a].clear();
      wt[a].clear();
      const double x = pos[3 * k + a];
      const int64_t base = (int64_t)std::floor(x);
      for (int64_t i = base - radius + 1; i <= base + radius; ++i) {
        if (i < 0 || i >= g->n[a]) continue;
        const double t = (double)i - x;
        const double u = t / radius;
        const double win = std::fabs(t) <= radius ? bessel_i0(kb * std::sqrt(std::max(0.0, 1.0 - u * u))) / i0b : 0.0;
        const double v = sinc_pi(t) * win;
        if (v != 0.0) {
          node[a].push_back(i);
          wt[a].push_back(v);
        }
      }
    }
    for (size_t ix = 0; ix < node[0].size(); ++ix)
      for (size_t iy = 0; iy < node[1].size(); ++iy)
        for (size_t iz = 0; iz < node[2].size(); ++iz) {
          P.lin.push_back((node[0][ix] * g->n[1] + node[1][iy]) * g->n[2] + node[2][iz]);
          P.w.push_back(wt[0][ix] * wt[1][iy] * wt[2][iz]);
        }
    P.ptr.push_back((int)P.lin.size());
  }
  return P;
}

// The selected (frequency, source) pairs of a misfit or derivative call:
// host tables, their device copies (in the context's small scratch) and the
// receiver node lists.  Pair p is row prow[p] = f * nsrc + s of the caller's
// [frequency][source] arrays; internal per-pair vectors are contiguous
// (offset p * N).
template <typename T>
struct Pairs {
  int np = 0, nall = 0, nsrc = 0, nrec = 0, nnode = 0, rblk = 0;
  int64_t N = 0;
  double scale = 1.0;  // 1 / #pairs with HELM_MG_RENORMALISE, else 1
  std::vector<int> prow;
  std::vector<helm::ProblemSpec> probs;
  int sblk = 1;  // entry blocks of the largest source
  // device tables
  int64_t *drow = nullptr, *uoff_int = nullptr, *uoff_store = nullptr, *node = nullptr,
          *ident = nullptr;  // ident[p] = p
  int *src_of_pair = nullptr, *sptr = nullptr, *rptr = nullptr;
  int64_t *slin = nullptr, *rlin = nullptr;
  double *sw = nullptr, *rw = nullptr, *node_w = nullptr;
  double2* amp = nullptr;
  double *w2 = nullptr, *wg = nullptr;  // omega^2; omega^2 * scale (model-space sums)
  helm::cx<T>* res = nullptr;           // [np][nrec] receiver values
  double* part = nullptr;               // [np][rblk] partial sums
  int *nptr = nullptr, *nrec_ord = nullptr;
};

template <typename T>
Pairs<T> plan_pairs(helm_ctx* ctx, const helm_grid* g, const void* m, int nfreq, const double* omega,
                    const PointSet& S, const double* src_amp, const uint8_t* mask, const PointSet& Rc,
                    bool renormalise, hipStream_t st) {
  using namespace helm;
  Pairs<T> P;
  const int nsrc = S.n(), nrec = Rc.n();
  P.N = (int64_t)g->n[0] * g->n[1] * g->n[2];
  P.nsrc = nsrc;
  P.nrec = nrec;
  P.nall = nfreq * nsrc;
  for (int k = 0; k < P.nall; ++k)
    if (!mask || mask[k]) P.prow.push_back(k);
  P.np = (int)P.prow.size();
  if (P.np == 0) return P;
  const int np = P.np;
  P.scale = renormalise ? 1.0 / np : 1.0;
  std::vector<int64_t> drow(np), uoff_int(np), uoff_store(np), ident(np);
  std::vector<int> src_of_pair(np);
  std::vector<double2> amp(np);
  std::vector<double> w2(np), wg(np);
  for (int p = 0; p < np; ++p) {
    const int fi = P.prow[p] / nsrc, s = P.prow[p] % nsrc;
    src_of_pair[p] = s;
    const double* a = src_amp ? src_amp + 2 * (size_t)P.prow[p] : nullptr;
    amp[p] = a ? make_double2(a[0], a[1]) : make_double2(1.0, 0.0);
    drow[p] = P.prow[p];
    uoff_int[p] = (int64_t)p * P.N;
    uoff_store[p] = (int64_t)P.prow[p] * P.N;
    ident[p] = p;
    w2[p] = omega[fi] * omega[fi];
    wg[p] = w2[p] * P.scale;
    P.probs.push_back(shared_problems(g, m, omega[fi], 0, 1)[0]);
  }
  int smax = 1;
  for (int k = 0; k < nsrc; ++k) smax = std::max(smax, S.ptr[k + 1] - S.ptr[k]);
  P.sblk = (int)ceil_div(smax, 256);
  // the nodes the receivers touch, ascending, each with its (receiver,
  // weight) entries in receiver order (a fixed summation order)
  const int nent = (int)Rc.lin.size();
  std::vector<int> ent(nent), ent_rec(nent);
  for (int k = 0; k < nrec; ++k)
    for (int e = Rc.ptr[k]; e < Rc.ptr[k + 1]; ++e) ent_rec[e] = k;
  for (int e = 0; e < nent; ++e) ent[e] = e;
  std::stable_sort(ent.begin(), ent.end(), [&](int x, int y) { return Rc.lin[x] < Rc.lin[y]; });
  std::vector<int64_t> node_lin;
  std::vector<int> node_ptr, node_rec(nent);
  std::vector<double> node_w(nent);
  for (int i = 0; i < nent; ++i) {
    const int e = ent[i];
    if (node_lin.empty() || node_lin.back() != Rc.lin[e]) {
      node_lin.push_back(Rc.lin[e]);
      node_ptr.push_back(i);
    }
    node_rec[i] = ent_rec[e];
    node_w[i] = Rc.w[e];
  }
  node_ptr.push_back(nent);
  P.nnode = (int)node_lin.size();
  P.rblk = (int)ceil_div(nrec, 256);
  const int nsent = (int)S.lin.size();
  auto r256 = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t small = 4 * r256(np * sizeof(int64_t)) + r256(np * sizeof(int)) + r256(np * sizeof(double2)) +
                       2 * r256(np * sizeof(double)) + r256((nsrc + 1) * sizeof(int)) +
                       r256(nsent * sizeof(int64_t)) + r256(nsent * sizeof(double)) +
                       r256((nrec + 1) * sizeof(int)) + r256(nent * sizeof(int64_t)) + r256(nent * sizeof(double)) +
                       r256((size_t)np * nrec * sizeof(cx<T>)) + r256((size_t)np * P.rblk * sizeof(double)) +
                       r256(P.nnode * sizeof(int64_t)) + r256((P.nnode + 1) * sizeof(int)) +
                       r256(nent * sizeof(int)) + r256(nent * sizeof(double));
  ctx->fwi_small.ensure(small);
  char* sp = (char*)ctx->fwi_small.p;
  char* const sp_end = sp + small;
  auto carve = [&](size_t b) {
    char* q = sp;
    sp += r256(b);
    if (sp > sp_end) throw Error{-3, "internal: misfit scratch layout overflow"};
    return (void*)q;
  };
  P.drow = (int64_t*)carve(np * sizeof(int64_t));
  P.uoff_int = (int64_t*)carve(np * sizeof(int64_t));
  P.uoff_store = (int64_t*)carve(np * sizeof(int64_t));
  P.ident = (int64_t*)carve(np * sizeof(int64_t));
  P.src_of_pair = (int*)carve(np * sizeof(int));
  P.amp = (double2*)carve(np * sizeof(double2));
  P.w2 = (double*)carve(np * sizeof(double));
  P.wg = (double*)carve(np * sizeof(double));
  P.sptr = (int*)carve((nsrc + 1) * sizeof(int));
  P.slin = (int64_t*)carve(nsent * sizeof(int64_t));
  P.sw = (double*)carve(nsent * sizeof(double));
  P.rptr = (int*)carve((nrec + 1) * sizeof(int));
  P.rlin = (int64_t*)carve(nent * sizeof(int64_t));
  P.rw = (double*)carve(nent * sizeof(double));
  P.res = (cx<T>*)carve((size_t)np * nrec * sizeof(cx<T>));
  P.part = (double*)carve((size_t)np * P.rblk * sizeof(double));
  P.node = (int64_t*)carve(P.nnode * sizeof(int64_t));
  P.nptr = (int*)carve((P.nnode + 1) * sizeof(int));
  P.nrec_ord = (int*)carve(nent * sizeof(int));
  P.node_w = (double*)carve(nent * sizeof(double));
  auto up = [&](void* dst, const void* src, size_t b) {
    if (b) HELM_HIP_CHECK(hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, st));
  };
  up(P.drow, drow.data(), np * sizeof(int64_t));
  up(P.uoff_int, uoff_int.data(), np * sizeof(int64_t));
  up(P.uoff_store, uoff_store.data(), np * sizeof(int64_t));
  up(P.ident, ident.data(), np * sizeof(int64_t));
  up(P.src_of_pair, src_of_pair.data(), np * sizeof(int));
  up(P.amp, amp.data(), np * sizeof(double2));
  up(P.w2, w2.data(), np * sizeof(double));
  up(P.wg, wg.data(), np * sizeof(double));
  up(P.sptr, S.ptr.data(), (nsrc + 1) * sizeof(int));
  up(P.slin, S.lin.data(), nsent * sizeof(int64_t));
  up(P.sw, S.w.data(), nsent * sizeof(double));
  up(P.rptr, Rc.ptr.data(), (nrec + 1) * sizeof(int));
  up(P.rlin, Rc.lin.data(), nent * sizeof(int64_t));
  up(P.rw, Rc.w.data(), nent * sizeof(double));
  up(P.node, node_lin.data(), P.nnode * sizeof(int64_t));
  up(P.nptr, node_ptr.data(), (P.nnode + 1) * sizeof(int));
  up(P.nrec_ord, node_rec.data(), nent * sizeof(int));
  up(P.node_w, node_w.data(), nent * sizeof(double));
  // the host vectors above go out of scope: the copies must have completed
  HELM_HIP_CHECK(hipStreamSynchronize(st));
  return P;
}

// Where kernels read per-pair fields: base pointer, per-pair element
// offsets (device), FP64 or the dtype.
struct FieldRef {
  const void* p;
  const int64_t* off;
  bool f64;
};

// The 27-point mass weights (centre, face, edge, corner); identity for 7-point.
inline void mass_weights(const helm_grid* g, double mw[4]) {
  const bool m27 = g->stencil == HELM_27PT;
  mw[0] = m27 ? g->w27[3] : 1.0;
  mw[1] = m27 ? g->w27[4] : 0.0;
  mw[2] = m27 ? g->w27[5] : 0.0;
  mw[3] = m27 ? g->w27[6] : 0.0;
}

// g (+)= sum_p Re(wg_p conj(u_p) (A v_p)) over the pairs (v contiguous per pair)
template <typename T>
void launch_gradient(const helm_grid* g, const Pairs<T>& P, const FieldRef& u, const helm::cx<T>* v, void* grad,
                     bool acc, hipStream_t st) {
  using namespace helm;
  const unsigned gb = std::min<unsigned>(4096, ceil_div(P.N, 256));
  double mw[4];
  mass_weights(g, mw);
  const bool m27 = g->stencil == HELM_27PT;
#define HELM_GRAD(TU, M27)                                                                                    \
  hipLaunchKernelGGL((k_gradient<TU, T, T, M27>), dim3(gb), dim3(256), 0, st, (const cx<TU>*)u.p, u.off, v,   \
                     P.np, g->n[0], g->n[1], g->n[2], (const double*)P.wg, mw[0], mw[1], mw[2], mw[3], (T*)grad, \
                     acc)
  if (u.f64) {
    if (m27) HELM_GRAD(double, true);
    else HELM_GRAD(double, false);
  } else {
    if (m27) HELM_GRAD(T, true);
    else HELM_GRAD(T, false);
  }
#undef HELM_GRAD
  HELM_HIP_CHECK(hipGetLastError());
}

// out_p = -omega_p^2 A (x_p * dm)  (DHADJ false)  or  -omega_p^2 dm * (A x_p)  (DHADJ true)
template <typename T, bool DHADJ>
void launch_born_source(const helm_grid* g, const Pairs<T>& P, const FieldRef& x, const void* dm, helm::cx<T>* out,
                        hipStream_t st) {
  using namespace helm;
  const dim3 grid(std::min<unsigned>(DOT_BLOCKS, ceil_div(P.N, 256)), P.np);
  double mw[4];
  mass_weights(g, mw);
  const bool m27 = g->stencil == HELM_27PT;
#define HELM_BORN(TX, M27)                                                                                     \
  hipLaunchKernelGGL((k_born_source<TX, T, M27, DHADJ>), grid, dim3(256), 0, st, (const cx<TX>*)x.p, x.off,    \
                     (const T*)dm, P.np, g->n[0], g->n[1], g->n[2], (const double*)P.w2, mw[0], mw[1], mw[2],   \
                     mw[3], out)
  if (x.f64) {
    if (m27) HELM_BORN(double, true);
    else HELM_BORN(double, false);
  } else {
    if (m27) HELM_BORN(T, true);
    else HELM_BORN(T, false);
  }
#undef HELM_BORN
  HELM_HIP_CHECK(hipGetLastError());
}

// b_p (+)= -P_r^T res[rrow_p] (b zeroed first unless add)
template <typename T>
void launch_adjoint_source(const Pairs<T>& P, helm::cx<T>* b, const helm::cx<T>* res, const int64_t* rrow,
                           bool add, hipStream_t st) {
  using namespace helm;
  if (!add)
    hipLaunchKernelGGL((k_fill_zero<T>), dim3(std::min<unsigned>(65536, ceil_div((int64_t)P.np * P.N, 256))),
                       dim3(256), 0, st, b, (int64_t)P.np * P.N);
  if (add)
    hipLaunchKernelGGL((k_adjoint_source<T, true>), dim3(ceil_div(P.nnode, 256), P.np), dim3(256), 0, st, b, P.N,
                       (const int64_t*)P.node, (const int*)P.nptr, (const int*)P.nrec_ord, (const double*)P.node_w,
                       P.nnode, res, P.nrec, rrow);
  else
    hipLaunchKernelGGL((k_adjoint_source<T, false>), dim3(ceil_div(P.nnode, 256), P.np), dim3(256), 0, st, b, P.N,
                       (const int64_t*)P.node, (const int*)P.nptr, (const int*)P.nrec_ord, (const double*)P.node_w,
                       P.nnode, res, P.nrec, rrow);
  HELM_HIP_CHECK(hipGetLastError());
}

// Forward fields of the selected pairs: solved from the point sources into U
// (and copied into u_store when given; its FP64 iterates with u64), or taken
// from u_store with reuse.  Returns where the solve's FP64 iterates
// (fwd_fp64, valid until the next solve; null with reuse) and the stored /
// working fields are.
template <typename T>
FieldRef forward_fields(const helm_grid* g, const Pairs<T>& P, helm::Solver<T>& S, helm::cx<T>* Q, helm::cx<T>* U,
                        void* u_store, bool reuse, bool u64, std::vector<helm::SolveInfo>& inf,
                        helm_solve_info* info, int& worst, const helm::cx<double>** fwd_fp64, hipStream_t st) {
  using namespace helm;
  const int64_t N = P.N;
  *fwd_fp64 = nullptr;
  if (reuse) return FieldRef{u_store, P.uoff_store, u64};
  // the discrete delta: 1/h^3, or 1/h^2 on a 2D grid (n[0] = 1)
  const double inv_h3 = g->n[0] == 1 ? 1.0 / (g->h * g->h) : 1.0 / (g->h * g->h * g->h);
  hipLaunchKernelGGL((k_fill_zero<T>), dim3(std::min<unsigned>(65536, ceil_div((int64_t)P.np * N, 256))), dim3(256), 0,
                     st, Q, (int64_t)P.np * N);
  hipLaunchKernelGGL((k_point_sources<T>), dim3(P.sblk, P.np), dim3(256), 0, st, Q, N, (const int*)P.src_of_pair,
                     (const int*)P.sptr, (const int64_t*)P.slin, (const double*)P.sw, (const double2*)P.amp, inv_h3);
  worst = std::max(worst, S.solve(0, Q, U, inf.data()));
  if (info)
    for (int p = 0; p < P.np; ++p) to_info(inf[p], info + P.prow[p]);
  *fwd_fp64 = S.iterate();
  if (u64) {  // keep the FP64 iterates as the stored fields
    const unsigned pb = std::min<unsigned>(65536, ceil_div(N, 256));
    for (int p = 0; p < P.np; ++p)
      hipLaunchKernelGGL((k_convert<double, double>), dim3(pb), dim3(256), 0, st, S.iterate() + p * N,
                         (cx<double>*)u_store + P.prow[p] * N, N);
    return FieldRef{u_store, P.uoff_store, true};
  }
  if (u_store && (cx<T>*)u_store != U)
    for (int p = 0; p < P.np; ++p)
      HELM_HIP_CHECK(hipMemcpyAsync((cx<T>*)u_store + P.prow[p] * N, U + p * N, N * sizeof(cx<T>),
                                    hipMemcpyDeviceToDevice, st));
  return FieldRef{U, P.uoff_int, false};
}

// sum of the partial sums |r|^2 written by k_sample_residual
template <typename T>
double residual_norm2(const Pairs<T>& P, hipStream_t st) {
  std::vector<double> hpart((size_t)P.np * P.rblk);
  HELM_HIP_CHECK(hipMemcpyAsync(hpart.data(), P.part, hpart.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HELM_HIP_CHECK(hipStreamSynchronize(st));
  double fsum = 0.0;
  for (size_t i = 0; i < hpart.size(); ++i) fsum += hpart[i];
  return fsum;
}

// r_p = P_r u_p - d_p from the forward solve's FP64 iterate, or from the
// given fields (reuse)
template <typename T>
void launch_residual(const Pairs<T>& P, const helm::cx<double>* fwd_fp64, const FieldRef& u, const void* d,
                     hipStream_t st) {
  using namespace helm;
  const dim3 grid(P.rblk, P.np);
  if (fwd_fp64)
    hipLaunchKernelGGL((k_sample_residual<double, T>), grid, dim3(256), 0, st, fwd_fp64, (const int64_t*)P.uoff_int,
                       (const int*)P.rptr, (const int64_t*)P.rlin, (const double*)P.rw, P.nrec, (const cx<T>*)d,
                       (const int64_t*)P.drow, P.res, P.part);
  else if (u.f64)
    hipLaunchKernelGGL((k_sample_residual<double, T>), grid, dim3(256), 0, st, (const cx<double>*)u.p, u.off,
                       (const int*)P.rptr, (const int64_t*)P.rlin, (const double*)P.rw, P.nrec, (const cx<T>*)d,
                       (const int64_t*)P.drow, P.res, P.part);
  else
    hipLaunchKernelGGL((k_sample_residual<T, T>), grid, dim3(256), 0, st, (const cx<T>*)u.p, u.off,
                       (const int*)P.rptr, (const int64_t*)P.rlin, (const double*)P.rw, P.nrec, (const cx<T>*)d,
                       (const int64_t*)P.drow, P.res, P.part);
  HELM_HIP_CHECK(hipGetLastError());
}

// misfit + gradient over the selected (frequency, source) pairs, element type T
template <typename T>
helm_status misfit_gradient_t(helm_ctx* ctx, const helm_grid* g, const void* m, int nfreq, const double* omega,
                              const PointSet& src, const double* src_amp, const uint8_t* mask, const PointSet& rec,
                              const void* d, double* f, void* grad,
                              void* u_store, int flags, const helm::SolveOpts& o, helm_solve_info* info,
                              void* caller) {
  using namespace helm;
  hipStream_t st = solve_stream(ctx, caller);
  const bool fwd_only = (flags & HELM_MG_FORWARD_ONLY) != 0;
  const bool reuse = (flags & HELM_MG_REUSE_U) != 0;
  const bool acc = (flags & HELM_MG_ACCUMULATE) != 0;
  const bool u64 = (flags & HELM_MG_U_FP64) != 0 && sizeof(T) == 4;
  if (info)
    for (int k = 0; k < 2 * nfreq * src.n(); ++k) to_info(SolveInfo(), info + k);
  Pairs<T> P = plan_pairs<T>(ctx, g, m, nfreq, omega, src, src_amp, mask, rec, (flags & HELM_MG_RENORMALISE) != 0,
                             st);
  const int64_t N = P.N;
  if (P.np == 0) {
    *f = 0.0;
    if (!fwd_only && !acc) HELM_HIP_CHECK(hipMemsetAsync(grad, 0, (size_t)N * sizeof(T), st));
    HELM_HIP_CHECK(hipStreamSynchronize(st));
    return HELM_OK;
  }
  const int np = P.np;
  // Device scratch: Q (sources, then adjoint sources), V, and U unless the
  // solve writes the caller's u_store directly (every pair selected, fields
  // stored in the dtype).
  const size_t fbytes = (size_t)np * N * sizeof(cx<T>);
  const bool direct_u = u_store && !u64 && np == P.nall;
  const bool own_u = !reuse && !direct_u;
  ctx->fwi_buf.ensure(fbytes * (own_u ? 3 : 2));
  char* base = (char*)ctx->fwi_buf.p;
  cx<T>* Q = (cx<T>*)base;
  cx<T>* V = (cx<T>*)(base + fbytes);
  cx<T>* U = direct_u ? (cx<T>*)u_store : own_u ? (cx<T>*)(base + 2 * fbytes) : nullptr;

  Solver<T>& S = solver_for<T>(ctx, P.probs, o, st);
  std::vector<SolveInfo> inf(np);
  int worst = 0;
  const cx<double>* fwd64 = nullptr;
  const FieldRef uf = forward_fields<T>(g, P, S, Q, U, u_store, reuse, u64, inf, info, worst, &fwd64, st);
  launch_residual<T>(P, fwd64, uf, d, st);
  *f = 0.5 * residual_norm2<T>(P, st) * P.scale;
  if (fwd_only) return (helm_status)worst;
  // adjoint sources b_p = -P_r^T r_p, then H^H v_p = b_p
  launch_adjoint_source<T>(P, Q, P.res, nullptr, false, st);
  worst = std::max(worst, S.solve(1, Q, V, inf.data()));
  if (info)
    for (int p = 0; p < np; ++p) to_info(inf[p], info + P.nall + P.prow[p]);
  launch_gradient<T>(g, P, uf, V, grad, acc, st);
  HELM_HIP_CHECK(hipStreamSynchronize(st));
  return (helm_status)worst;
}

// Linearised products over the selected (frequency, source) pairs (the
// PDEfunc modes JACOB_FORW, JACOB_ADJ, HESS_GN, HESS), element type T.
// Solves of pair p, in order, with their info rows (k * nall + row):
//   forward fields u (k = 0; absent with REUSE_U), then
//   JACOB_FORW: du = -H^{-1} T dm (1);            out = P_r du
//   JACOB_ADJ:  v  = -H^{-H} P_r^T y (1);          out = sum Re(T^* v)
//   HESS_GN:    du (1), w = -H^{-H} P_r^T P_r du (2); out = sum Re(T^* w)
//   HESS:       v = -H^{-H} P_r^T r (1), du (2),
//               dv = H^{-H}(-omega^2 dm (A v) - P_r^T P_r du) (3);
//               out = sum Re(omega^2 conj(du) (A v)) + Re(T^* dv)
template <typename T>
helm_status derivative_t(helm_ctx* ctx, int mode, const helm_grid* g, const void* m, int nfreq, const double* omega,
                         const PointSet& src, const double* src_amp, const uint8_t* mask, const PointSet& rec,
                         const void* in, const void* d, void* out, void* u_store, int flags, const helm::SolveOpts& o,
                         helm_solve_info* info, void* caller) {
  using namespace helm;
  hipStream_t st = solve_stream(ctx, caller);
  const bool reuse = (flags & HELM_MG_REUSE_U) != 0;
  const bool acc = (flags & HELM_MG_ACCUMULATE) != 0;
  const bool u64 = (flags & HELM_MG_U_FP64) != 0 && sizeof(T) == 4;
  const int nall = nfreq * src.n(), nrec = rec.n();
  if (info)
    for (int k = 0; k < 4 * nall; ++k) to_info(SolveInfo(), info + k);
  Pairs<T> P = plan_pairs<T>(ctx, g, m, nfreq, omega, src, src_amp, mask, rec, (flags & HELM_MG_RENORMALISE) != 0,
                             st);
  const int64_t N = P.N;
  const int np = P.np;
  if (mode == HELM_JACOB_FORW)  // rows of unselected pairs are zero
    hipLaunchKernelGGL((k_fill_zero<T>), dim3(std::min<unsigned>(65536, ceil_div((int64_t)nall * nrec, 256))),
                       dim3(256), 0, st, (cx<T>*)out, (int64_t)nall * nrec);
  else if (!acc)
    hipLaunchKernelGGL((k_fill_zero_real<T>), dim3(std::min<unsigned>(65536, ceil_div(N, 256))), dim3(256), 0, st,
                       (T*)out, N);
  HELM_HIP_CHECK(hipGetLastError());
  if (np == 0) {
    HELM_HIP_CHECK(hipStreamSynchronize(st));
    return HELM_OK;
  }
  // work vectors: Q (right-hand sides), U (forward fields unless reused),
  // B1, B2, B3 (the linearised fields)
  const size_t fbytes = (size_t)np * N * sizeof(cx<T>);
  const int nwork = mode == HELM_HESS ? 4 : mode == HELM_HESS_GN ? 3 : 2;
  ctx->fwi_buf.ensure(fbytes * (nwork + (reuse ? 0 : 1)));
  char* base = (char*)ctx->fwi_buf.p;
  cx<T>* Q = (cx<T>*)base;
  cx<T>* B[3] = {(cx<T>*)(base + fbytes), nwork > 2 ? (cx<T>*)(base + 2 * fbytes) : nullptr,
                 nwork > 3 ? (cx<T>*)(base + 3 * fbytes) : nullptr};
  cx<T>* U = reuse ? nullptr : (cx<T>*)(base + (size_t)nwork * fbytes);

  Solver<T>& S = solver_for<T>(ctx, P.probs, o, st);
  std::vector<SolveInfo> inf(np);
  int worst = 0, k = 1;
  auto solve = [&](int dir, cx<T>* rhs, cx<T>* x) {
    worst = std::max(worst, S.solve(dir, rhs, x, inf.data()));
    if (info)
      for (int p = 0; p < np; ++p) to_info(inf[p], info + (size_t)k * nall + P.prow[p]);
    ++k;
  };
  const cx<double>* fwd64 = nullptr;
  const FieldRef uf = forward_fields<T>(g, P, S, Q, U, u_store, reuse, u64, inf, info, worst, &fwd64, st);
  const FieldRef b0{B[0], P.uoff_int, false};
  const dim3 sgrid(P.rblk, np);
  if (mode == HELM_JACOB_FORW || mode == HELM_HESS_GN) {
    launch_born_source<T, false>(g, P, uf, in, Q, st);  // -T dm
    solve(0, Q, B[0]);                                  // du
    if (mode == HELM_JACOB_FORW) {
      hipLaunchKernelGGL((k_sample<double, T>), sgrid, dim3(256), 0, st, S.iterate(), (const int64_t*)P.uoff_int,
                         (const int*)P.rptr, (const int64_t*)P.rlin, (const double*)P.rw, nrec, (cx<T>*)out,
                         (const int64_t*)P.drow);
    } else {
      hipLaunchKernelGGL((k_sample<double, T>), sgrid, dim3(256), 0, st, S.iterate(), (const int64_t*)P.uoff_int,
                         (const int*)P.rptr, (const int64_t*)P.rlin, (const double*)P.rw, nrec, P.res,
                         (const int64_t*)P.ident);
      HELM_HIP_CHECK(hipGetLastError());
      launch_adjoint_source<T>(P, Q, P.res, nullptr, false, st);  // -P_r^T P_r du
      solve(1, Q, B[1]);                                            // w
      launch_gradient<T>(g, P, uf, B[1], out, true, st);
    }
  } else if (mode == HELM_JACOB_ADJ) {
    launch_adjoint_source<T>(P, Q, (const cx<T>*)in, P.drow, false, st);  // -P_r^T y
    solve(1, Q, B[0]);                                                    // v
    launch_gradient<T>(g, P, uf, B[0], out, true, st);
  } else {  // HESS
    launch_residual<T>(P, fwd64, uf, d, st);                 // r
    launch_adjoint_source<T>(P, Q, P.res, nullptr, false, st);
    solve(1, Q, B[0]);                                         // v
    launch_born_source<T, false>(g, P, uf, in, Q, st);         // -T dm
    solve(0, Q, B[1]);                                         // du
    hipLaunchKernelGGL((k_sample<double, T>), sgrid, dim3(256), 0, st, S.iterate(), (const int64_t*)P.uoff_int,
                       (const int*)P.rptr, (const int64_t*)P.rlin, (const double*)P.rw, nrec, P.res,
                         (const int64_t*)P.ident);
    HELM_HIP_CHECK(hipGetLastError());
    launch_born_source<T, true>(g, P, b0, in, Q, st);          // -omega^2 dm (A v)
    launch_adjoint_source<T>(P, Q, P.res, nullptr, true, st);  // - P_r^T P_r du
    solve(1, Q, B[2]);                                         // dv
    launch_gradient<T>(g, P, FieldRef{B[1], P.uoff_int, false}, B[0], out, true, st);
    launch_gradient<T>(g, P, uf, B[2], out, true, st);
  }
  HELM_HIP_CHECK(hipGetLastError());
  HELM_HIP_CHECK(hipStreamSynchronize(st));
  return (helm_status)worst;
}

// Argument checks shared by the misfit and derivative entry points.
// WRI objective and gradient over the selected (frequency, source) pairs
// (Penalty Method subsection, eqs. wri and wrifieldeq; Appendix B):
//   u  = argmin 1/2 ||P_r u - d||^2 + lambda^2/2 ||H u - q||^2
//      = u0 + H^{-1} H^{-H} P_r^T y,  u0 = H^{-1} q,
//        (P_r H^{-1} H^{-H} P_r^T + lambda^2 I) y = d - P_r u0   (CG, per pair)
//   f  = c sum (1/2 ||P_r u - d||^2 + lambda^2/2 ||H u - q||^2)
//   g  = c sum lambda^2 Re(omega^2 conj(u) (A^H (H u - q)))
// Per CG step every active pair costs one adjoint and one forward solve,
// batched over the pairs; converged pairs get a zero right-hand side (their
// solves drop out at once).  The field is accumulated in FP64 from the
// solves' FP64 outer iterates, and H u - q is formed in FP64.
template <typename T>
helm_status wri_t(helm_ctx* ctx, const helm_grid* g, const void* m, int nfreq, const double* omega,
                  const PointSet& src, const double* src_amp, const uint8_t* mask, const PointSet& rec,
                  const void* d, double lam, double cg_tol, int cg_max, double* f, void* grad, void* u_store,
                  int flags, const helm::SolveOpts& o, helm_solve_info* info, void* caller) {
  using namespace helm;
  hipStream_t st = solve_stream(ctx, caller);
  const bool fwd_only = (flags & HELM_MG_FORWARD_ONLY) != 0;
  const bool acc = (flags & HELM_MG_ACCUMULATE) != 0;
  const bool u64 = (flags & HELM_MG_U_FP64) != 0;
  const int nall = nfreq * src.n();
  if (info)
    for (int k = 0; k < nall; ++k) to_info(SolveInfo(), info + k);
  Pairs<T> P = plan_pairs<T>(ctx, g, m, nfreq, omega, src, src_amp, mask, rec, (flags & HELM_MG_RENORMALISE) != 0,
                             st);
  const int64_t N = P.N;
  if (P.np == 0) {
    *f = 0.0;
    if (!fwd_only && !acc) HELM_HIP_CHECK(hipMemsetAsync(grad, 0, (size_t)N * sizeof(T), st));
    HELM_HIP_CHECK(hipStreamSynchronize(st));
    return HELM_OK;
  }
  const int np = P.np, nrec = P.nrec, rblk = P.rblk;
  const double lam2 = lam * lam;
  auto r256 = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t fb = r256((size_t)np * N * sizeof(cx<T>)), ub = r256((size_t)np * N * sizeof(cx<double>));
  const size_t rb = r256((size_t)np * nrec * sizeof(cx<double>)), pb = r256((size_t)np * rblk * sizeof(double));
  const size_t sb = r256((size_t)np * sizeof(double));
  ctx->fwi_buf.ensure(3 * fb + ub + 3 * rb + pb + 2 * sb);
  char* base = (char*)ctx->fwi_buf.p;
  cx<T>* Q = (cx<T>*)base;
  cx<T>* B = (cx<T>*)(base + fb);
  cx<T>* W = (cx<T>*)(base + 2 * fb);
  cx<double>* U = (cx<double>*)(base + 3 * fb);
  char* rbase = base + 3 * fb + ub;
  cx<double>* rho = (cx<double>*)rbase;
  cx<double>* pv = (cx<double>*)(rbase + rb);
  cx<double>* ap = (cx<double>*)(rbase + 2 * rb);
  double* part = (double*)(rbase + 3 * rb);
  double* alpha_d = (double*)(rbase + 3 * rb + pb);
  double* beta_d = (double*)(rbase + 3 * rb + pb + sb);

  Solver<T>& S = solver_for<T>(ctx, P.probs, o, st);
  std::vector<SolveInfo> inf(np);
  int worst = 0;
  const cx<double>* fwd64 = nullptr;
  forward_fields<T>(g, P, S, Q, W, nullptr, false, false, inf, nullptr, worst, &fwd64, st);
  HELM_HIP_CHECK(hipMemcpyAsync(U, fwd64, (size_t)np * N * sizeof(cx<double>), hipMemcpyDeviceToDevice, st));
  // Q still holds the sources (forward_fields solved into W)
  std::vector<double> hp((size_t)np * rblk);
  auto pair_sums = [&]() {
    HELM_HIP_CHECK(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HELM_HIP_CHECK(hipStreamSynchronize(st));
    std::vector<double> out(np, 0.0);
    for (int p = 0; p < np; ++p)
      for (int b = 0; b < rblk; ++b) out[p] += hp[(size_t)p * rblk + b];
    return out;
  };
  const dim3 rgrid(rblk, np);
  hipLaunchKernelGGL((k_wri_start<T>), rgrid, dim3(256), 0, st, (const cx<double>*)U, (const int64_t*)P.uoff_int,
                     (const int*)P.rptr, (const int64_t*)P.rlin, (const double*)P.rw, nrec, (const cx<T>*)d,
                     (const int64_t*)P.drow, rho, pv, part);
  HELM_HIP_CHECK(hipGetLastError());
  const std::vector<double> rr0 = pair_sums();
  std::vector<double> rr = rr0, alpha(np), beta(np), rel(np, 0.0);
  std::vector<int> active(np), iters(np, 0), solves(np, 1), cg_status(np, 0);
  for (int p = 0; p < np; ++p) {
    active[p] = rr0[p] > 0.0 && std::isfinite(rr0[p]);
    if (!std::isfinite(rr0[p])) cg_status[p] = 2;
  }
  const unsigned fblk = std::min<unsigned>(1024, ceil_div(N, 256));
  for (int it = 0; it < cg_max; ++it) {
    const Range rcg("helm wri CG step");
    int n_active = 0;
    for (int p = 0; p < np; ++p) n_active += active[p];
    if (n_active == 0) break;
    // z = H^{-1} H^{-H} P_r^T p
    hipLaunchKernelGGL((k_fill_zero<T>), dim3(std::min<unsigned>(65536, ceil_div((int64_t)np * N, 256))), dim3(256),
                       0, st, B, (int64_t)np * N);
    hipLaunchKernelGGL((k_wri_spread<T>), dim3(ceil_div(P.nnode, 256), np), dim3(256), 0, st, B, N,
                       (const int64_t*)P.node, (const int*)P.nptr, (const int*)P.nrec_ord, (const double*)P.node_w,
                       P.nnode, (const cx<double>*)pv, nrec);
    HELM_HIP_CHECK(hipGetLastError());
    worst = std::max(worst, S.solve(1, B, W, inf.data()));
    worst = std::max(worst, S.solve(0, W, B, inf.data()));
    const cx<double>* z = S.iterate();
    hipLaunchKernelGGL(k_wri_apply, rgrid, dim3(256), 0, st, z, N, (const int*)P.rptr, (const int64_t*)P.rlin,
                       (const double*)P.rw, nrec, lam2, (const cx<double>*)pv, ap, part);
    HELM_HIP_CHECK(hipGetLastError());
    const std::vector<double> pap = pair_sums();
    for (int p = 0; p < np; ++p) {
      alpha[p] = 0.0;
      if (!active[p]) continue;
      if (!(pap[p] > 0.0) || !std::isfinite(pap[p])) {  // breakdown: keep the field so far
        active[p] = 0;
        cg_status[p] = 2;
        continue;
      }
      alpha[p] = rr[p] / pap[p];
    }
    HELM_HIP_CHECK(hipMemcpyAsync(alpha_d, alpha.data(), np * sizeof(double), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_wri_field, dim3(fblk, np), dim3(256), 0, st, U, z, (const double*)alpha_d, N);
    hipLaunchKernelGGL(k_wri_residual, rgrid, dim3(256), 0, st, rho, (const cx<double>*)ap, (const double*)alpha_d,
                       nrec, part);
    HELM_HIP_CHECK(hipGetLastError());
    const std::vector<double> rrn = pair_sums();
    for (int p = 0; p < np; ++p) {
      beta[p] = -1.0;
      if (!active[p]) continue;
      iters[p] += 1;
      solves[p] += 2;
      rel[p] = std::sqrt(rrn[p] / rr0[p]);
      if (rel[p] <= cg_tol) {
        active[p] = 0;
      } else {
        beta[p] = rrn[p] / rr[p];
        rr[p] = rrn[p];
      }
    }
    HELM_HIP_CHECK(hipMemcpyAsync(beta_d, beta.data(), np * sizeof(double), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_wri_direction, rgrid, dim3(256), 0, st, pv, (const cx<double>*)rho, (const double*)beta_d,
                       nrec);
    HELM_HIP_CHECK(hipGetLastError());
  }
  for (int p = 0; p < np; ++p)
    if (active[p]) cg_status[p] = std::max(cg_status[p], 1);  // iteration limit reached
  // objective: data term from the FP64 field, penalty term ||q - H u|| in FP64
  launch_residual<T>(P, U, FieldRef{U, P.uoff_int, true}, d, st);
  const double f_data = 0.5 * residual_norm2<T>(P, st);
  const std::vector<double> en = S.residual(0, U, Q, W);  // W = q - H u (rounded)
  double f_pen = 0.0;
  for (int p = 0; p < np; ++p) f_pen += en[p] * en[p];
  *f = (f_data + 0.5 * lam2 * f_pen) * P.scale;
  if (u_store) {
    const unsigned pbk = std::min<unsigned>(65536, ceil_div(N, 256));
    for (int p = 0; p < np; ++p) {
      if (u64)
        HELM_HIP_CHECK(hipMemcpyAsync((cx<double>*)u_store + P.prow[p] * N, U + (int64_t)p * N,
                                      N * sizeof(cx<double>), hipMemcpyDeviceToDevice, st));
      else
        hipLaunchKernelGGL((k_convert<T, double>), dim3(pbk), dim3(256), 0, st, (const cx<double>*)(U + p * N),
                           (cx<T>*)u_store + P.prow[p] * N, N);
    }
  }
  if (!fwd_only) {
    // g = c lambda^2 sum Re(omega^2 conj(u) A (H u - q)) = -c lambda^2 sum Re(omega^2 conj(u) A W)
    std::vector<double> wg(np);
    for (int p = 0; p < np; ++p) {
      const double om = omega[P.prow[p] / P.nsrc];
      wg[p] = -lam2 * om * om * P.scale;
    }
    HELM_HIP_CHECK(hipMemcpyAsync(P.wg, wg.data(), np * sizeof(double), hipMemcpyHostToDevice, st));
    launch_gradient<T>(g, P, FieldRef{U, P.uoff_int, true}, W, grad, acc, st);
  }
  HELM_HIP_CHECK(hipStreamSynchronize(st));
  for (int p = 0; p < np; ++p) {
    worst = std::max(worst, cg_status[p]);
    if (info) {
      helm_solve_info& r = info[P.prow[p]];
      r.status = cg_status[p];
      r.cycles = iters[p];
      r.inner_its = 0;
      r.pad_ = 0;
      r.matvecs = solves[p];
      r.relres_fp64 = rel[p];
    }
  }
  return (helm_status)worst;
}

// Gauss-Legendre nodes (ascending) and weights on [0, K]: Newton's method on
// the Legendre polynomial of degree n, evaluated by its three-term
// recurrence, from the starting guesses cos(pi (i + 3/4) / (n + 1/2)).
void gauss_legendre(int n, double K, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;  // P_{k-1}, P_k
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) p0 = 1.0;
      dp = n * (t * p1 - p0) / (t * t - 1.0);  // P_n'(t)
      const double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) <= 1e-16) break;
    }
    double p0 = 1.0, p1 = t;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) p0 = 1.0;
    dp = n * (t * p1 - p0) / (t * t - 1.0);
    x[n - 1 - i] = 0.5 * K * (t + 1.0);
    w[n - 1 - i] = K / ((1.0 - t * t) * dp * dp);
  }
}

// 2.5D modelling, misfit and gradient (the 2.5D subsection) on a 2D grid
// (n[0] = 1): every selected (frequency, source) row contributes nky 2D
// problems, one per Gauss-Legendre node k_i of [0, min(p_kc omega / v_min,
// pi / h)], with model m - k_i^2 / omega^2; all rows x nodes are solved in
// one batched solve per direction.  Receiver r of row (f, s) reads
// sum_i (w_i / pi) cos(k_i (y_r - y_s)) u~_{f,s,i}(node_r).
template <typename T>
helm_status model25d_t(helm_ctx* ctx, const helm_grid* g, const void* m, int nfreq, const double* omega, int nky,
                       double p_kc, double v_min, const PointSet& src, const double* src_y, const double* src_amp,
                       const uint8_t* mask, const PointSet& rec, const double* rec_y, const void* d, double* f,
                       void* grad, void* d_pred, int flags, const helm::SolveOpts& o, helm_solve_info* info,
                       void* caller) {
  using namespace helm;
  hipStream_t st = solve_stream(ctx, caller);
  const bool fwd_only = (flags & HELM_MG_FORWARD_ONLY) != 0;
  const bool acc = (flags & HELM_MG_ACCUMULATE) != 0;
  const int nsrc = src.n(), nrec = rec.n();
  const int64_t N = (int64_t)g->n[0] * g->n[1] * g->n[2];
  const int nall = nfreq * nsrc;
  if (info)
    for (int k = 0; k < 2 * nall * nky; ++k) to_info(SolveInfo(), info + k);
  std::vector<int> rows;
  for (int k = 0; k < nall; ++k)
    if (!mask || mask[k]) rows.push_back(k);
  const int nrow = (int)rows.size(), np = nrow * nky;
  if (np == 0) {
    if (f) *f = 0.0;
    if (!fwd_only && !acc) HELM_HIP_CHECK(hipMemsetAsync(grad, 0, (size_t)N * sizeof(T), st));
    HELM_HIP_CHECK(hipStreamSynchronize(st));
    return HELM_OK;
  }
  const double scale = (flags & HELM_MG_RENORMALISE) ? 1.0 / nrow : 1.0;
  std::vector<double> kq((size_t)nfreq * nky), wq((size_t)nfreq * nky);
  for (int fi = 0; fi < nfreq; ++fi) {
    const double K = std::min(p_kc * omega[fi] / v_min, M_PI / g->h);
    gauss_legendre(nky, K, &kq[(size_t)fi * nky], &wq[(size_t)fi * nky]);
    for (int i = 0; i < nky; ++i) wq[(size_t)fi * nky + i] /= M_PI;
  }
  std::vector<int> mslot(nfreq, -1);  // model set of each frequency with a selected row
  int nmf = 0;
  for (int k : rows)
    if (mslot[k / nsrc] < 0) mslot[k / nsrc] = nmf++;
  const int nm = nmf * nky;
  std::vector<double> shift(nm);
  for (int fi = 0; fi < nfreq; ++fi)
    if (mslot[fi] >= 0)
      for (int i = 0; i < nky; ++i) {
        const double kk = kq[(size_t)fi * nky + i];
        shift[(size_t)mslot[fi] * nky + i] = kk * kk / (omega[fi] * omega[fi]);
      }
  std::vector<int> src_of_pair(np);
  std::vector<double2> amp(np);
  std::vector<double> pk(np), pw(np), pys(np), wg(np);
  std::vector<int64_t> drow(nrow), uoff(np);
  for (int r = 0; r < nrow; ++r) {
    const int k = rows[r], fi = k / nsrc, s = k % nsrc;
    drow[r] = k;
    for (int i = 0; i < nky; ++i) {
      const int p = r * nky + i;
      src_of_pair[p] = s;
      amp[p] = src_amp ? make_double2(src_amp[2 * (size_t)k], src_amp[2 * (size_t)k + 1]) : make_double2(1.0, 0.0);
      pk[p] = kq[(size_t)fi * nky + i];
      pw[p] = wq[(size_t)fi * nky + i];
      pys[p] = src_y[s];
      wg[p] = omega[fi] * omega[fi] * scale;
      uoff[p] = (int64_t)p * N;
    }
  }
  // receiver node lists (distinct nodes ascending, each with its (receiver,
  // weight) entries in receiver order: a fixed summation order)
  const int nent = (int)rec.lin.size();
  std::vector<int> ent(nent), ent_rec(nent);
  for (int k = 0; k < nrec; ++k)
    for (int e = rec.ptr[k]; e < rec.ptr[k + 1]; ++e) ent_rec[e] = k;
  for (int e = 0; e < nent; ++e) ent[e] = e;
  std::stable_sort(ent.begin(), ent.end(), [&](int x, int y) { return rec.lin[x] < rec.lin[y]; });
  std::vector<int64_t> node_lin;
  std::vector<int> node_ptr, node_rec(nent);
  std::vector<double> node_w(nent);
  for (int i = 0; i < nent; ++i) {
    const int e = ent[i];
    if (node_lin.empty() || node_lin.back() != rec.lin[e]) {
      node_lin.push_back(rec.lin[e]);
      node_ptr.push_back(i);
    }
    node_rec[i] = ent_rec[e];
    node_w[i] = rec.w[e];
  }
  node_ptr.push_back(nent);
  const int nnode = (int)node_lin.size();
  const int rblk = (int)ceil_div(nrec, 256);
  int smax = 1;
  for (int k = 0; k < nsrc; ++k) smax = std::max(smax, src.ptr[k + 1] - src.ptr[k]);
  const int nsent = (int)src.lin.size();
  // small device tables
  auto r256 = [](size_t b) { return (b + 255) / 256 * 256; };
  struct Up {
    const void* h;
    size_t b;
    void** d;
  };
  int *d_src_of_pair, *d_sptr, *d_rptr, *d_nptr, *d_nrec;
  double2* d_amp;
  double *d_pk, *d_pw, *d_pys, *d_wg, *d_shift, *d_sw, *d_rw, *d_nw, *d_recy, *d_part;
  int64_t *d_drow, *d_uoff, *d_slin, *d_rlin, *d_node;
  cx<T>* d_res;
  std::vector<Up> ups = {
      {src_of_pair.data(), np * sizeof(int), (void**)&d_src_of_pair},
      {amp.data(), np * sizeof(double2), (void**)&d_amp},
      {pk.data(), np * sizeof(double), (void**)&d_pk},
      {pw.data(), np * sizeof(double), (void**)&d_pw},
      {pys.data(), np * sizeof(double), (void**)&d_pys},
      {wg.data(), np * sizeof(double), (void**)&d_wg},
      {shift.data(), nm * sizeof(double), (void**)&d_shift},
      {drow.data(), nrow * sizeof(int64_t), (void**)&d_drow},
      {uoff.data(), np * sizeof(int64_t), (void**)&d_uoff},
      {src.ptr.data(), (nsrc + 1) * sizeof(int), (void**)&d_sptr},
      {src.lin.data(), nsent * sizeof(int64_t), (void**)&d_slin},
      {src.w.data(), nsent * sizeof(double), (void**)&d_sw},
      {rec.ptr.data(), (nrec + 1) * sizeof(int), (void**)&d_rptr},
      {rec.lin.data(), nent * sizeof(int64_t), (void**)&d_rlin},
      {rec.w.data(), nent * sizeof(double), (void**)&d_rw},
      {node_lin.data(), nnode * sizeof(int64_t), (void**)&d_node},
      {node_ptr.data(), (nnode + 1) * sizeof(int), (void**)&d_nptr},
      {node_rec.data(), nent * sizeof(int), (void**)&d_nrec},
      {node_w.data(), nent * sizeof(double), (void**)&d_nw},
      {rec_y, nrec * sizeof(double), (void**)&d_recy},
      {nullptr, (size_t)nrow * nrec * sizeof(cx<T>), (void**)&d_res},
      {nullptr, (size_t)nrow * rblk * sizeof(double), (void**)&d_part}};
  size_t small = 0;
  for (const Up& u : ups) small += r256(u.b);
  ctx->fwi_small.ensure(small);
  char* sp = (char*)ctx->fwi_small.p;
  for (const Up& u : ups) {
    *u.d = sp;
    if (u.h && u.b) HELM_HIP_CHECK(hipMemcpyAsync(sp, u.h, u.b, hipMemcpyHostToDevice, st));
    sp += r256(u.b);
  }
  // large buffers: the shifted models, then Q, U, V (pairs contiguous)
  const size_t mb = r256((size_t)nm * N * sizeof(T)), fb = r256((size_t)np * N * sizeof(cx<T>));
  ctx->fwi_buf.ensure(mb + 3 * fb);
  char* base = (char*)ctx->fwi_buf.p;
  T* models = (T*)base;
  cx<T>* Q = (cx<T>*)(base + mb);
  cx<T>* U = (cx<T>*)(base + mb + fb);
  cx<T>* V = (cx<T>*)(base + mb + 2 * fb);
  hipLaunchKernelGGL((k_shift_models<T>), dim3(std::min<unsigned>(1024, ceil_div(N, 256)), nm), dim3(256), 0, st,
                     (const T*)m, N, (const double*)d_shift, models);
  HELM_HIP_CHECK(hipGetLastError());
  std::vector<ProblemSpec> probs;
  for (int r = 0; r < nrow; ++r) {
    const int fi = rows[r] / nsrc;
    for (int i = 0; i < nky; ++i)
      probs.push_back(shared_problems(g, models + ((size_t)mslot[fi] * nky + i) * N, omega[fi], 0, 1)[0]);
  }
  // the host tables above go out of scope with the function: copies must be done
  HELM_HIP_CHECK(hipStreamSynchronize(st));
  Solver<T>& S = solver_for<T>(ctx, probs, o, st);
  std::vector<SolveInfo> inf(np);
  int worst = 0;
  const double inv_h2 = 1.0 / (g->h * g->h);
  hipLaunchKernelGGL((k_fill_zero<T>), dim3(std::min<unsigned>(65536, ceil_div((int64_t)np * N, 256))), dim3(256), 0,
                     st, Q, (int64_t)np * N);
  hipLaunchKernelGGL((k_point_sources<T>), dim3((unsigned)ceil_div(smax, 256), np), dim3(256), 0, st, Q, N,
                     (const int*)d_src_of_pair, (const int*)d_sptr, (const int64_t*)d_slin, (const double*)d_sw,
                     (const double2*)d_amp, inv_h2);
  HELM_HIP_CHECK(hipGetLastError());
  worst = std::max(worst, S.solve(0, Q, U, inf.data()));
  auto put_info = [&](int which) {
    if (!info) return;
    for (int r = 0; r < nrow; ++r)
      for (int i = 0; i < nky; ++i)
        to_info(inf[r * nky + i], info + (size_t)which * nall * nky + (size_t)rows[r] * nky + i);
  };
  put_info(0);
  const Quad25 q{d_pk, d_pw, d_pys};
  hipLaunchKernelGGL((k_synth25d<T>), dim3(rblk, nrow), dim3(256), 0, st, S.iterate(), N, nky, q,
                     (const int*)d_rptr, (const int64_t*)d_rlin, (const double*)d_rw, (const double*)d_recy, nrec,
                     (const cx<T>*)d, (const int64_t*)d_drow, d_res, (cx<T>*)d_pred, d_part);
  HELM_HIP_CHECK(hipGetLastError());
  std::vector<double> hpart((size_t)nrow * rblk);
  HELM_HIP_CHECK(hipMemcpyAsync(hpart.data(), d_part, hpart.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HELM_HIP_CHECK(hipStreamSynchronize(st));
  double fsum = 0.0;
  for (double v : hpart) fsum += v;
  if (f) *f = 0.5 * fsum * scale;
  if (fwd_only) return (helm_status)worst;
  hipLaunchKernelGGL((k_fill_zero<T>), dim3(std::min<unsigned>(65536, ceil_div((int64_t)np * N, 256))), dim3(256), 0,
                     st, Q, (int64_t)np * N);
  hipLaunchKernelGGL((k_adjoint25d<T>), dim3((unsigned)ceil_div(nnode, 256), np), dim3(256), 0, st, Q, N, nky, q,
                     (const int64_t*)d_node, (const int*)d_nptr, (const int*)d_nrec, (const double*)d_nw, nnode,
                     (const double*)d_recy, (const cx<T>*)d_res, nrec);
  HELM_HIP_CHECK(hipGetLastError());
  worst = std::max(worst, S.solve(1, Q, V, inf.data()));
  put_info(1);
  hipLaunchKernelGGL((k_gradient<T, T, T, false>), dim3(std::min<unsigned>(4096, ceil_div(N, 256))), dim3(256), 0, st,
                     (const cx<T>*)U, (const int64_t*)d_uoff, (const cx<T>*)V, np, g->n[0], g->n[1], g->n[2],
                     (const double*)d_wg, 1.0, 0.0, 0.0, 0.0, (T*)grad, acc);
  HELM_HIP_CHECK(hipGetLastError());
  HELM_HIP_CHECK(hipStreamSynchronize(st));
  return (helm_status)worst;
}

// Per-pair kernels take the pair from blockIdx.y, whose extent HIP bounds by
// 65536 blocks.
constexpr int64_t kMaxPairs = 65535;

void check_pair_args(const helm_grid* g, const void* m, int nfreq, const double* omega, int nsrc, int nrec) {
  check_grid(g);
  HELM_REQUIRE(m, "null model pointer");
  HELM_REQUIRE(nfreq >= 1 && omega, "nfreq must be >= 1 with an omega array");
  for (int k = 0; k < nfreq; ++k) HELM_REQUIRE(omega[k] > 0.0 && std::isfinite(omega[k]), "omega must be positive");
  HELM_REQUIRE(nsrc >= 1 && nrec >= 1, "nsrc and nrec must be >= 1");
  HELM_REQUIRE((int64_t)nfreq * nsrc <= kMaxPairs, "more than 65535 (frequency, source) pairs");
}

void check_nodes(const helm_grid* g, int n, const int32_t* idx, const char* what) {
  for (int k = 0; k < n; ++k)
    for (int a = 0; a < 3; ++a) HELM_REQUIRE(idx[3 * k + a] >= 0 && idx[3 * k + a] < g->n[a], what);
}

void check_sinc(const helm_grid* g, int nsrc, const double* src_pos, int nrec, const double* rec_pos, int radius,
                double kb) {
  HELM_REQUIRE(radius >= 1 && radius <= 8, "sinc radius must be in 1..8");
  HELM_REQUIRE(kb >= 0.0 && kb <= 100.0, "Kaiser window shape must be in [0, 100]");
  for (int k = 0; k < nsrc; ++k)
    for (int a = 0; a < 3; ++a)
      HELM_REQUIRE(std::isfinite(src_pos[3 * k + a]) && src_pos[3 * k + a] >= 0.0 &&
                       src_pos[3 * k + a] <= g->n[a] - 1,
                   "source outside the grid");
  for (int k = 0; k < nrec; ++k)
    for (int a = 0; a < 3; ++a)
      HELM_REQUIRE(std::isfinite(rec_pos[3 * k + a]) && rec_pos[3 * k + a] >= 0.0 &&
                       rec_pos[3 * k + a] <= g->n[a] - 1,
                   "receiver outside the grid");
  HELM_REQUIRE((int64_t)nrec * (2 * radius) * (2 * radius) * (2 * radius) < ((int64_t)1 << 31),
               "too many receiver interpolation entries");
}

helm_status misfit_common(helm_ctx* ctx, const helm_grid* g, const void* m, int nfreq, const double* omega,
                          const PointSet& src, const double* src_amp, const uint8_t* mask, const PointSet& rec,
                          const void* d, double* f, void* grad, void* u_store, int flags, const helm_solver_opts* o,
                          helm_solve_info* info, void* stream) {
  HELM_REQUIRE(d && f, "null pointer argument");
  HELM_REQUIRE((flags & HELM_MG_FORWARD_ONLY) || grad, "null gradient");
  HELM_REQUIRE(!(flags & HELM_MG_REUSE_U) || u_store, "HELM_MG_REUSE_U needs u_store");
  HELM_REQUIRE(!(flags & HELM_MG_U_FP64) || u_store, "HELM_MG_U_FP64 needs u_store");
  HELM_REQUIRE((flags & ~31) == 0, "unknown flag bits");
  const helm::SolveOpts so = opts_of(o);
  check_coarse_sizes(g, so);
  if (g->dtype == HELM_C64)
    return misfit_gradient_t<float>(ctx, g, m, nfreq, omega, src, src_amp, mask, rec, d, f, grad, u_store, flags, so,
                                    info, stream);
  return misfit_gradient_t<double>(ctx, g, m, nfreq, omega, src, src_amp, mask, rec, d, f, grad, u_store, flags, so,
                                   info, stream);
}

helm_status derivative_common(helm_ctx* ctx, int mode, const helm_grid* g, const void* m, int nfreq,
                              const double* omega, const PointSet& src, const double* src_amp, const uint8_t* mask,
                              const PointSet& rec, const void* input, const void* d, void* output, void* u_store,
                              int flags, const helm_solver_opts* o, helm_solve_info* info, void* stream) {
  HELM_REQUIRE(mode == HELM_JACOB_FORW || mode == HELM_JACOB_ADJ || mode == HELM_HESS_GN || mode == HELM_HESS,
               "unknown derivative mode");
  HELM_REQUIRE(input && output, "null pointer argument");
  HELM_REQUIRE(mode != HELM_HESS || d, "HELM_HESS needs the observed data d");
  HELM_REQUIRE(!(flags & HELM_MG_REUSE_U) || u_store, "HELM_MG_REUSE_U needs u_store");
  HELM_REQUIRE(!(flags & HELM_MG_U_FP64) || u_store, "HELM_MG_U_FP64 needs u_store");
  HELM_REQUIRE((flags & ~(HELM_MG_REUSE_U | HELM_MG_ACCUMULATE | HELM_MG_U_FP64 | HELM_MG_RENORMALISE)) == 0,
               "unknown or unsupported flag bits");
  const helm::SolveOpts so = opts_of(o);
  check_coarse_sizes(g, so);
  if (g->dtype == HELM_C64)
    return derivative_t<float>(ctx, mode, g, m, nfreq, omega, src, src_amp, mask, rec, input, d, output, u_store,
                               flags, so, info, stream);
  return derivative_t<double>(ctx, mode, g, m, nfreq, omega, src, src_amp, mask, rec, input, d, output, u_store, flags,
                              so, info, stream);
}

#include "driver.hip"

// Opt-in input scan (environment HELM_CHECK=1): a NaN or Inf in a caller's
// input array returns HELM_E_INVAL naming the array.  One pass per array on
// the caller's stream and a synchronisation of that stream, before the
// call's own work; rows of unselected (frequency, source) pairs, which the
// calls do not read, are not scanned.
bool input_check_on() {
  const char* e = std::getenv("HELM_CHECK");
  return e && e[0] == '1';
}

// flag[blockIdx.y * gridDim.x + blockIdx.x] = 1 if any of the n scalars of
// row blockIdx.y (at a + row_off[blockIdx.y], or at a without row_off) is
// not finite
template <typename T>
__global__ __launch_bounds__(256) void k_nonfinite(const T* __restrict__ a, const int64_t* __restrict__ row_off,
                                                   int64_t n, int* __restrict__ flag) {
  const T* r = a + (row_off ? row_off[blockIdx.y] : 0);
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    bad |= isfinite(r[i]) ? 0 : 1;
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) flag[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = bad;
}

// n scalars (double with dbl, else float) per row; rows at the scalar
// offsets `off` (at most 65535 of them), or one row at a when off is NULL
void scan_finite(helm_ctx* ctx, const void* a, int64_t n, const std::vector<int64_t>* off, bool dbl,
                 const std::string& what, void* stream) {
  if (!a || n <= 0 || (off && off->empty())) return;
  hipStream_t st = (hipStream_t)stream;
  const int nrow = off ? (int)off->size() : 1;
  const unsigned nb = (unsigned)std::min<int64_t>(off ? 16 : 1024, helm::ceil_div(n, 256));
  const size_t fb = ((size_t)nrow * nb * sizeof(int) + 255) / 256 * 256;
  ctx->chk.ensure(fb + (off ? off->size() * sizeof(int64_t) : 0));
  int* flag = (int*)ctx->chk.p;
  int64_t* doff = off ? (int64_t*)((char*)ctx->chk.p + fb) : nullptr;
  if (doff)
    HELM_HIP_CHECK(hipMemcpyAsync(doff, off->data(), off->size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
  if (dbl)
    hipLaunchKernelGGL(k_nonfinite<double>, dim3(nb, nrow), dim3(256), 0, st, (const double*)a,
                       (const int64_t*)doff, n, flag);
  else
    hipLaunchKernelGGL(k_nonfinite<float>, dim3(nb, nrow), dim3(256), 0, st, (const float*)a,
                       (const int64_t*)doff, n, flag);
  HELM_HIP_CHECK(hipGetLastError());
  std::vector<int> h((size_t)nrow * nb);
  HELM_HIP_CHECK(hipMemcpyAsync(h.data(), flag, h.size() * sizeof(int), hipMemcpyDeviceToHost, st));
  HELM_HIP_CHECK(hipStreamSynchronize(st));
  for (int v : h) HELM_REQUIRE(v == 0, "non-finite value (NaN or Inf) in " + what + " (HELM_CHECK=1)");
}

int64_t grid_points(const helm_grid* g) { return (int64_t)g->n[0] * g->n[1] * g->n[2]; }

// the model and, over the selected (frequency, source) rows, an array of
// nrec complex values per pair (data, or the adjoint Jacobian's input)
void scan_model(helm_ctx* ctx, const helm_grid* g, const void* m, void* stream) {
  scan_finite(ctx, m, grid_points(g), nullptr, g->dtype == HELM_C128, "the model m", stream);
}
void scan_pair_rows(helm_ctx* ctx, const helm_grid* g, int nfreq, int nsrc, const uint8_t* mask, int nrec,
                    const void* a, const std::string& what, void* stream) {
  std::vector<int64_t> off;
  for (int k = 0; k < nfreq * nsrc; ++k)
    if (!mask || mask[k]) off.push_back((int64_t)k * nrec * 2);
  scan_finite(ctx, a, (int64_t)nrec * 2, &off, g->dtype == HELM_C128, what, stream);
}

void scan_misfit_inputs(helm_ctx* ctx, const helm_grid* g, const void* m, int nfreq, int nsrc, const uint8_t* mask,
                        int nrec, const void* d, void* stream) {
  if (!input_check_on()) return;
  scan_model(ctx, g, m, stream);
  scan_pair_rows(ctx, g, nfreq, nsrc, mask, nrec, d, "the data d", stream);
}

void scan_derivative_inputs(helm_ctx* ctx, int mode, const helm_grid* g, const void* m, int nfreq, int nsrc,
                            const uint8_t* mask, int nrec, const void* input, const void* d, void* stream) {
  if (!input_check_on()) return;
  scan_model(ctx, g, m, stream);
  if (mode == HELM_JACOB_ADJ)
    scan_pair_rows(ctx, g, nfreq, nsrc, mask, nrec, input, "the input y", stream);
  else
    scan_finite(ctx, input, grid_points(g), nullptr, g->dtype == HELM_C128, "the input dm", stream);
  if (mode == HELM_HESS) scan_pair_rows(ctx, g, nfreq, nsrc, mask, nrec, d, "the data d", stream);
}

// (the bounds may be infinite; a NaN bound is rejected by the driver itself)
void scan_fwi_inputs(helm_ctx* ctx, const helm_grid* g, const void* m, int nfreq, int nsrc, int nrec, const void* d,
                     void* stream) {
  if (!input_check_on()) return;
  scan_model(ctx, g, m, stream);
  scan_finite(ctx, d, 2 * (int64_t)nfreq * nsrc * nrec, nullptr, g->dtype == HELM_C128, "the data d", stream);
}

}  // namespace

extern "C" {

const char* helm_version(void) { return "helm-gfx950 0.2"; }

helm_status helm_create(helm_ctx** ctx, int device) {
  if (!ctx) return fail(nullptr, HELM_E_INVAL, "null output pointer");
  *ctx = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return fail(nullptr, HELM_E_HIP, "no such HIP device");
  }
  // the device address of the allocation-free entry point's scratch array,
  // resolved once per device with that device current
  int prev = 0;
  (void)hipGetDevice(&prev);
  try {
    HELM_HIP_CHECK(hipSetDevice(device));
    (void)helm::scratch_address(device);
  } catch (const helm::Error& err) {
    (void)hipGetLastError();
    (void)hipSetDevice(prev);
    return fail(nullptr, err.code, err.msg);
  }
  (void)hipSetDevice(prev);
  helm_ctx* c = new (std::nothrow) helm_ctx();
  if (!c) return fail(nullptr, HELM_E_NOMEM, "out of host memory");
  c->device = device;
  *ctx = c;
  return HELM_OK;
}

helm_status helm_destroy(helm_ctx* ctx) {
  if (!ctx) return HELM_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  ctx->solver.s32.reset();
  ctx->solver.s64.reset();
  ctx->apply_h.reset();
  if (ctx->ev) (void)hipEventDestroy(ctx->ev);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return HELM_OK;
}

const char* helm_last_error(const helm_ctx* ctx) { return ctx ? ctx->err.c_str() : g_global_err.c_str(); }

void helm_default_opts(helm_solver_opts* o) {
  if (!o) return;
  o->method = HELM_FGMRES_ML;
  o->restart = 5;
  o->max_cycles = 50;
  o->tol = 1e-6;
  o->ks_o = 3;
  o->ks_i = 5;
  o->kc_o = 3;
  o->kc_i = 5;
  o->levels = 3;
  o->warm_start = 0;
}

size_t helm_workspace_bytes(const helm_grid* g, const helm_solver_opts* o, int nrhs) {
  try {
    check_grid(g);
    if (nrhs < 1) return 0;
    const helm::SolveOpts so = opts_of(o);
    check_coarse_sizes(g, so);
    const int nlev = so.method == HELM_FGMRES_ML ? so.levels : 1;
    std::vector<int64_t> Nlev(nlev);
    const bool pairs = helm::Hierarchy::uses_pairs(g->stencil, g->dtype == HELM_C64 ? 4 : 8);
    const bool pad = pairs && (g->n[2] & 1);  // as in a solve (wants_pad)
    for (int l = 0; l < nlev; ++l) Nlev[l] = helm::Hierarchy::level_points(g->n, l, pairs, pad) * nrhs;
    return g->dtype == HELM_C64 ? helm::Solver<float>::workspace_bytes(Nlev, so)
                                : helm::Solver<double>::workspace_bytes(Nlev, so);
  } catch (...) {
    return 0;
  }
}

helm_status helm_apply(helm_ctx* ctx, const helm_grid* g, const void* m, double omega, int adjoint, int nrhs,
                       const void* x, void* y, void* stream) {
  return guarded(ctx, [&]() -> helm_status {
    const helm::Range range_("helm_apply");
    check_grid(g);
    HELM_REQUIRE(m && x && y, "null device pointer");
    HELM_REQUIRE(omega > 0.0 && std::isfinite(omega), "omega must be positive");
    HELM_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    HELM_REQUIRE(x != y, "x and y must not overlap");
    if (input_check_on()) {
      scan_model(ctx, g, m, stream);
      scan_finite(ctx, x, 2 * grid_points(g) * nrhs, nullptr, g->dtype == HELM_C128, "the input x", stream);
    }
    hipStream_t st = (hipStream_t)stream;
    auto probs = shared_problems(g, m, omega, adjoint ? 1 : 0, nrhs);
    const helm::SolveOpts so = opts_of(nullptr);
    const std::string key = key_of(probs, so, g->dtype) + (adjoint ? "A" : "F");
    if (!ctx->apply_h || ctx->apply_key != key) {
      // rebuilding frees the previous operator: finish work that may use it
      if (ctx->apply_h) HELM_HIP_CHECK(hipDeviceSynchronize());
      ctx->apply_h.reset(new helm::Hierarchy(probs, 1, g->dtype == HELM_C64 ? 4 : 8, st));
      ctx->apply_key = key;
      // stencil tiles, timed on the caller's buffers (y is overwritten below)
      if (g->dtype == HELM_C64)
        helm::tune_tiles_apply<float>(*ctx->apply_h, (const helm::cx<float>*)x, (helm::cx<float>*)y, st);
      else
        helm::tune_tiles_apply<double>(*ctx->apply_h, (const helm::cx<double>*)x, (helm::cx<double>*)y, st);
    }
    const helm::LevelSet& L = ctx->apply_h->level(0);
    if (g->dtype == HELM_C64)
      helm::launch_h<float, float, float, float, float, false, false>(
          L, (const helm::cx<float>*)x, nullptr, (const helm::cx<float>*)nullptr, nullptr, (helm::cx<float>*)y,
          nullptr, nullptr, st);
    else
      helm::launch_h<double, double, double, double, double, false, false>(
          L, (const helm::cx<double>*)x, nullptr, (const helm::cx<double>*)nullptr, nullptr,
          (helm::cx<double>*)y, nullptr, nullptr, st);
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
  });
}

helm_status helm_apply_noalloc(helm_ctx* ctx, const helm_grid* g, const void* m, double omega, int adjoint,
                               int nrhs, const void* x, void* y, void* stream) {
  return guarded(ctx, [&]() -> helm_status {
    check_grid(g);
    HELM_REQUIRE(m && x && y, "null device pointer");
    HELM_REQUIRE(omega > 0.0 && std::isfinite(omega), "omega must be positive");
    HELM_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    HELM_REQUIRE(x != y, "x and y must not overlap");
    const helm::GridSpec s = spec_of(g);
    if (g->dtype == HELM_C64)
      helm::apply_noalloc<float>(ctx->device, s, m, omega, adjoint ? 1 : 0, nrhs, x, y, (hipStream_t)stream);
    else
      helm::apply_noalloc<double>(ctx->device, s, m, omega, adjoint ? 1 : 0, nrhs, x, y, (hipStream_t)stream);
    return HELM_OK;
  });
}

helm_status helm_solve(helm_ctx* ctx, const helm_grid* g, const void* m, double omega, int adjoint, int nrhs,
                       const void* q, void* u, const helm_solver_opts* o, helm_solve_info* info, void* stream) {
  return guarded(ctx, [&]() -> helm_status {
    const helm::Range range_("helm_solve");
    check_grid(g);
    HELM_REQUIRE(m && q && u, "null device pointer");
    HELM_REQUIRE(omega > 0.0 && std::isfinite(omega), "omega must be positive");
    HELM_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    const helm::SolveOpts so = opts_of(o);
    check_coarse_sizes(g, so);
    if (input_check_on()) {
      const bool dbl = g->dtype == HELM_C128;
      scan_model(ctx, g, m, stream);
      scan_finite(ctx, q, 2 * grid_points(g) * nrhs, nullptr, dbl, "the right-hand side q", stream);
      if (so.warm_start) scan_finite(ctx, u, 2 * grid_points(g) * nrhs, nullptr, dbl, "the initial guess u", stream);
    }
    if (g->dtype == HELM_C64) return solve_t<float>(ctx, g, m, omega, adjoint ? 1 : 0, nrhs, q, u, so, info, stream);
    return solve_t<double>(ctx, g, m, omega, adjoint ? 1 : 0, nrhs, q, u, so, info, stream);
  });
}

helm_status helm_solve_batched(helm_ctx* ctx, int nprob, const helm_problem* probs, int adjoint,
                               const helm_solver_opts* o, helm_solve_info* info, void* stream) {
  return guarded(ctx, [&]() -> helm_status {
    const helm::Range range_("helm_solve_batched");
    HELM_REQUIRE(nprob >= 1 && probs, "need at least one problem");
    const helm::SolveOpts so = opts_of(o);
    for (int i = 0; i < nprob; ++i) {
      check_grid(&probs[i].grid);
      check_coarse_sizes(&probs[i].grid, so);
      HELM_REQUIRE(probs[i].m && probs[i].q && probs[i].u, "null device pointer in a problem");
      HELM_REQUIRE(probs[i].omega > 0.0 && std::isfinite(probs[i].omega), "omega must be positive");
      HELM_REQUIRE(probs[i].grid.dtype == probs[0].grid.dtype, "all problems must have the same dtype");
      HELM_REQUIRE(probs[i].grid.stencil == probs[0].grid.stencil, "all problems must use the same stencil");
    }
    if (input_check_on())
      for (int i = 0; i < nprob; ++i) {
        const helm_grid* gi = &probs[i].grid;
        const bool dbl = gi->dtype == HELM_C128;
        const std::string pre = "problem " + std::to_string(i) + ": ";
        scan_finite(ctx, probs[i].m, grid_points(gi), nullptr, dbl, pre + "the model m", stream);
        scan_finite(ctx, probs[i].q, 2 * grid_points(gi), nullptr, dbl, pre + "the right-hand side q", stream);
        if (so.warm_start)
          scan_finite(ctx, probs[i].u, 2 * grid_points(gi), nullptr, dbl, pre + "the initial guess u", stream);
      }
    if (probs[0].grid.dtype == HELM_C64)
      return solve_batched_t<float>(ctx, nprob, probs, adjoint ? 1 : 0, so, info, stream);
    return solve_batched_t<double>(ctx, nprob, probs, adjoint ? 1 : 0, so, info, stream);
  });
}

helm_status misfit_gradient(helm_ctx* ctx, const helm_grid* g, const void* m, int nfreq, const double* omega,
                            int nsrc, const int32_t* src_idx, const double* src_amp, const uint8_t* mask, int nrec,
                            const int32_t* rec_idx, const void* d, double* f, void* grad, void* u_store, int flags,
                            const helm_solver_opts* o, helm_solve_info* info, void* stream) {
  return guarded(ctx, [&]() -> helm_status {
    const helm::Range range_("misfit_gradient");
    check_pair_args(g, m, nfreq, omega, nsrc, nrec);
    HELM_REQUIRE(src_idx && rec_idx, "null source / receiver index array");
    check_nodes(g, nsrc, src_idx, "source outside the grid");
    check_nodes(g, nrec, rec_idx, "receiver outside the grid");
    scan_misfit_inputs(ctx, g, m, nfreq, nsrc, mask, nrec, d, stream);
    return misfit_common(ctx, g, m, nfreq, omega, on_node_points(g, nsrc, src_idx), src_amp, mask,
                         on_node_points(g, nrec, rec_idx), d, f, grad, u_store, flags, o, info, stream);
  });
}

helm_status misfit_gradient_offgrid(helm_ctx* ctx, const helm_grid* g, const void* m, int nfreq,
                                    const double* omega, int nsrc, const double* src_pos, const double* src_amp,
                                    const uint8_t* mask, int nrec, const double* rec_pos, int radius,
                                    double kaiser_b, const void* d, double* f, void* grad, void* u_store, int flags,
                                    const helm_solver_opts* o, helm_solve_info* info, void* stream) {
  return guarded(ctx, [&]() -> helm_status {
    const helm::Range range_("misfit_gradient_offgrid");
    check_pair_args(g, m, nfreq, omega, nsrc, nrec);
    HELM_REQUIRE(src_pos && rec_pos, "null source / receiver position array");
    check_sinc(g, nsrc, src_pos, nrec, rec_pos, radius, kaiser_b);
    scan_misfit_inputs(ctx, g, m, nfreq, nsrc, mask, nrec, d, stream);
    return misfit_common(ctx, g, m, nfreq, omega, sinc_points(g, nsrc, src_pos, radius, kaiser_b), src_amp, mask,
                         sinc_points(g, nrec, rec_pos, radius, kaiser_b), d, f, grad, u_store, flags, o, info,
                         stream);
  });
}

helm_status pde_derivative(helm_ctx* ctx, int mode, const helm_grid* g, const void* m, int nfreq,
                           const double* omega, int nsrc, const int32_t* src_idx, const double* src_amp,
                           const uint8_t* mask, int nrec, const int32_t* rec_idx, const void* input, const void* d,
                           void* output, void* u_store, int flags, const helm_solver_opts* o, helm_solve_info* info,
                           void* stream) {
  return guarded(ctx, [&]() -> helm_status {
    const helm::Range range_("pde_derivative");
    check_pair_args(g, m, nfreq, omega, nsrc, nrec);
    HELM_REQUIRE(src_idx && rec_idx, "null source / receiver index array");
    check_nodes(g, nsrc, src_idx, "source outside the grid");
    check_nodes(g, nrec, rec_idx, "receiver outside the grid");
    scan_derivative_inputs(ctx, mode, g, m, nfreq, nsrc, mask, nrec, input, d, stream);
    return derivative_common(ctx, mode, g, m, nfreq, omega, on_node_points(g, nsrc, src_idx), src_amp, mask,
                             on_node_points(g, nrec, rec_idx), input, d, output, u_store, flags, o, info, stream);
  });
}

helm_status pde_derivative_offgrid(helm_ctx* ctx, int mode, const helm_grid* g, const void* m, int nfreq,
                                   const double* omega, int nsrc, const double* src_pos, const double* src_amp,
                                   const uint8_t* mask, int nrec, const double* rec_pos, int radius, double kaiser_b,
                                   const void* input, const void* d, void* output, void* u_store, int flags,
                                   const helm_solver_opts* o, helm_solve_info* info, void* stream) {
  return guarded(ctx, [&]() -> helm_status {
    const helm::Range range_("pde_derivative_offgrid");
    check_pair_args(g, m, nfreq, omega, nsrc, nrec);
    HELM_REQUIRE(src_pos && rec_pos, "null source / receiver position array");
    check_sinc(g, nsrc, src_pos, nrec, rec_pos, radius, kaiser_b);
    scan_derivative_inputs(ctx, mode, g, m, nfreq, nsrc, mask, nrec, input, d, stream);
    return derivative_common(ctx, mode, g, m, nfreq, omega, sinc_points(g, nsrc, src_pos, radius, kaiser_b),
                             src_amp, mask, sinc_points(g, nrec, rec_pos, radius, kaiser_b), input, d, output,
                             u_store, flags, o, info, stream);
  });
}

int helm_fwi_draw_count(int nfreq, const helm_fwi_params* p) {
  try {
    HELM_REQUIRE(nfreq >= 1, "nfreq must be >= 1");
    check_fwi_params(p);
    return fwi_band_count(nfreq, p->band_size, p->band_overlap) * p->subproblems;
  } catch (...) {
    return -1;
  }
}

helm_status fwi_invert(helm_ctx* ctx, const helm_grid* g, void* m, const double* lo, const double* hi, int nfreq,
                       const double* omega, int nsrc, const int32_t* src_idx, const double* src_amp, int nrec,
                       const int32_t* rec_idx, const void* d, const helm_fwi_params* p, const helm_solver_opts* o,
                       helm_fwi_draw* draws, int32_t* sources, helm_fwi_record* recs, int rec_cap, int* nrecs,
                       void* stream) {
  return guarded(ctx, [&]() -> helm_status {
    const helm::Range range_("fwi_invert");
    check_pair_args(g, m, nfreq, omega, nsrc, nrec);
    HELM_REQUIRE(src_idx && rec_idx, "null source / receiver index array");
    check_nodes(g, nsrc, src_idx, "source outside the grid");
    check_nodes(g, nrec, rec_idx, "receiver outside the grid");
    scan_fwi_inputs(ctx, g, m, nfreq, nsrc, nrec, d, stream);
    return fwi_common(ctx, g, m, lo, hi, nfreq, omega, on_node_points(g, nsrc, src_idx), src_amp,
                      on_node_points(g, nrec, rec_idx), d, p, o, draws, sources, recs, rec_cap, nrecs, stream);
  });
}

helm_status fwi_invert_offgrid(helm_ctx* ctx, const helm_grid* g, void* m, const double* lo, const double* hi,
                               int nfreq, const double* omega, int nsrc, const double* src_pos,
                               const double* src_amp, int nrec, const double* rec_pos, int radius, double kaiser_b,
                               const void* d, const helm_fwi_params* p, const helm_solver_opts* o,
                               helm_fwi_draw* draws, int32_t* sources, helm_fwi_record* recs, int rec_cap,
                               int* nrecs, void* stream) {
  return guarded(ctx, [&]() -> helm_status {
    const helm::Range range_("fwi_invert_offgrid");
    check_pair_args(g, m, nfreq, omega, nsrc, nrec);
    HELM_REQUIRE(src_pos && rec_pos, "null source / receiver position array");
    check_sinc(g, nsrc, src_pos, nrec, rec_pos, radius, kaiser_b);
    scan_fwi_inputs(ctx, g, m, nfreq, nsrc, nrec, d, stream);
    return fwi_common(ctx, g, m, lo, hi, nfreq, omega, sinc_points(g, nsrc, src_pos, radius, kaiser_b), src_amp,
                      sinc_points(g, nrec, rec_pos, radius, kaiser_b), d, p, o, draws, sources, recs, rec_cap, nrecs,
                      stream);
  });
}

helm_status wri_misfit_gradient(helm_ctx* ctx, const helm_grid* g, const void* m, int nfreq,
                                const double* omega, int nsrc, const int32_t* src_idx, const double* src_amp,
                                const uint8_t* mask, int nrec, const int32_t* rec_idx, const void* d, double lambda,
                                double cg_tol, int cg_max, double* f, void* grad, void* u_store, int flags,
                                const helm_solver_opts* o, helm_solve_info* info, void* stream) {
  return guarded(ctx, [&]() -> helm_status {
    const helm::Range range_("wri_misfit_gradient");
    check_pair_args(g, m, nfreq, omega, nsrc, nrec);
    HELM_REQUIRE(src_idx && rec_idx, "null source / receiver index array");
    check_nodes(g, nsrc, src_idx, "source outside the grid");
    check_nodes(g, nrec, rec_idx, "receiver outside the grid");
    HELM_REQUIRE(d && f, "null pointer argument");
    HELM_REQUIRE((flags & HELM_MG_FORWARD_ONLY) || grad, "null gradient");
    HELM_REQUIRE(!(flags & HELM_MG_U_FP64) || u_store, "HELM_MG_U_FP64 needs u_store");
    HELM_REQUIRE((flags & ~(HELM_MG_FORWARD_ONLY | HELM_MG_ACCUMULATE | HELM_MG_U_FP64 | HELM_MG_RENORMALISE)) == 0,
                 "unknown or unsupported flag bits");
    HELM_REQUIRE(lambda > 0.0 && std::isfinite(lambda), "lambda must be positive");
    HELM_REQUIRE(cg_tol >= 0.0 && cg_tol < 1.0, "cg_tol must be in [0, 1)");
    HELM_REQUIRE(cg_max >= 0, "cg_max must be >= 0");
    const helm::SolveOpts so = opts_of(o);
    check_coarse_sizes(g, so);
    scan_misfit_inputs(ctx, g, m, nfreq, nsrc, mask, nrec, d, stream);
    const PointSet S = on_node_points(g, nsrc, src_idx), R = on_node_points(g, nrec, rec_idx);
    if (g->dtype == HELM_C64)
      return wri_t<float>(ctx, g, m, nfreq, omega, S, src_amp, mask, R, d, lambda, cg_tol, cg_max, f, grad, u_store,
                          flags, so, info, stream);
    return wri_t<double>(ctx, g, m, nfreq, omega, S, src_amp, mask, R, d, lambda, cg_tol, cg_max, f, grad, u_store,
                         flags, so, info, stream);
  });
}

helm_status misfit_gradient_25d(helm_ctx* ctx, const helm_grid* g, const void* m, int nfreq,
                                const double* omega, int nky, double p_kc, double v_min, int nsrc,
                                const int32_t* src_idx, const double* src_y, const double* src_amp,
                                const uint8_t* mask, int nrec, const int32_t* rec_idx, const double* rec_y,
                                const void* d, double* f, void* grad, void* d_pred, int flags,
                                const helm_solver_opts* o, helm_solve_info* info, void* stream) {
  return guarded(ctx, [&]() -> helm_status {
    const helm::Range range_("misfit_gradient_25d");
    check_pair_args(g, m, nfreq, omega, nsrc, nrec);
    HELM_REQUIRE(g->n[0] == 1, "2.5D modelling runs on a 2D grid (n[0] = 1)");
    HELM_REQUIRE(nky >= 1 && nky <= 4096, "nky must be in 1..4096");
    HELM_REQUIRE(p_kc > 0.0 && std::isfinite(p_kc), "p_kc must be positive");
    HELM_REQUIRE(v_min > 0.0 && std::isfinite(v_min), "v_min must be positive");
    HELM_REQUIRE(src_idx && rec_idx && src_y && rec_y && f, "null pointer argument");
    HELM_REQUIRE((flags & ~(HELM_MG_FORWARD_ONLY | HELM_MG_ACCUMULATE | HELM_MG_RENORMALISE)) == 0,
                 "unknown or unsupported flag bits");
    HELM_REQUIRE(d || (flags & HELM_MG_FORWARD_ONLY), "observed data needed for the gradient");
    HELM_REQUIRE((flags & HELM_MG_FORWARD_ONLY) || grad, "null gradient");
    for (int k = 0; k < nsrc; ++k) HELM_REQUIRE(std::isfinite(src_y[k]), "non-finite source coordinate");
    for (int k = 0; k < nrec; ++k) HELM_REQUIRE(std::isfinite(rec_y[k]), "non-finite receiver coordinate");
    std::vector<int32_t> s3(3 * (size_t)nsrc), r3(3 * (size_t)nrec);
    for (int k = 0; k < nsrc; ++k) {
      s3[3 * k] = 0;
      s3[3 * k + 1] = src_idx[2 * k];
      s3[3 * k + 2] = src_idx[2 * k + 1];
    }
    for (int k = 0; k < nrec; ++k) {
      r3[3 * k] = 0;
      r3[3 * k + 1] = rec_idx[2 * k];
      r3[3 * k + 2] = rec_idx[2 * k + 1];
    }
    check_nodes(g, nsrc, s3.data(), "source outside the grid");
    check_nodes(g, nrec, r3.data(), "receiver outside the grid");
    HELM_REQUIRE((int64_t)nfreq * nsrc * nky <= kMaxPairs, "more than 65535 2D problems (nfreq*nsrc*nky)");
    const helm::SolveOpts so = opts_of(o);
    check_coarse_sizes(g, so);
    scan_misfit_inputs(ctx, g, m, nfreq, nsrc, mask, nrec, d, stream);
    const PointSet S = on_node_points(g, nsrc, s3.data()), R = on_node_points(g, nrec, r3.data());
    if (g->dtype == HELM_C64)
      return model25d_t<float>(ctx, g, m, nfreq, omega, nky, p_kc, v_min, S, src_y, src_amp, mask, R, rec_y, d, f,
                               grad, d_pred, flags, so, info, stream);
    return model25d_t<double>(ctx, g, m, nfreq, omega, nky, p_kc, v_min, S, src_y, src_amp, mask, R, rec_y, d, f,
                              grad, d_pred, flags, so, info, stream);
  });
}

}  // extern "C"
