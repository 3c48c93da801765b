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
  for (int a = 0; a < 3; ++a) HELM_REQUIRE(g->n[a] >= 3, "grid sizes must be >= 3");
  HELM_REQUIRE((int64_t)g->n[0] * g->n[1] * g->n[2] < ((int64_t)1 << 40), "grid too large");
  HELM_REQUIRE(g->h > 0.0 && std::isfinite(g->h), "grid spacing must be positive");
  HELM_REQUIRE(g->npml >= 0, "npml must be >= 0");
  for (int a = 0; a < 3; ++a) HELM_REQUIRE(2 * g->npml < g->n[a], "npml must be < n/2 on every axis");
  if (g->npml > 0) {
    HELM_REQUIRE(g->pml_R > 0.0 && g->pml_R < 1.0, "pml_R must be in (0, 1)");
    HELM_REQUIRE(g->v_ref > 0.0 && std::isfinite(g->v_ref), "v_ref must be positive");
  }
  HELM_REQUIRE(g->stencil == HELM_7PT || g->stencil == HELM_27PT, "unknown stencil");
  HELM_REQUIRE(g->dtype == HELM_C64 || g->dtype == HELM_C128, "unknown dtype");
  if (g->stencil == HELM_27PT)
    for (int c = 0; c < 7; ++c) HELM_REQUIRE(std::isfinite(g->w27[c]), "27-point weights must be finite");
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

// misfit + gradient over the selected (frequency, source) pairs, element type T
template <typename T>
helm_status misfit_gradient_t(helm_ctx* ctx, const helm_grid* g, const void* m, int nfreq, const double* omega,
                              int nsrc, const int32_t* src_idx, const double* src_amp, const uint8_t* mask,
                              int nrec, const int32_t* rec_idx, const void* d, double* f, void* grad,
                              void* u_store, int flags, const helm::SolveOpts& o, helm_solve_info* info,
                              void* caller) {
  using namespace helm;
  hipStream_t st = solve_stream(ctx, caller);
  const int64_t N = (int64_t)g->n[0] * g->n[1] * g->n[2];
  const int64_t plane = (int64_t)g->n[1] * g->n[2];
  auto lin = [&](const int32_t* p) { return (int64_t)p[0] * plane + (int64_t)p[1] * g->n[2] + p[2]; };
  const bool fwd_only = (flags & HELM_MG_FORWARD_ONLY) != 0;
  const bool reuse = (flags & HELM_MG_REUSE_U) != 0;
  const bool acc = (flags & HELM_MG_ACCUMULATE) != 0;
  const bool u64 = (flags & HELM_MG_U_FP64) != 0 && sizeof(T) == 4;
  const int nall = nfreq * nsrc;
  if (info)
    for (int k = 0; k < 2 * nall; ++k) to_info(SolveInfo(), info + k);
  // the selected pairs, frequency-major; row = f * nsrc + s
  std::vector<int> prow;
  for (int k = 0; k < nall; ++k)
    if (!mask || mask[k]) prow.push_back(k);
  const int np = (int)prow.size();
  if (np == 0) {
    *f = 0.0;
    if (!fwd_only && !acc) HELM_HIP_CHECK(hipMemsetAsync(grad, 0, (size_t)N * sizeof(T), st));
    HELM_HIP_CHECK(hipStreamSynchronize(st));
    return HELM_OK;
  }
  const double scale = (flags & HELM_MG_RENORMALISE) ? 1.0 / np : 1.0;
  // host tables per pair
  std::vector<int64_t> src_lin(np), drow(np), uoff_int(np), uoff_store(np);
  std::vector<double2> amp(np);
  std::vector<double> wgt(np);
  std::vector<ProblemSpec> probs;
  for (int p = 0; p < np; ++p) {
    const int fi = prow[p] / nsrc, s = prow[p] % nsrc;
    src_lin[p] = lin(src_idx + 3 * s);
    const double* a = src_amp ? src_amp + 2 * (size_t)prow[p] : nullptr;
    amp[p] = a ? make_double2(a[0], a[1]) : make_double2(1.0, 0.0);
    drow[p] = prow[p];
    uoff_int[p] = (int64_t)p * N;
    uoff_store[p] = (int64_t)prow[p] * N;
    wgt[p] = omega[fi] * omega[fi] * scale;
    probs.push_back(shared_problems(g, m, omega[fi], 0, 1)[0]);
  }
  std::vector<int64_t> rec_lin(nrec);
  for (int k = 0; k < nrec; ++k) rec_lin[k] = lin(rec_idx + 3 * k);
  // distinct receiver nodes, ascending, each with its receivers in order
  std::vector<int> order(nrec);
  for (int k = 0; k < nrec; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return rec_lin[a] < rec_lin[b]; });
  std::vector<int64_t> node_lin;
  std::vector<int> node_ptr, node_rec(nrec);
  for (int e = 0; e < nrec; ++e) {
    const int k = order[e];
    if (node_lin.empty() || node_lin.back() != rec_lin[k]) {
      node_lin.push_back(rec_lin[k]);
      node_ptr.push_back(e);
    }
    node_rec[e] = k;
  }
  node_ptr.push_back(nrec);
  const int nnode = (int)node_lin.size();
  // Device scratch: Q (sources, then adjoint sources), V, and U unless the
  // solve writes the caller's u_store directly (every pair selected, fields
  // stored in the dtype).
  const size_t fbytes = (size_t)np * N * sizeof(cx<T>);
  const bool direct_u = u_store && !u64 && np == nall;
  const bool own_u = !reuse && !direct_u;
  ctx->fwi_buf.ensure(fbytes * (own_u ? 3 : 2));
  char* base = (char*)ctx->fwi_buf.p;
  cx<T>* Q = (cx<T>*)base;
  cx<T>* V = (cx<T>*)(base + fbytes);
  cx<T>* U = direct_u ? (cx<T>*)u_store : own_u ? (cx<T>*)(base + 2 * fbytes) : nullptr;
  const int rblk = (int)ceil_div(nrec, 256);
  auto r256 = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t small = 4 * r256(np * sizeof(int64_t)) + r256(np * sizeof(double2)) + r256(np * sizeof(double)) +
                       r256(nrec * sizeof(int64_t)) + r256((size_t)np * nrec * sizeof(cx<T>)) +
                       r256((size_t)np * rblk * sizeof(double)) + r256(nnode * sizeof(int64_t)) +
                       r256((nnode + 1) * sizeof(int)) + r256(nrec * sizeof(int));
  ctx->fwi_small.ensure(small);
  char* sp = (char*)ctx->fwi_small.p;
  char* const sp_end = sp + small;
  auto carve = [&](size_t b) {
    char* p = sp;
    sp += r256(b);
    if (sp > sp_end) throw Error{-3, "internal: misfit scratch layout overflow"};
    return (void*)p;
  };
  int64_t* d_src = (int64_t*)carve(np * sizeof(int64_t));
  int64_t* d_drow = (int64_t*)carve(np * sizeof(int64_t));
  int64_t* d_uoff_int = (int64_t*)carve(np * sizeof(int64_t));
  int64_t* d_uoff_store = (int64_t*)carve(np * sizeof(int64_t));
  double2* d_amp = (double2*)carve(np * sizeof(double2));
  double* d_w = (double*)carve(np * sizeof(double));
  int64_t* d_rec = (int64_t*)carve(nrec * sizeof(int64_t));
  cx<T>* d_res = (cx<T>*)carve((size_t)np * nrec * sizeof(cx<T>));
  double* d_part = (double*)carve((size_t)np * rblk * sizeof(double));
  int64_t* d_node = (int64_t*)carve(nnode * sizeof(int64_t));
  int* d_nptr = (int*)carve((nnode + 1) * sizeof(int));
  int* d_nrec = (int*)carve(nrec * sizeof(int));
  auto up = [&](void* dst, const void* src, size_t b) {
    HELM_HIP_CHECK(hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, st));
  };
  up(d_src, src_lin.data(), np * sizeof(int64_t));
  up(d_drow, drow.data(), np * sizeof(int64_t));
  up(d_uoff_int, uoff_int.data(), np * sizeof(int64_t));
  up(d_uoff_store, uoff_store.data(), np * sizeof(int64_t));
  up(d_amp, amp.data(), np * sizeof(double2));
  up(d_w, wgt.data(), np * sizeof(double));
  up(d_rec, rec_lin.data(), nrec * sizeof(int64_t));
  up(d_node, node_lin.data(), nnode * sizeof(int64_t));
  up(d_nptr, node_ptr.data(), (nnode + 1) * sizeof(int));
  up(d_nrec, node_rec.data(), nrec * sizeof(int));

  Solver<T>& S = solver_for<T>(ctx, probs, o, st);
  std::vector<SolveInfo> inf(np);
  int worst = 0;
  const unsigned fb = std::min<unsigned>(65536, ceil_div((int64_t)np * N, 256));
  // where the gradient reads the forward fields: (pointer, per-pair offsets, FP64?)
  const void* ug = U;
  const int64_t* ug_off = d_uoff_int;
  bool ug64 = false;
  if (!reuse) {
    const double inv_h3 = 1.0 / (g->h * g->h * g->h);
    hipLaunchKernelGGL((k_point_sources<T>), dim3(std::min<unsigned>(DOT_BLOCKS, ceil_div(N, 256)), np), dim3(256),
                       0, st, Q, N, (const int64_t*)d_src, (const double2*)d_amp, inv_h3);
    worst = std::max(worst, S.solve(0, Q, U, inf.data()));
    if (info)
      for (int p = 0; p < np; ++p) to_info(inf[p], info + prow[p]);
    if (u64) {  // keep the FP64 iterates as the stored fields
      if (np == nall) {
        hipLaunchKernelGGL((k_convert<double, double>), dim3(fb), dim3(256), 0, st, S.iterate(),
                           (cx<double>*)u_store, N * np);
      } else {
        const unsigned pb = std::min<unsigned>(65536, ceil_div(N, 256));
        for (int p = 0; p < np; ++p)
          hipLaunchKernelGGL((k_convert<double, double>), dim3(pb), dim3(256), 0, st, S.iterate() + p * N,
                             (cx<double>*)u_store + prow[p] * N, N);
      }
      ug = u_store;
      ug_off = d_uoff_store;
      ug64 = true;
    } else if (u_store && !direct_u) {
      for (int p = 0; p < np; ++p)
        HELM_HIP_CHECK(hipMemcpyAsync((cx<T>*)u_store + prow[p] * N, U + p * N, N * sizeof(cx<T>),
                                      hipMemcpyDeviceToDevice, st));
    }
    hipLaunchKernelGGL((k_sample_residual<double, T>), dim3(rblk, np), dim3(256), 0, st, S.iterate(),
                       (const int64_t*)d_uoff_int, (const int64_t*)d_rec, nrec, (const cx<T>*)d,
                       (const int64_t*)d_drow, d_res, d_part);
  } else {
    ug = u_store;
    ug_off = d_uoff_store;
    ug64 = u64;
    if (u64)
      hipLaunchKernelGGL((k_sample_residual<double, T>), dim3(rblk, np), dim3(256), 0, st,
                         (const cx<double>*)u_store, (const int64_t*)d_uoff_store, (const int64_t*)d_rec, nrec,
                         (const cx<T>*)d, (const int64_t*)d_drow, d_res, d_part);
    else
      hipLaunchKernelGGL((k_sample_residual<T, T>), dim3(rblk, np), dim3(256), 0, st, (const cx<T>*)u_store,
                         (const int64_t*)d_uoff_store, (const int64_t*)d_rec, nrec, (const cx<T>*)d,
                         (const int64_t*)d_drow, d_res, d_part);
  }
  std::vector<double> hpart((size_t)np * rblk);
  HELM_HIP_CHECK(hipMemcpyAsync(hpart.data(), d_part, hpart.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HELM_HIP_CHECK(hipStreamSynchronize(st));
  double fsum = 0.0;
  for (size_t i = 0; i < hpart.size(); ++i) fsum += hpart[i];
  *f = 0.5 * fsum * scale;
  if (fwd_only) return (helm_status)worst;
  // adjoint sources b_p = -P_r^T r_p, then H^H v_p = b_p
  hipLaunchKernelGGL((k_fill_zero<T>), dim3(fb), dim3(256), 0, st, Q, (int64_t)np * N);
  hipLaunchKernelGGL((k_adjoint_source<T>), dim3(ceil_div(nnode, 256), np), dim3(256), 0, st, Q, N,
                     (const int64_t*)d_node, (const int*)d_nptr, (const int*)d_nrec, nnode, (const cx<T>*)d_res,
                     nrec);
  worst = std::max(worst, S.solve(1, Q, V, inf.data()));
  if (info)
    for (int p = 0; p < np; ++p) to_info(inf[p], info + nall + prow[p]);
  // gradient
  const unsigned gb = std::min<unsigned>(4096, ceil_div(N, 256));
  const bool m27 = g->stencil == HELM_27PT;
  const double mw[4] = {m27 ? g->w27[3] : 1.0, m27 ? g->w27[4] : 0.0, m27 ? g->w27[5] : 0.0,
                        m27 ? g->w27[6] : 0.0};
#define HELM_GRAD(TU, M27)                                                                                \
  hipLaunchKernelGGL((k_gradient<TU, T, T, M27>), dim3(gb), dim3(256), 0, st, (const cx<TU>*)ug, ug_off,  \
                     (const cx<T>*)V, np, g->n[0], g->n[1], g->n[2], (const double*)d_w, mw[0], mw[1], mw[2], \
                     mw[3], (T*)grad, acc)
  if (ug64) {
    if (m27) HELM_GRAD(double, true);
    else HELM_GRAD(double, false);
  } else {
    if (m27) HELM_GRAD(T, true);
    else HELM_GRAD(T, false);
  }
#undef HELM_GRAD
  HELM_HIP_CHECK(hipGetLastError());
  HELM_HIP_CHECK(hipStreamSynchronize(st));
  return (helm_status)worst;
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
    check_grid(g);
    HELM_REQUIRE(m && x && y, "null device pointer");
    HELM_REQUIRE(omega > 0.0 && std::isfinite(omega), "omega must be positive");
    HELM_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    HELM_REQUIRE(x != y, "x and y must not overlap");
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
    check_grid(g);
    HELM_REQUIRE(m && q && u, "null device pointer");
    HELM_REQUIRE(omega > 0.0 && std::isfinite(omega), "omega must be positive");
    HELM_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    const helm::SolveOpts so = opts_of(o);
    check_coarse_sizes(g, so);
    if (g->dtype == HELM_C64) return solve_t<float>(ctx, g, m, omega, adjoint ? 1 : 0, nrhs, q, u, so, info, stream);
    return solve_t<double>(ctx, g, m, omega, adjoint ? 1 : 0, nrhs, q, u, so, info, stream);
  });
}

helm_status helm_solve_batched(helm_ctx* ctx, int nprob, const helm_problem* probs, int adjoint,
                               const helm_solver_opts* o, helm_solve_info* info, void* stream) {
  return guarded(ctx, [&]() -> helm_status {
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
    check_grid(g);
    HELM_REQUIRE(m && d && f, "null pointer argument");
    HELM_REQUIRE(nfreq >= 1 && omega, "nfreq must be >= 1 with an omega array");
    for (int k = 0; k < nfreq; ++k)
      HELM_REQUIRE(omega[k] > 0.0 && std::isfinite(omega[k]), "omega must be positive");
    HELM_REQUIRE(nsrc >= 1 && nrec >= 1, "nsrc and nrec must be >= 1");
    HELM_REQUIRE((int64_t)nfreq * nsrc <= (1 << 20), "too many (frequency, source) pairs");
    HELM_REQUIRE(src_idx && rec_idx, "null source / receiver index array");
    HELM_REQUIRE((flags & HELM_MG_FORWARD_ONLY) || grad, "null gradient");
    HELM_REQUIRE(!(flags & HELM_MG_REUSE_U) || u_store, "HELM_MG_REUSE_U needs u_store");
    HELM_REQUIRE(!(flags & HELM_MG_U_FP64) || u_store, "HELM_MG_U_FP64 needs u_store");
    HELM_REQUIRE((flags & ~31) == 0, "unknown flag bits");
    for (int s = 0; s < nsrc; ++s)
      for (int a = 0; a < 3; ++a)
        HELM_REQUIRE(src_idx[3 * s + a] >= 0 && src_idx[3 * s + a] < g->n[a], "source outside the grid");
    for (int k = 0; k < nrec; ++k)
      for (int a = 0; a < 3; ++a)
        HELM_REQUIRE(rec_idx[3 * k + a] >= 0 && rec_idx[3 * k + a] < g->n[a], "receiver outside the grid");
    const helm::SolveOpts so = opts_of(o);
    check_coarse_sizes(g, so);
    if (g->dtype == HELM_C64)
      return misfit_gradient_t<float>(ctx, g, m, nfreq, omega, nsrc, src_idx, src_amp, mask, nrec, rec_idx, d, f,
                                      grad, u_store, flags, so, info, stream);
    return misfit_gradient_t<double>(ctx, g, m, nfreq, omega, nsrc, src_idx, src_amp, mask, nrec, rec_idx, d, f,
                                     grad, u_store, flags, so, info, stream);
  });
}

}  // extern "C"
