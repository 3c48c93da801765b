// Inversion driver (arXiv:1703.09268: the 2D inversion example -- frequency
// bands with overlap, a fixed number of box-constrained L-BFGS iterations
// per band, each band warm-started from the previous one, the
// source/frequency mask selecting the band -- and the stochastic inversion
// section -- per band, T draws of a uniformly random source subset I_k of
// size p, each approximately minimising the subset average of the misfit
// under m_LB <= m <= m_UB in r_sub ceil(N_s / p) iterations, warm-starting
// the next draw; p grows by a fixed amount after a failed line search).
// Host-side control flow only: every vector operation is a kernel of
// lbfgs.hip, every objective and gradient a misfit_gradient_t call on the
// device-resident model.  Included by libhelm.hip inside its anonymous
// namespace.
//
// The paper uses an external bound-constrained quasi-Newton code without
// stating its steps; this one is a projected L-BFGS:
//   F = points not held at a bound by the gradient;
//   d = -H g over F (two-loop recursion on the restricted pairs, initial
//       scaling s.y / y.y of the newest pair), 0 elsewhere; d = -g_F step0 /
//       max|g_F| with no pair or when g.d >= 0;
//   stop when max|g_F| <= gtol * (its value at the subproblem's start);
//   x_t = clamp(x + t d), t = 1, 1/2, ... until f(x_t) <= f(x) + c1 g.(x_t - x)
//       (at most max_ls trials; a failed search ends the subproblem);
//   the pair (x_t - x, g_t - g) is kept when s.y > 1e-10 |s| |y|.
// Source subsets: a partial Fisher-Yates shuffle whose swap at step i takes
// i + (u mod (N_s - i)), u the next SplitMix64 output (one counter over the
// whole run; a draw of every source uses none), sorted ascending.

uint64_t splitmix64(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

std::vector<std::vector<int>> freq_bands(int nfreq, int size, int overlap) {
  std::vector<std::vector<int>> out;
  for (int b = 0;; b += size - overlap) {
    std::vector<int> band;
    for (int f = b; f < std::min(b + size, nfreq); ++f) band.push_back(f);
    out.push_back(band);
    if (b + size >= nfreq) return out;
  }
}

int fwi_band_count(int nfreq, int size, int overlap) { return (int)freq_bands(nfreq, size, overlap).size(); }

void check_fwi_params(const helm_fwi_params* p) {
  HELM_REQUIRE(p, "null parameter struct");
  HELM_REQUIRE(p->band_size >= 1 && p->band_overlap >= 0 && p->band_overlap < p->band_size,
               "band_size >= 1 and 0 <= band_overlap < band_size");
  HELM_REQUIRE(p->r_sub >= 1, "r_sub must be >= 1");
  HELM_REQUIRE(p->memory >= 0 && p->memory <= helm::LB_MAXMEM, "memory must be in 0..16");
  HELM_REQUIRE(p->subproblems >= 1, "subproblems must be >= 1");
  HELM_REQUIRE(p->batch_increase >= 0, "batch_increase must be >= 0");
  HELM_REQUIRE(p->max_ls >= 1 && p->max_ls <= 60, "max_ls must be in 1..60");
  HELM_REQUIRE(p->c1 > 0.0 && p->c1 < 1.0, "c1 must be in (0, 1)");
  HELM_REQUIRE(p->gtol >= 0.0 && std::isfinite(p->gtol), "gtol must be >= 0");
  HELM_REQUIRE(p->step0 > 0.0 && std::isfinite(p->step0), "step0 must be positive");
  HELM_REQUIRE(!std::isnan(p->lo) && !std::isnan(p->hi), "NaN bound");
}

template <typename T>
helm_status fwi_t(helm_ctx* ctx, const helm_grid* g, void* m, const double* lo, const double* hi, int nfreq,
                  const double* omega, const PointSet& src, const double* src_amp, const PointSet& rec, const void* d,
                  const helm_fwi_params& p, const helm::SolveOpts& o, helm_fwi_draw* draws, int32_t* sources,
                  helm_fwi_record* recs, int rec_cap, int* nrec_out, void* caller) {
  using namespace helm;
  hipStream_t st = solve_stream(ctx, caller);
  const int64_t N = (int64_t)g->n[0] * g->n[1] * g->n[2];
  const int nsrc = src.n();
  const int nslot = p.memory + 1;  // one spare slot for the pair being formed
  const unsigned nb = std::min<unsigned>(LB_BLOCKS, ceil_div(N, 256));
  auto r256 = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t vb = r256((size_t)N * sizeof(double)), tb = r256((size_t)N * sizeof(T));
  const size_t pb = r256((size_t)nb * 2 * LB_MAXMEM * sizeof(double));
  const bool narrow = sizeof(T) != sizeof(double);  // the solves read a converted copy of the trial point
  ctx->drv_buf.ensure((4 + 2 * (size_t)nslot) * vb + (narrow ? 2 : 1) * tb + pb);
  char* base = (char*)ctx->drv_buf.p;
  double* x = (double*)base;
  double* gr = (double*)(base + vb);
  double* xt = (double*)(base + 2 * vb);
  double* q = (double*)(base + 3 * vb);
  std::vector<double*> S(nslot), Y(nslot);
  for (int k = 0; k < nslot; ++k) {
    S[k] = (double*)(base + (4 + 2 * (size_t)k) * vb);
    Y[k] = (double*)(base + (5 + 2 * (size_t)k) * vb);
  }
  char* tail = base + (4 + 2 * (size_t)nslot) * vb;
  T* gT = (T*)tail;
  T* mT = narrow ? (T*)(tail + tb) : nullptr;
  double* part = (double*)(tail + (narrow ? 2 : 1) * tb);
  const T* model = narrow ? mT : (const T*)xt;
  const Box bx{lo, hi, p.lo, p.hi};
  std::vector<double> hp((size_t)nb * 2 * LB_MAXMEM);

  // sums (or maxima) of `width` partials per workgroup, in workgroup order
  auto fetch = [&](int width) {
    HELM_HIP_CHECK(hipMemcpyAsync(hp.data(), part, (size_t)nb * width * sizeof(double), hipMemcpyDeviceToHost, st));
    HELM_HIP_CHECK(hipStreamSynchronize(st));
  };
  auto total = [&](int width, int k) {
    double s = 0.0;
    for (unsigned b = 0; b < nb; ++b) s += hp[(size_t)b * width + k];
    return s;
  };
  auto maximum = [&]() {
    double s = 0.0;
    for (unsigned b = 0; b < nb; ++b) s = std::max(s, hp[b]);
    return s;
  };
  auto update = [&](double c, const double* u, double scale, const double* w) {
    hipLaunchKernelGGL(k_lb_update, dim3(nb), dim3(256), 0, st, q, c, u, scale, w, (const double*)x,
                       (const double*)gr, bx, N, part);
    HELM_HIP_CHECK(hipGetLastError());
    if (!w) return 0.0;
    fetch(1);
    return total(1, 0);
  };
  auto start = [&]() {
    hipLaunchKernelGGL(k_lb_start, dim3(nb), dim3(256), 0, st, (const double*)x, (const double*)gr, bx, q, N, part);
    HELM_HIP_CHECK(hipGetLastError());
    fetch(1);
    return maximum();
  };

  hipLaunchKernelGGL((k_lb_init<T>), dim3(nb), dim3(256), 0, st, (const T*)m, bx, x, N, part);
  HELM_HIP_CHECK(hipGetLastError());
  fetch(1);
  HELM_REQUIRE(total(1, 0) == 0.0, "a lower bound lies above its upper bound (or is NaN)");

  const auto bands = freq_bands(nfreq, p.band_size, p.band_overlap);
  uint64_t counter = 0;
  int psz = (p.batch <= 0 || p.batch >= nsrc) ? nsrc : p.batch;
  int worst = 0, nrec = 0, ndraw = 0;
  std::vector<uint8_t> mask((size_t)nfreq * nsrc);
  for (int bi = 0; bi < (int)bands.size(); ++bi) {
    for (int t = 0; t < p.subproblems; ++t, ++ndraw) {
      const Range rdraw("helm fwi draw");
      std::vector<int> sel(nsrc);
      for (int i = 0; i < nsrc; ++i) sel[i] = i;
      if (psz < nsrc) {
        for (int i = 0; i < psz; ++i) {
          const int j = i + (int)(splitmix64(p.seed, counter++) % (uint64_t)(nsrc - i));
          std::swap(sel[i], sel[j]);
        }
        sel.resize(psz);
        std::sort(sel.begin(), sel.end());
      }
      std::fill(mask.begin(), mask.end(), 0);
      for (int fi : bands[bi])
        for (int s : sel) mask[(size_t)fi * nsrc + s] = 1;
      int evals = 0, dstatus = 0;
      auto evaluate = [&]() {
        double f = 0.0;
        const int s = misfit_gradient_t<T>(ctx, g, model, nfreq, omega, src, src_amp, mask.data(), rec, d, &f, gT,
                                           nullptr, HELM_MG_RENORMALISE, o, nullptr, st);
        ++evals;
        dstatus = std::max(dstatus, s);
        return f;
      };
      // objective and gradient of this draw at the current iterate
      hipLaunchKernelGGL((k_lb_trial<T>), dim3(nb), dim3(256), 0, st, (const double*)x, (const double*)nullptr, 0.0,
                         bx, xt, mT, (const double*)nullptr, N, part);
      HELM_HIP_CHECK(hipGetLastError());
      double f = evaluate();
      hipLaunchKernelGGL((k_lb_accept<T>), dim3(nb), dim3(256), 0, st, x, gr, (const double*)xt, (const T*)gT,
                         (double*)nullptr, (double*)nullptr, N, part);
      HELM_HIP_CHECK(hipGetLastError());
      const double f_start = f;
      const int nit = p.r_sub * (int)ceil_div(nsrc, psz);
      std::vector<int> order;  // slots of the stored pairs, newest first
      double g0max = -1.0;
      bool failed = false;
      int it = 0;
      for (; it < nit; ++it) {
        const double gmax = start();
        if (g0max < 0.0) g0max = gmax;
        if (gmax == 0.0 || gmax <= p.gtol * g0max) break;
        double gd = 0.0;
        bool have_dir = false;
        const int np = (int)order.size();
        if (np > 0) {
          PairPtrs pp{};
          for (int k = 0; k < np; ++k) {
            pp.s[k] = S[order[k]];
            pp.y[k] = Y[order[k]];
          }
          hipLaunchKernelGGL(k_lb_pair_dots, dim3(nb), dim3(256), 0, st, pp, np, (const double*)x,
                             (const double*)gr, bx, N, part);
          HELM_HIP_CHECK(hipGetLastError());
          fetch(2 * LB_MAXMEM);
          std::vector<double> rho(np), a(np);
          for (int k = 0; k < np; ++k) {
            const double sy = total(2 * LB_MAXMEM, 2 * k);
            rho[k] = sy != 0.0 ? 1.0 / sy : 0.0;
          }
          const double sy0 = total(2 * LB_MAXMEM, 0), yy0 = total(2 * LB_MAXMEM, 1);
          const double gamma = yy0 > 0.0 ? sy0 / yy0 : 1.0;
          // newest to oldest: a_k = rho_k s_k.q, q -= a_k y_k; then r = gamma q
          a[0] = rho[0] * update(0.0, nullptr, 1.0, pp.s[0]);
          double b = 0.0;
          for (int k = 0; k < np; ++k) {
            if (k + 1 < np) a[k + 1] = rho[k + 1] * update(-a[k], pp.y[k], 1.0, pp.s[k + 1]);
            else b = rho[np - 1] * update(-a[k], pp.y[k], gamma, pp.y[np - 1]);
          }
          // oldest to newest: r += (a_k - rho_k y_k.r) s_k; then d = -r
          for (int k = np - 1; k >= 0; --k) {
            if (k > 0) b = rho[k - 1] * update(a[k] - b, pp.s[k], 1.0, pp.y[k - 1]);
            else gd = update(a[0] - b, pp.s[0], -1.0, gr);
          }
          have_dir = gd < 0.0;
        }
        if (!have_dir) {
          start();
          gd = update(0.0, nullptr, -p.step0 / gmax, gr);
        }
        // backtracking on the projected path
        double tt = 1.0, ft = 0.0;
        bool accepted = false;
        int trial = 1;
        for (; trial <= p.max_ls; ++trial) {
          hipLaunchKernelGGL((k_lb_trial<T>), dim3(nb), dim3(256), 0, st, (const double*)x, (const double*)q, tt, bx,
                             xt, mT, (const double*)gr, N, part);
          HELM_HIP_CHECK(hipGetLastError());
          fetch(1);
          const double gdx = total(1, 0);
          ft = evaluate();
          if (ft <= f + p.c1 * gdx) {
            accepted = true;
            break;
          }
          tt *= 0.5;
        }
        if (recs && nrec < rec_cap) {
          helm_fwi_record& r = recs[nrec];
          r.band = bi;
          r.draw = t;
          r.iter = it;
          r.nsel = (int)sel.size();
          r.trials = std::min(trial, p.max_ls);
          r.accepted = accepted ? 1 : 0;
          r.status = dstatus;
          r.pad_ = 0;
          r.f = f;
          r.f_new = ft;
          r.step = tt;
          r.pgmax = gmax;
        }
        ++nrec;
        if (!accepted) {
          failed = true;
          break;
        }
        int slot = 0;
        while (std::find(order.begin(), order.end(), slot) != order.end()) ++slot;
        hipLaunchKernelGGL((k_lb_accept<T>), dim3(nb), dim3(256), 0, st, x, gr, (const double*)xt, (const T*)gT,
                           S[slot], Y[slot], N, part);
        HELM_HIP_CHECK(hipGetLastError());
        fetch(3);
        const double sy = total(3, 0), ss = total(3, 1), yy = total(3, 2);
        if (sy > 1e-10 * std::sqrt(ss) * std::sqrt(yy)) {
          order.insert(order.begin(), slot);
          if ((int)order.size() > p.memory) order.pop_back();
        }
        f = ft;
      }
      if (draws) {
        helm_fwi_draw& dr = draws[ndraw];
        dr.band = bi;
        dr.draw = t;
        dr.nsel = (int)sel.size();
        dr.max_iters = nit;
        dr.iters = failed ? it + 1 : it;
        dr.failed = failed ? 1 : 0;
        dr.evals = evals;
        dr.status = dstatus;
        dr.f_start = f_start;
        dr.f_end = f;
      }
      if (sources)
        for (int i = 0; i < nsrc; ++i) sources[(size_t)ndraw * nsrc + i] = i < (int)sel.size() ? sel[i] : -1;
      worst = std::max(worst, dstatus);
      if (failed) psz = std::min(nsrc, psz + p.batch_increase);
    }
  }
  hipLaunchKernelGGL((k_lb_store<T>), dim3(nb), dim3(256), 0, st, (const double*)x, (T*)m, N);
  HELM_HIP_CHECK(hipGetLastError());
  HELM_HIP_CHECK(hipEventRecord(ctx->ev, st));
  HELM_HIP_CHECK(hipStreamWaitEvent((hipStream_t)caller, ctx->ev, 0));
  HELM_HIP_CHECK(hipStreamSynchronize(st));
  if (nrec_out) *nrec_out = nrec;
  return (helm_status)worst;
}

helm_status fwi_common(helm_ctx* ctx, const helm_grid* g, void* m, const double* lo, const double* hi, int nfreq,
                       const double* omega, const PointSet& src, const double* src_amp, const PointSet& rec,
                       const void* d, const helm_fwi_params* p, const helm_solver_opts* o, helm_fwi_draw* draws,
                       int32_t* sources, helm_fwi_record* recs, int rec_cap, int* nrec_out, void* stream) {
  HELM_REQUIRE(d, "null data pointer");
  check_fwi_params(p);
  HELM_REQUIRE(rec_cap >= 0, "negative record capacity");
  const helm::SolveOpts so = opts_of(o);
  check_coarse_sizes(g, so);
  if (g->dtype == HELM_C64)
    return fwi_t<float>(ctx, g, m, lo, hi, nfreq, omega, src, src_amp, rec, d, *p, so, draws, sources, recs, rec_cap,
                        nrec_out, stream);
  return fwi_t<double>(ctx, g, m, lo, hi, nfreq, omega, src, src_amp, rec, d, *p, so, draws, sources, recs, rec_cap,
                       nrec_out, stream);
}
