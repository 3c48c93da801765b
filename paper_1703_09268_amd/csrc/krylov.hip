// Krylov building blocks for restarted (F)GMRES on many segments at once
// (all sources of a frequency, or a batch of uneven problems; each segment
// keeps its own Krylov state).  Every scalar of the method (Hessenberg
// entries, Givens rotations, residual estimates, basis scales) stays on the
// device; sums are accumulated in FP64 with a fixed reduction order, so
// results are bitwise reproducible run to run.
//
// Orthogonalisation is classical Gram-Schmidt in two kernels (all inner
// products of a column in one pass over the basis, then one fused
// "w -= sum c_i V_i; ||w||^2" pass), with lazy normalisation: basis vector
// V_i is stored unnormalised together with scale_i = 1/||V_i|| per segment,
// and consumers fold the scale into their first use.
//
// Vector kernels run vnblk workgroups per segment (grid-stride over the
// segment's N); partial sums of workgroup wg go to part[wg * PSTRIDE + ...];
// the per-segment reducers (one 64-lane workgroup per segment) read the
// segment's range of workgroups in a fixed order.
#pragma once

#include "common.h"
#include "segment.h"

namespace helm {

constexpr int DOT_BLOCKS = 240;        // default cap of vector workgroups per segment
constexpr int DOT_BLOCKS_MAX = 4096;   // hard cap (reducers loop over any count)

// Up to KMAX+1 vector pointers (element Seg::off + p of each).
template <typename T>
struct VecList {
  const cx<T>* v[KMAX + 1];
};

// Device-resident state of one (F)GMRES instance, structure of arrays over
// segments: entry [idx][s] is at idx*nseg + s.
struct KState {
  double2* H;     // (KMAX+1) x KMAX Hessenberg / R factor, [(i*KMAX+j)][s]
  double* cs;     // Givens cosines [j][s]
  double2* sn;    // Givens sines   [j][s]
  double2* g;     // rotated right-hand side [i][s]
  double* scale;  // 1/||V_i|| [i][s]
  double2* coef;  // CGS coefficients of the current column, scale folded in
  double* part;   // partial sums scratch [wg][PSTRIDE]
  int nseg;
};

// which workgroup range of a segment holds the partial sums being reduced
enum PartRange { PR_STENCIL = 0, PR_VECTOR = 1, PR_POINT = 2 };

__device__ __forceinline__ void seg_range(const Seg& S, int which, int& b0, int& nb) {
  if (which == PR_STENCIL) { b0 = S.sblk0; nb = S.snblk; }
  else if (which == PR_VECTOR) { b0 = S.vblk0; nb = S.vnblk; }
  else { b0 = S.tblk0; nb = S.tnblk; }
}

__device__ __forceinline__ double2 d2(double a, double b) { return make_double2(a, b); }

// Column sums s[c] = sum_b part[(b0+b)*PSTRIDE + c], c < NC (c < nc unless
// EXACT), over the segment's workgroups, by one 256-lane workgroup.  Every
// lane issues the loads of all its rows and columns before adding, so the
// reduction costs one memory round trip; lanes add their rows in increasing
// order and the four wave totals are added in a fixed order (deterministic).
// The result is valid in every lane.  `red` holds 4*NC doubles of LDS.
template <int NC, bool EXACT>
__device__ __forceinline__ void seg_sums(const double* __restrict__ part, int b0, int nb, int nc,
                                         double (&s)[NC], double* red) {
#pragma unroll
  for (int c = 0; c < NC; ++c) s[c] = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    const double* row = part + (int64_t)(b0 + b) * PSTRIDE;
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (EXACT || c < nc) s[c] += row[c];
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double v = wave_sum(s[c]);
    if (lane == 0) red[wid * NC + c] = v;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NC; ++c) s[c] = red[c] + red[NC + c] + red[2 * NC + c] + red[3 * NC + c];
}

// single column 0
__device__ __forceinline__ double seg_sum0(const double* __restrict__ part, int b0, int nb, double* red) {
  double s[1];
  seg_sums<1, true>(part, b0, nb, 1, s, red);
  return s[0];
}

// ---------------------------------------------------------------------------
// partial inner products  s_i = sum_p conj(V_i[p]) w[p],  i < nv
// ---------------------------------------------------------------------------
// NV = NVMAX exactly when EXACT (no per-vector guards, so every load of an
// element is in flight at once); otherwise nv <= NVMAX.  Each lane visits
// its elements in increasing order two at a time.
template <typename T, int NVMAX, bool EXACT>
__global__ __launch_bounds__(256) void k_dots(const Seg* __restrict__ segs, const int* __restrict__ vmap,
                                             VecList<T> V, int nv, const cx<T>* __restrict__ w,
                                             double* __restrict__ part, const int* __restrict__ active) {
  __shared__ double red[4][2 * NVMAX];
  const int wg = blockIdx.x;
  const int sid = vmap[wg];
  const Seg& S = segs[sid];
  double* out = part + (int64_t)wg * PSTRIDE;
  if (EXACT) nv = NVMAX;
  if (active && !active[sid]) {
    if (threadIdx.x < 2 * nv) out[threadIdx.x] = 0.0;
    return;
  }
  double ar[NVMAX], ai[NVMAX];
#pragma unroll
  for (int i = 0; i < NVMAX; ++i) ar[i] = ai[i] = 0.0;
  const int64_t N = S.N, off = S.off;
  const int64_t stride = (int64_t)S.vnblk * 256;
  auto acc = [&](const cx<T>& wv, const cx<T>* a) {
#pragma unroll
    for (int i = 0; i < NVMAX; ++i) {
      if (EXACT || i < nv) {
        ar[i] += (double)a[i].re * (double)wv.re + (double)a[i].im * (double)wv.im;
        ai[i] += (double)a[i].re * (double)wv.im - (double)a[i].im * (double)wv.re;
      }
    }
  };
  int64_t p = (int64_t)(wg - S.vblk0) * 256 + threadIdx.x;
  if (EXACT) {  // two elements per iteration: twice the loads in flight
    for (; p + stride < N; p += 2 * stride) {
      const cx<T> w0 = w[off + p], w1 = w[off + p + stride];
      cx<T> a0[NVMAX], a1[NVMAX];
#pragma unroll
      for (int i = 0; i < NVMAX; ++i) {
        if (EXACT || i < nv) {
          a0[i] = V.v[i][off + p];
          a1[i] = V.v[i][off + p + stride];
        }
      }
      acc(w0, a0);
      acc(w1, a1);
    }
  }
  for (; p < N; p += stride) {
    const cx<T> w0 = w[off + p];
    cx<T> a0[NVMAX];
#pragma unroll
    for (int i = 0; i < NVMAX; ++i)
      if (EXACT || i < nv) a0[i] = V.v[i][off + p];
    acc(w0, a0);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NVMAX; ++i) {
    if (EXACT || i < nv) {
      const double sr = wave_sum(ar[i]);
      const double si = wave_sum(ai[i]);
      if (lane == 0) {
        red[wid][2 * i] = sr;
        red[wid][2 * i + 1] = si;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * nv)
    out[threadIdx.x] = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

// 1/||w|| from ||w||^2 (0 on breakdown)
__device__ __forceinline__ double basis_scale(double s) {
  const double hn = sqrt(s);
  return hn > 0.0 ? 1.0 / hn : 0.0;
}

// Finish Arnoldi column j of segment sid from s = ||w||^2 (sum of the
// partials): h_{j+1,j} = sqrt(s); apply the previous rotations to column j,
// build rotation j, update g, set scale_{j+1} = 1/h_{j+1,j} (0 on
// breakdown).  The whole workgroup first stages what this needs in LDS
// (givens_stage: one memory round trip; a single thread's loads would each
// wait behind its stores to the same arrays), then one thread finishes it
// (givens_finish), leaving the rotated column and g_j in the stage.
struct GivensStage {
  double2 col[KMAX + 1];  // H[0..j][j]
  double cs[KMAX];
  double2 sn[KMAX];
  double2 g[KMAX + 1];    // g_0..g_j
};

// all threads; a barrier must follow before givens_finish
__device__ __forceinline__ void givens_stage(const KState& st, int sid, int j, int gcount, GivensStage& G) {
  const int ns = st.nseg;
  const int t = threadIdx.x;
  if (t <= j) G.col[t] = st.H[(t * KMAX + j) * ns + sid];
  if (t < j) {
    G.cs[t] = st.cs[t * ns + sid];
    G.sn[t] = st.sn[t * ns + sid];
  }
  if (t < gcount) G.g[t] = st.g[t * ns + sid];  // gcount >= j + 1
}

// one thread
__device__ __forceinline__ void givens_finish(const KState& st, int sid, int j, double s, GivensStage& G) {
  const int ns = st.nseg;
  const double hn = sqrt(s);
  for (int i = 0; i < j; ++i) {
    const double2 a = G.col[i];
    const double2 b = G.col[i + 1];
    const double c = G.cs[i];
    const double2 sn = G.sn[i];
    // [c, s; -conj(s), c] [a; b]
    G.col[i] = d2(c * a.x + (sn.x * b.x - sn.y * b.y), c * a.y + (sn.x * b.y + sn.y * b.x));
    G.col[i + 1] = d2(-(sn.x * a.x + sn.y * a.y) + c * b.x, -(sn.x * a.y - sn.y * a.x) + c * b.y);
  }
  const double2 a = G.col[j];
  const double absa = hypot(a.x, a.y);
  double c;
  double2 sn, rr;
  if (hn == 0.0) {
    c = 1.0;
    sn = d2(0.0, 0.0);
    rr = a;
  } else if (absa == 0.0) {
    c = 0.0;
    sn = d2(1.0, 0.0);  // conj(b)/|b| with b = hn real
    rr = d2(hn, 0.0);
  } else {
    const double nrm = hypot(absa, hn);
    c = absa / nrm;
    const double2 ph = d2(a.x / absa, a.y / absa);
    sn = d2(ph.x * hn / nrm, ph.y * hn / nrm);  // (a/|a|) conj(b)/nrm, b real
    rr = d2(ph.x * nrm, ph.y * nrm);
  }
  G.col[j] = rr;
  for (int i = 0; i <= j; ++i) st.H[(i * KMAX + j) * ns + sid] = G.col[i];
  st.H[((j + 1) * KMAX + j) * ns + sid] = d2(0.0, 0.0);
  st.cs[j * ns + sid] = c;
  st.sn[j * ns + sid] = sn;
  const double2 gj = G.g[j];
  // g_{j+1} = -conj(s) g_j ; g_j = c g_j
  const double2 g1 = d2(-(sn.x * gj.x + sn.y * gj.y), -(sn.x * gj.y - sn.y * gj.x));
  G.g[j] = d2(c * gj.x, c * gj.y);
  st.g[(j + 1) * ns + sid] = g1;
  st.g[j * ns + sid] = G.g[j];
  st.scale[(j + 1) * ns + sid] = basis_scale(s);
}

// One workgroup per segment: H[i][j] = scale_i * sum of partials (of the
// workgroup range `which`: the vector pass or the fused stencil pass),
// coef_i = H[i][j] * scale_i.
// With gprev >= 0 the deferred Givens step of column gprev (= j - 1) runs
// first, from the partial norms in the vector range of st.part; the
// inner-product partials come from `src` (range `which`).
template <int NVMAX, bool EXACT>
__global__ __launch_bounds__(256) void k_reduce_dots(const Seg* __restrict__ segs, KState st, int nv, int j,
                                                     int which, const double* __restrict__ src, int gprev,
                                                     const int* __restrict__ active) {
  __shared__ double red[4 * 2 * NVMAX > 4 ? 4 * 2 * NVMAX : 4];
  __shared__ GivensStage G;
  __shared__ double scl[NVMAX];
  const int sid = blockIdx.x;
  if (active && !active[sid]) return;
  const Seg& S = segs[sid];
  const int ns = st.nseg;
  if (EXACT) nv = NVMAX;
  // the basis scales, loaded together (scale_j is set by the deferred step)
  if ((int)threadIdx.x < nv) scl[threadIdx.x] = st.scale[threadIdx.x * ns + sid];
  if (gprev >= 0) {
    givens_stage(st, sid, gprev, gprev + 1, G);
    const double sn = seg_sum0(st.part, S.vblk0, S.vnblk, red);  // (its barriers order the stage)
    if (threadIdx.x == 0) {
      givens_finish(st, sid, gprev, sn, G);
      scl[gprev + 1] = basis_scale(sn);
    }
  }
  __syncthreads();  // red is reused below; scl complete
  int b0, nb;
  seg_range(S, which, b0, nb);
  double s[2 * NVMAX];
  seg_sums<2 * NVMAX, EXACT>(src, b0, nb, 2 * nv, s, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NVMAX; ++i) {
      if (EXACT || i < nv) {
        const double sc = scl[i];
        const double2 h = d2(sc * s[2 * i], sc * s[2 * i + 1]);
        st.H[(i * KMAX + j) * ns + sid] = h;
        st.coef[i * ns + sid] = d2(h.x * sc, h.y * sc);
      }
    }
  }
}

// w <- w - sum_i coef_i V_i  (in place), partial ||w||^2 per workgroup.
template <typename T, int NVMAX, bool EXACT>
__global__ __launch_bounds__(256) void k_axpy_norm(const Seg* __restrict__ segs, const int* __restrict__ vmap,
                                                  VecList<T> V, int nv, cx<T>* __restrict__ w, KState st,
                                                  const int* __restrict__ active) {
  __shared__ double red[16];
  const int wg = blockIdx.x;
  const int sid = vmap[wg];
  const Seg& S = segs[sid];
  double* out = st.part + (int64_t)wg * PSTRIDE;
  if (active && !active[sid]) {
    if (threadIdx.x == 0) out[0] = 0.0;
    return;
  }
  if (EXACT) nv = NVMAX;
  cx<T> c[NVMAX];
#pragma unroll
  for (int i = 0; i < NVMAX; ++i) {
    if (EXACT || i < nv) {
      const double2 q = st.coef[i * st.nseg + sid];
      c[i] = mk<T>((T)q.x, (T)q.y);
    }
  }
  const int64_t N = S.N, off = S.off;
  const int64_t stride = (int64_t)S.vnblk * 256;
  double nrm = 0.0;
  auto upd = [&](cx<T> acc, const cx<T>* a) {
#pragma unroll
    for (int i = 0; i < NVMAX; ++i)
      if (EXACT || i < nv) acc = acc - c[i] * a[i];
    return acc;
  };
  int64_t p = (int64_t)(wg - S.vblk0) * 256 + threadIdx.x;
  if (EXACT) {  // two elements per iteration: twice the loads in flight
    for (; p + stride < N; p += 2 * stride) {
      const cx<T> w0 = w[off + p], w1 = w[off + p + stride];
      cx<T> a0[NVMAX], a1[NVMAX];
#pragma unroll
      for (int i = 0; i < NVMAX; ++i) {
        if (EXACT || i < nv) {
          a0[i] = V.v[i][off + p];
          a1[i] = V.v[i][off + p + stride];
        }
      }
      const cx<T> r0 = upd(w0, a0), r1 = upd(w1, a1);
      w[off + p] = r0;
      w[off + p + stride] = r1;
      nrm += (double)r0.re * (double)r0.re + (double)r0.im * (double)r0.im;
      nrm += (double)r1.re * (double)r1.re + (double)r1.im * (double)r1.im;
    }
  }
  for (; p < N; p += stride) {
    const cx<T> w0 = w[off + p];
    cx<T> a0[NVMAX];
#pragma unroll
    for (int i = 0; i < NVMAX; ++i)
      if (EXACT || i < nv) a0[i] = V.v[i][off + p];
    const cx<T> r0 = upd(w0, a0);
    w[off + p] = r0;
    nrm += (double)r0.re * (double)r0.re + (double)r0.im * (double)r0.im;
  }
  const double s = block_sum(nrm, red);
  if (threadIdx.x == 0) out[0] = s;
}

// partial ||x||^2 per workgroup
template <typename T>
__global__ __launch_bounds__(256) void k_norm2(const Seg* __restrict__ segs, const int* __restrict__ vmap,
                                              const cx<T>* __restrict__ x, double* __restrict__ part,
                                              const int* __restrict__ active) {
  __shared__ double red[16];
  const int wg = blockIdx.x;
  const int sid = vmap[wg];
  const Seg& S = segs[sid];
  double* out = part + (int64_t)wg * PSTRIDE;
  if (active && !active[sid]) {
    if (threadIdx.x == 0) out[0] = 0.0;
    return;
  }
  const int64_t N = S.N, off = S.off;
  const int64_t stride = (int64_t)S.vnblk * 256;
  double nrm = 0.0;
  for (int64_t p = (int64_t)(wg - S.vblk0) * 256 + threadIdx.x; p < N; p += stride) {
    const cx<T> a = x[off + p];
    nrm += (double)a.re * (double)a.re + (double)a.im * (double)a.im;
  }
  const double s = block_sum(nrm, red);
  if (threadIdx.x == 0) out[0] = s;
}

// out[sid] = sqrt(sum of the segment's partial norms) (range `which`)
__global__ __launch_bounds__(256) void k_seg_norm(const Seg* __restrict__ segs, const double* __restrict__ part,
                                                  int which, double* __restrict__ out) {
  __shared__ double red[4];
  const int sid = blockIdx.x;
  int b0, nb;
  seg_range(segs[sid], which, b0, nb);
  const double s = seg_sum0(part, b0, nb, red);
  if (threadIdx.x == 0) out[sid] = sqrt(s);
}

// Start of a cycle: beta = vscale_in * sqrt(sum of partials of range
// `which`) (the partials are of the unscaled residual vector), g = (beta, 0,
// ...), scale_0 = vscale_in / beta (0 when beta == 0), beta_out = beta.
__global__ __launch_bounds__(256) void k_start_cycle(const Seg* __restrict__ segs, KState st, int which,
                                                     const double* __restrict__ vscale_in,
                                                     double* __restrict__ beta_out,
                                                     const int* __restrict__ active) {
  __shared__ double red[4];
  const int sid = blockIdx.x;
  if (active && !active[sid]) return;
  int b0, nb;
  seg_range(segs[sid], which, b0, nb);
  const double s = seg_sum0(st.part, b0, nb, red);
  if (threadIdx.x == 0) {
    const int ns = st.nseg;
    const double vin = vscale_in ? vscale_in[sid] : 1.0;
    const double beta = fabs(vin) * sqrt(s);
    st.g[sid] = d2(beta, 0.0);
    for (int i = 1; i <= KMAX; ++i) st.g[i * ns + sid] = d2(0.0, 0.0);
    st.scale[sid] = beta > 0.0 ? vin / beta : 0.0;
    if (beta_out) beta_out[sid] = beta;
  }
}

// Back substitution R y = g (k x k upper triangular, zero pivots -> y_i = 0)
// from R and g staged in LDS.  One thread.
__device__ __forceinline__ void solve_upper(const double2* R, const double2* g, int k, double2* y) {
  for (int i = k - 1; i >= 0; --i) {
    double2 acc = g[i];
    for (int l = i + 1; l < k; ++l) {
      const double2 h = R[i * KMAX + l];
      acc.x -= h.x * y[l].x - h.y * y[l].y;
      acc.y -= h.x * y[l].y + h.y * y[l].x;
    }
    const double2 d = R[i * KMAX + i];
    const double den = d.x * d.x + d.y * d.y;
    y[i] = den == 0.0 ? d2(0.0, 0.0)
                      : d2((acc.x * d.x + acc.y * d.y) / den, (acc.y * d.x - acc.x * d.y) / den);
  }
}

// Finish Arnoldi column j (partials of the vector range of st.part).  With
// solve_k > 0 (the cycle's last column, solve_k = j + 1) also solve R y = g
// and leave y_i * s_i in coef (s = basis scale, or 1 for a flexible space)
// for the update of the iterate.  Everything the step reads is staged in
// LDS by the workgroup first.
__global__ __launch_bounds__(256) void k_givens(const Seg* __restrict__ segs, KState st, int j, int solve_k,
                                                int use_scale, const int* __restrict__ active) {
  __shared__ double red[4];
  __shared__ GivensStage G;
  __shared__ double2 R[KMAX * KMAX];  // columns 0..solve_k-2 of R (column j comes from G)
  __shared__ double scl[KMAX];
  const int sid = blockIdx.x;
  if (active && !active[sid]) return;
  const Seg& S = segs[sid];
  const int ns = st.nseg;
  givens_stage(st, sid, j, j + 1, G);
  for (int idx = threadIdx.x; idx < solve_k * j; idx += blockDim.x) {  // rows 0..solve_k-1, columns 0..j-1
    const int i = idx / j, l = idx - (idx / j) * j;
    if (l >= i) R[i * KMAX + l] = st.H[(i * KMAX + l) * ns + sid];
  }
  if ((int)threadIdx.x < solve_k) scl[threadIdx.x] = use_scale ? st.scale[threadIdx.x * ns + sid] : 1.0;
  const double s = seg_sum0(st.part, S.vblk0, S.vnblk, red);  // (its barriers order the stage)
  if (threadIdx.x == 0) {
    givens_finish(st, sid, j, s, G);
    if (solve_k > 0) {
      for (int i = 0; i <= j; ++i) R[i * KMAX + j] = G.col[i];
      double2 y[KMAX];
      solve_upper(R, G.g, solve_k, y);
      for (int i = 0; i < solve_k; ++i) st.coef[i * ns + sid] = d2(y[i].x * scl[i], y[i].y * scl[i]);
    }
  }
}


// x += sum_j y_j * s_j * D_j, with D = V (GMRES, s = scale) or Z (FGMRES,
// s = 1); y_j s_j were left in coef by the cycle's last Givens step.  x may
// be of higher precision than D (mixed-precision outer iterate).
template <typename TX, typename T, int KM, bool EXACT>
__global__ __launch_bounds__(256) void k_update_x(const Seg* __restrict__ segs, const int* __restrict__ vmap,
                                                 VecList<T> D, int k, KState st, cx<TX>* __restrict__ x,
                                                 const int* __restrict__ active) {
  const int wg = blockIdx.x;
  const int sid = vmap[wg];
  if (active && !active[sid]) return;
  const Seg& S = segs[sid];
  if (EXACT) k = KM;
  cx<TX> c[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    if (EXACT || j < k) {
      const double2 ys = st.coef[j * st.nseg + sid];
      c[j] = mk<TX>((TX)ys.x, (TX)ys.y);
    }
  }
  const int64_t N = S.N, off = S.off;
  const int64_t stride = (int64_t)S.vnblk * 256;
  auto upd = [&](cx<TX> acc, const cx<T>* d) {
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (EXACT || j < k) acc = cfma(c[j], cast<TX>(d[j]), acc);
    return acc;
  };
  int64_t p = (int64_t)(wg - S.vblk0) * 256 + threadIdx.x;
  if (EXACT) {  // two elements per iteration: twice the loads in flight
    for (; p + stride < N; p += 2 * stride) {
      const cx<TX> x0 = x[off + p], x1 = x[off + p + stride];
      cx<T> d0[KM], d1[KM];
#pragma unroll
      for (int j = 0; j < KM; ++j) {
        if (EXACT || j < k) {
          d0[j] = D.v[j][off + p];
          d1[j] = D.v[j][off + p + stride];
        }
      }
      x[off + p] = upd(x0, d0);
      x[off + p + stride] = upd(x1, d1);
    }
  }
  for (; p < N; p += stride) {
    const cx<TX> x0 = x[off + p];
    cx<T> d0[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (EXACT || j < k) d0[j] = D.v[j][off + p];
    x[off + p] = upd(x0, d0);
  }
}

// x = 0 on the active segments
template <typename T>
__global__ __launch_bounds__(256) void k_zero(const Seg* __restrict__ segs, const int* __restrict__ vmap,
                                              cx<T>* __restrict__ x, const int* __restrict__ active) {
  const int wg = blockIdx.x;
  const int sid = vmap[wg];
  if (active && !active[sid]) return;
  const Seg& S = segs[sid];
  const int64_t stride = (int64_t)S.vnblk * 256;
  for (int64_t p = (int64_t)(wg - S.vblk0) * 256 + threadIdx.x; p < S.N; p += stride)
    x[S.off + p] = czero<T>();
}

// elementwise precision conversion over a flat range
template <typename TO, typename TI>
__global__ __launch_bounds__(256) void k_convert(const cx<TI>* __restrict__ in, cx<TO>* __restrict__ out,
                                                 int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += stride) out[p] = cast<TO>(in[p]);
}

// flat zero fill (used by the misfit driver)
template <typename T>
__global__ __launch_bounds__(256) void k_fill_zero(cx<T>* __restrict__ x, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += stride) x[p] = czero<T>();
}

}  // namespace helm
