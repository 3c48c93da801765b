// Krylov building blocks for restarted (F)GMRES on many right-hand sides at
// once (all sources of one frequency share the operator; each keeps its own
// Krylov state).  Every scalar of the method (Hessenberg entries, Givens
// rotations, residual estimates, basis scales) stays on the device; sums
// are accumulated in FP64 with a fixed reduction order, so results are
// bitwise reproducible run to run.
//
// Orthogonalisation is classical Gram-Schmidt in two kernels (all inner
// products of a column in one pass over the basis, then one fused
// "w -= sum c_i V_i; ||w||^2" pass), with lazy normalisation: basis vector
// V_i is stored unnormalised together with scale_i = 1/||V_i|| per
// right-hand side, and consumers fold the scale into their first use.
#pragma once

#include "common.h"

namespace helm {

constexpr int DOT_BLOCKS = 240;  // workgroups per right-hand side for the dot pass

// Up to KMAX+1 vector pointers of one right-hand-side block (element r*N+p).
template <typename T>
struct VecList {
  const cx<T>* v[KMAX + 1];
};

// Device-resident state of one (F)GMRES instance, structure of arrays over
// right-hand sides: entry [idx][r] is at idx*nrhs + r.
struct KState {
  double2* H;      // (KMAX+1) x KMAX Hessenberg / R factor, [(i*KMAX+j)][r]
  double* cs;      // Givens cosines [j][r]
  double2* sn;     // Givens sines   [j][r]
  double2* g;      // rotated right-hand side [i][r]
  double* scale;   // 1/||V_i|| [i][r]
  double2* coef;   // CGS coefficients of the current column, scale folded in
  double* part;    // partial sums scratch [r][blk][2*(KMAX+1)]
  int nrhs;
};

__device__ __forceinline__ double2 d2(double a, double b) { return make_double2(a, b); }

// ---------------------------------------------------------------------------
// partial inner products  s_i = sum_p conj(V_i[p]) w[p],  i < nv
// part[(r*nblk + blk)*2*(KMAX+1) + 2i + {0,1}]
// ---------------------------------------------------------------------------
template <typename T, int NVMAX>
__global__ __launch_bounds__(256) void k_dots(VecList<T> V, int nv, const cx<T>* __restrict__ w,
                                             int64_t N, double* __restrict__ part,
                                             const int* __restrict__ active) {
  __shared__ double red[4][2 * NVMAX];
  const int r = blockIdx.y;
  const int nblk = gridDim.x;
  double* out = part + ((int64_t)r * nblk + blockIdx.x) * PSTRIDE;
  if (active && !active[r]) {
    if (threadIdx.x < 2 * NVMAX) out[threadIdx.x] = 0.0;
    return;
  }
  double ar[NVMAX], ai[NVMAX];
#pragma unroll
  for (int i = 0; i < NVMAX; ++i) ar[i] = ai[i] = 0.0;
  const cx<T>* wr = w + r * N;
  const int64_t stride = (int64_t)nblk * 256;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < N; p += stride) {
    const cx<T> wv = wr[p];
#pragma unroll
    for (int i = 0; i < NVMAX; ++i) {
      if (i < nv) {
        const cx<T> a = V.v[i][r * N + p];
        // conj(a) * w
        ar[i] += (double)a.re * (double)wv.re + (double)a.im * (double)wv.im;
        ai[i] += (double)a.re * (double)wv.im - (double)a.im * (double)wv.re;
      }
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NVMAX; ++i) {
    if (i < nv) {
      const double sr = wave_sum(ar[i]);
      const double si = wave_sum(ai[i]);
      if (lane == 0) {
        red[wid][2 * i] = sr;
        red[wid][2 * i + 1] = si;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * nv) {
    out[threadIdx.x] = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                       red[3][threadIdx.x];
  }
}

// One workgroup of 64 lanes per right-hand side: H[i][j] = scale_i * sum of
// partials, coef_i = H[i][j] * scale_i.
__global__ __launch_bounds__(64) void k_reduce_dots(KState st, int nv, int j, int nblk,
                                                    const int* __restrict__ active) {
  const int r = blockIdx.x;
  if (active && !active[r]) return;
  const int nrhs = st.nrhs;
  const double* base = st.part + (int64_t)r * nblk * PSTRIDE;
  for (int i = 0; i < nv; ++i) {
    double sr = 0.0, si = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 64) {
      sr += base[(int64_t)b * PSTRIDE + 2 * i];
      si += base[(int64_t)b * PSTRIDE + 2 * i + 1];
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (threadIdx.x == 0) {
      const double s = st.scale[i * nrhs + r];
      const double2 h = d2(s * sr, s * si);
      st.H[(i * KMAX + j) * nrhs + r] = h;
      st.coef[i * nrhs + r] = d2(h.x * s, h.y * s);
    }
  }
}

// w <- w - sum_i coef_i V_i  (in place), partial ||w||^2 per workgroup
// into part[(r*nblk + blk)*2*(KMAX+1)].
template <typename T, int NVMAX>
__global__ __launch_bounds__(256) void k_axpy_norm(VecList<T> V, int nv, cx<T>* __restrict__ w,
                                                  int64_t N, KState st,
                                                  const int* __restrict__ active) {
  __shared__ double red[16];
  const int r = blockIdx.y;
  const int nblk = gridDim.x;
  double* out = st.part + ((int64_t)r * nblk + blockIdx.x) * PSTRIDE;
  if (active && !active[r]) {
    if (threadIdx.x == 0) out[0] = 0.0;
    return;
  }
  cx<T> c[NVMAX];
#pragma unroll
  for (int i = 0; i < NVMAX; ++i) {
    if (i < nv) {
      const double2 q = st.coef[i * st.nrhs + r];
      c[i] = mk<T>((T)q.x, (T)q.y);
    }
  }
  cx<T>* wr = w + r * N;
  double nrm = 0.0;
  const int64_t stride = (int64_t)nblk * 256;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < N; p += stride) {
    cx<T> acc = wr[p];
#pragma unroll
    for (int i = 0; i < NVMAX; ++i) {
      if (i < nv) {
        const cx<T> a = V.v[i][r * N + p];
        acc = acc - c[i] * a;
      }
    }
    wr[p] = acc;
    nrm += (double)acc.re * (double)acc.re + (double)acc.im * (double)acc.im;
  }
  const double s = block_sum(nrm, red);
  if (threadIdx.x == 0) out[0] = s;
}

// plain partial ||x||^2 (x with optional per-rhs scale applied afterwards)
template <typename T>
__global__ __launch_bounds__(256) void k_norm2(const cx<T>* __restrict__ x, int64_t N,
                                              double* __restrict__ part,
                                              const int* __restrict__ active) {
  __shared__ double red[16];
  const int r = blockIdx.y;
  const int nblk = gridDim.x;
  double* out = part + ((int64_t)r * nblk + blockIdx.x) * PSTRIDE;
  if (active && !active[r]) {
    if (threadIdx.x == 0) out[0] = 0.0;
    return;
  }
  const cx<T>* xr = x + r * N;
  double nrm = 0.0;
  const int64_t stride = (int64_t)nblk * 256;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < N; p += stride) {
    const cx<T> a = xr[p];
    nrm += (double)a.re * (double)a.re + (double)a.im * (double)a.im;
  }
  const double s = block_sum(nrm, red);
  if (threadIdx.x == 0) out[0] = s;
}

// Start of a cycle: beta = vscale_in[r] * sqrt(sum partials) (the partials
// are of the unscaled residual vector), g = (beta, 0, ...), scale_0 =
// vscale_in/beta (or 0 when beta == 0), beta_out[r] = beta.
__global__ __launch_bounds__(64) void k_start_cycle(KState st, int nblk,
                                                    const double* __restrict__ vscale_in,
                                                    double* __restrict__ beta_out,
                                                    const int* __restrict__ active) {
  const int r = blockIdx.x;
  if (active && !active[r]) return;
  const int nrhs = st.nrhs;
  const double* base = st.part + (int64_t)r * nblk * PSTRIDE;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) s += base[(int64_t)b * PSTRIDE];
  s = wave_sum(s);
  if (threadIdx.x == 0) {
    const double vin = vscale_in ? vscale_in[r] : 1.0;
    const double beta = fabs(vin) * sqrt(s);
    st.g[r] = d2(beta, 0.0);
    for (int i = 1; i <= KMAX; ++i) st.g[i * nrhs + r] = d2(0.0, 0.0);
    st.scale[r] = beta > 0.0 ? vin / beta : 0.0;
    if (beta_out) beta_out[r] = beta;
  }
}

// Finish Arnoldi column j: h_{j+1,j} = sqrt(sum partials); apply the
// previous rotations to column j, build rotation j, update g, set
// scale_{j+1} = 1/h_{j+1,j} (0 on breakdown).
__global__ __launch_bounds__(64) void k_givens(KState st, int j, int nblk,
                                               const int* __restrict__ active) {
  const int r = blockIdx.x;
  if (active && !active[r]) return;
  const int nrhs = st.nrhs;
  const double* base = st.part + (int64_t)r * nblk * PSTRIDE;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) s += base[(int64_t)b * PSTRIDE];
  s = wave_sum(s);
  if (threadIdx.x != 0) return;
  const double hn = sqrt(s);
  // rotate column j by the previous rotations
  for (int i = 0; i < j; ++i) {
    const double2 a = st.H[(i * KMAX + j) * nrhs + r];
    const double2 b = st.H[((i + 1) * KMAX + j) * nrhs + r];
    const double c = st.cs[i * nrhs + r];
    const double2 sn = st.sn[i * nrhs + r];
    // [c, s; -conj(s), c] [a; b]
    const double2 na = d2(c * a.x + (sn.x * b.x - sn.y * b.y), c * a.y + (sn.x * b.y + sn.y * b.x));
    const double2 nb = d2(-(sn.x * a.x + sn.y * a.y) + c * b.x, -(sn.x * a.y - sn.y * a.x) + c * b.y);
    st.H[(i * KMAX + j) * nrhs + r] = na;
    st.H[((i + 1) * KMAX + j) * nrhs + r] = nb;
  }
  const double2 a = st.H[(j * KMAX + j) * nrhs + r];
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
  st.cs[j * nrhs + r] = c;
  st.sn[j * nrhs + r] = sn;
  st.H[(j * KMAX + j) * nrhs + r] = rr;
  st.H[((j + 1) * KMAX + j) * nrhs + r] = d2(0.0, 0.0);
  const double2 gj = st.g[j * nrhs + r];
  // g_{j+1} = -conj(s) g_j ; g_j = c g_j
  st.g[(j + 1) * nrhs + r] = d2(-(sn.x * gj.x + sn.y * gj.y), -(sn.x * gj.y - sn.y * gj.x));
  st.g[j * nrhs + r] = d2(c * gj.x, c * gj.y);
  st.scale[(j + 1) * nrhs + r] = hn > 0.0 ? 1.0 / hn : 0.0;
}

// Back substitution R y = g (k x k upper triangular, zero pivots -> y_i = 0)
// done by lane 0 of the workgroup into shared memory.
__device__ __forceinline__ void solve_upper(const KState& st, int r, int k, double2* y) {
  const int nrhs = st.nrhs;
  for (int i = k - 1; i >= 0; --i) {
    double2 acc = st.g[i * nrhs + r];
    for (int l = i + 1; l < k; ++l) {
      const double2 h = st.H[(i * KMAX + l) * nrhs + r];
      acc.x -= h.x * y[l].x - h.y * y[l].y;
      acc.y -= h.x * y[l].y + h.y * y[l].x;
    }
    const double2 d = st.H[(i * KMAX + i) * nrhs + r];
    const double den = d.x * d.x + d.y * d.y;
    if (den == 0.0) {
      y[i] = d2(0.0, 0.0);
    } else {
      y[i] = d2((acc.x * d.x + acc.y * d.y) / den, (acc.y * d.x - acc.x * d.y) / den);
    }
  }
}

// x += sum_j y_j * s_j * D_j, with D = V (GMRES, s = scale) or Z (FGMRES,
// s = 1).  y from R y = g solved per workgroup.  x may be of higher
// precision than D (mixed-precision outer iterate).
template <typename TX, typename T, int KM>
__global__ __launch_bounds__(256) void k_update_x(VecList<T> D, int k, bool use_scale, KState st,
                                                 cx<TX>* __restrict__ x, int64_t N,
                                                 const int* __restrict__ active) {
  __shared__ double2 ys[KMAX];
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  if (threadIdx.x == 0) {
    double2 y[KMAX];
    solve_upper(st, r, k, y);
    for (int j = 0; j < k; ++j) {
      const double s = use_scale ? st.scale[j * st.nrhs + r] : 1.0;
      ys[j] = d2(y[j].x * s, y[j].y * s);
    }
  }
  __syncthreads();
  cx<TX> c[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j)
    if (j < k) c[j] = mk<TX>((TX)ys[j].x, (TX)ys[j].y);
  cx<TX>* xr = x + r * N;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < N; p += stride) {
    cx<TX> acc = xr[p];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      if (j < k) acc = cfma(c[j], cast<TX>(D.v[j][r * N + p]), acc);
    }
    xr[p] = acc;
  }
}

// ---------------------------------------------------------------------------
// small elementwise helpers
// ---------------------------------------------------------------------------
template <typename TO, typename TI>
__global__ __launch_bounds__(256) void k_convert(const cx<TI>* __restrict__ in, cx<TO>* __restrict__ out,
                                                 int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += stride)
    out[p] = cast<TO>(in[p]);
}

// x[r] = 0 for active right-hand sides
template <typename T>
__global__ __launch_bounds__(256) void k_zero(cx<T>* __restrict__ x, int64_t N,
                                              const int* __restrict__ active) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < N; p += stride)
    x[r * N + p] = czero<T>();
}

}  // namespace helm
