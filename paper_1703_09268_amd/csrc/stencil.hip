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
// Launch shape: a workgroup of 256 lanes owns 256 consecutive points of the
// flattened (y, z) plane (so a ragged nz wastes no lanes) and marches along
// x over `xchunk` planes; smap / slocal give its segment and its tile index
// inside the segment.  x[i-1], x[i], x[i+1] of its own column sit in
// registers and x[i+2] is already in flight while plane i is computed; the
// y and z neighbours are the neighbouring lanes' own loads and come from the
// vector cache.  Every access is a contiguous 64-lane run; workgroups are
// renumbered so that one XCD runs a contiguous range of tiles (shared halos
// stay in one L2).
#pragma once

#include "common.h"
#include <type_traits>

#include "krylov.hip"
#include "segment.h"

namespace helm {

template <typename T>
struct Tab7 {
  const cx<T>* al[3];
  const cx<T>* be[3];
  const cx<T>* de[3];
};

template <typename TC>
__device__ __forceinline__ Tab7<TC> seg_tables(const Seg& S);
template <>
__device__ __forceinline__ Tab7<float> seg_tables<float>(const Seg& S) {
  Tab7<float> t;
  const cx<float>* base = reinterpret_cast<const cx<float>*>(S.tabf) + (int64_t)S.dir * S.tdir;
  for (int a = 0; a < 3; ++a) {
    t.al[a] = base + S.tpre[a];
    t.be[a] = base + S.tpre[a] + S.n[a];
    t.de[a] = base + S.tpre[a] + 2 * S.n[a];
  }
  return t;
}
template <>
__device__ __forceinline__ Tab7<double> seg_tables<double>(const Seg& S) {
  Tab7<double> t;
  const cx<double>* base = reinterpret_cast<const cx<double>*>(S.tabd) + (int64_t)S.dir * S.tdir;
  for (int a = 0; a < 3; ++a) {
    t.al[a] = base + S.tpre[a];
    t.be[a] = base + S.tpre[a] + S.n[a];
    t.de[a] = base + S.tpre[a] + 2 * S.n[a];
  }
  return t;
}

template <typename TX, typename TC>
__device__ __forceinline__ cx<TC> ld(const cx<TX>* p) {
  return cast<TC>(*p);
}

// Workgroup-uniform table entry through the scalar cache (constant address
// space: the tables are read-only while any kernel runs).  Keeps these reads
// off the vector memory counter, so they never wait for the field loads in
// flight.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
__device__ __forceinline__ cx<T> uload(const cx<T>* p, int i) {
  typedef const __attribute__((address_space(4))) cx<T> ccx;
  return ((ccx*)p)[i];
}
// global address space pointers (a plain pointer read from a segment
// descriptor would otherwise be accessed with flat instructions, which wait
// for every vector and scalar access in flight)
#define HELM_GLOBAL __attribute__((address_space(1)))
#else
template <typename T>
__device__ __forceinline__ cx<T> uload(const cx<T>* p, int i) {
  return p[i];
}
#define HELM_GLOBAL
#endif

// out = s_x * H x            (RESID = false)
// out = s_b * b - s_x * H x  (RESID = true)
// s_x, s_b: per-segment scales (null = 1).  With NORM, the workgroup's sum of
// |out|^2 (FP64) goes to part[(sblk0 + local) * PSTRIDE].
// Any precision; one point per lane (a pair tile is walked as two halves).
// Pad entries (k >= n2 on a padded level) are written as zero.
template <typename TC, typename TX, typename TM, typename TB, typename TO, bool RESID, bool NORM>
__global__ __launch_bounds__(256) void k_h7(const Seg* __restrict__ segs, const int* __restrict__ smap,
                                            const int* __restrict__ slocal,
                                            const cx<TX>* __restrict__ x, const double* __restrict__ xs,
                                            const cx<TB>* __restrict__ b, const double* __restrict__ bs,
                                            cx<TO>* __restrict__ out, double* __restrict__ part,
                                            const int* __restrict__ active) {
  __shared__ double red[16];
  const int wg = xcd_logical(blockIdx.x, gridDim.x);
  const int sid = smap[wg];
  const int local = slocal[wg];
  const Seg& S = segs[sid];
  // partial sums go to the segment's own range, whatever the launch order
  double* const pslot = NORM ? part + (int64_t)(S.sblk0 + local) * PSTRIDE : nullptr;
  if (active && !active[sid]) {
    if (NORM && threadIdx.x == 0) *pslot = 0.0;
    return;  // uniform across the workgroup
  }
  const int nx = S.n[0], ny = S.n[1], nz = S.n[2], pz = S.pz;
  const int xc = local / S.plane_blocks;
  const int pb = local - xc * S.plane_blocks;
  const int64_t plane = (int64_t)ny * pz;
  const Tab7<TC> tab = seg_tables<TC>(S);
  const TC w2 = (TC)S.w2;
  const TM* __restrict__ m = reinterpret_cast<const TM*>(S.m);
  const cx<TX>* __restrict__ xr = x + S.off;
  const TC sx = xs ? (TC)xs[sid] : TC(1);
  TC sb = TC(1);
  if (RESID) sb = bs ? (TC)bs[sid] : TC(1);
  const int i0 = xc * S.xchunk;
  const int i1 = min(nx, i0 + S.xchunk);
  double nrm = 0.0;
  const int halves = S.pair ? 2 : 1;
  for (int half = 0; half < halves; ++half) {
    const int idx = (pb * halves + half) * 256 + threadIdx.x;
    const bool in = idx < plane;
    const int j = in ? idx / pz : 0;
    const int k = in ? idx - j * pz : 0;
    const bool real = in && k < nz;
    cx<TC> az = czero<TC>(), bz = az, dz = az, ay = az, by = az, dy = az;
    if (real) {
      az = tab.al[2][k]; bz = tab.be[2][k]; dz = tab.de[2][k];
      ay = tab.al[1][j]; by = tab.be[1][j]; dy = tab.de[1][j];
    }
    const bool has_ym = real && j > 0, has_yp = real && j + 1 < ny;
    const bool has_zm = real && k > 0, has_zp = real && k + 1 < nz;
    int64_t p = (int64_t)i0 * plane + idx;
    cx<TC> xm = czero<TC>(), xcur = czero<TC>(), xp = czero<TC>();
    if (real) {
      if (i0 > 0) xm = ld<TX, TC>(xr + p - plane);
      xcur = ld<TX, TC>(xr + p);
      if (i0 + 1 < nx) xp = ld<TX, TC>(xr + p + plane);
    }
    for (int i = i0; i < i1; ++i, p += plane) {
      cx<TC> ym = czero<TC>(), yp = ym, zm = ym, zp = ym;
      TC mv = TC(0);
      if (real) {
        if (has_ym) ym = ld<TX, TC>(xr + p - pz);
        if (has_yp) yp = ld<TX, TC>(xr + p + pz);
        if (has_zm) zm = ld<TX, TC>(xr + p - 1);
        if (has_zp) zp = ld<TX, TC>(xr + p + 1);
        mv = (TC)m[p];
      }
      // plane i+2 goes in flight while plane i is computed
      cx<TC> xpp = czero<TC>();
      if (real && i + 2 < nx) xpp = ld<TX, TC>(xr + p + 2 * plane);
      if (in) {
        cx<TC> acc = czero<TC>();
        if (real) {
          const cx<TC> ax = uload(tab.al[0], i), bx = uload(tab.be[0], i), dx = uload(tab.de[0], i);
          acc = mk<TC>(w2 * mv + dx.re + dy.re + dz.re, dx.im + dy.im + dz.im) * xcur;
          acc = cfma(ax, xp - xcur, acc);
          acc = cfma(bx, xm - xcur, acc);
          acc = cfma(ay, yp - xcur, acc);
          acc = cfma(by, ym - xcur, acc);
          acc = cfma(az, zp - xcur, acc);
          acc = cfma(bz, zm - xcur, acc);
          acc = sx * acc;
          if (RESID) acc = sb * ld<TB, TC>(b + S.off + p) - acc;
        }
        out[S.off + p] = cast<TO>(acc);
        if (NORM) nrm += (double)acc.re * (double)acc.re + (double)acc.im * (double)acc.im;
      }
      xm = xcur;
      xcur = xp;
      xp = xpp;
    }
  }
  if (NORM) {
    const double s = block_sum(nrm, red);
    if (threadIdx.x == 0) *pslot = s;
  }
}

// ---------------------------------------------------------------------------
// complex64 7-point operator with pair tiles: a lane owns two consecutive
// z-points (e0, e0 + 1) of the flattened (y, z) plane, e0 even, and moves
// them with 16-byte accesses; a workgroup covers 512 points of the plane and
// marches along x.  Per plane and pair: one 16-byte load of x (plane i+2, the
// three before it are in registers), two 16-byte loads of the y neighbour
// pairs, two 8-byte loads of the outer z neighbours (the inner ones are the
// pair itself), one 8-byte model load and one 16-byte store.
// Requirements (checked by the launcher): every segment of the level has an
// even z pitch and an even element offset, and x, b, out are 16-byte aligned.
// Couplings to nodes outside the grid are zero in the tables (folded into
// delta), so clamped neighbour addresses need no masks.  Out-of-plane lanes
// compute the plane's last pair again (same inputs, same instructions) and
// store the identical values, which keeps the loop body branch-free.  The
// output must not alias x or b.
// ---------------------------------------------------------------------------
struct alignas(16) c32x2 {
  float a, b, c, d;  // (re, im) of element 0, then of element 1
};

// Buffer access to one plane of a level vector: a resource built from the
// workgroup-uniform plane address (raw buffer, 32-bit words), addressed by
// the lanes with 32-bit byte offsets, so no access needs 64-bit address
// arithmetic per lane.  The resource spans the plane; accesses beyond it
// read zero and write nothing.
#if defined(__HIP_DEVICE_COMPILE__)
typedef __amdgpu_buffer_rsrc_t prsrc;
__device__ __forceinline__ prsrc plane_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float pld_f(prsrc r, uint32_t o) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0));
}
__device__ __forceinline__ c32 pld_c(prsrc r, uint32_t o) {
  return __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(r, o, 0, 0));
}
__device__ __forceinline__ c32x2 pld_c2(prsrc r, uint32_t o) {
  return __builtin_bit_cast(c32x2, __builtin_amdgcn_raw_buffer_load_b128(r, o, 0, 0));
}
__device__ __forceinline__ void pst_c2(c32x2 v, prsrc r, uint32_t o) {
  typedef decltype(__builtin_amdgcn_raw_buffer_load_b128(r, o, 0, 0)) w4;
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(w4, v), r, o, 0, 0);
}
// Buffer load straight into LDS (no registers): lane i of the wave writes
// its `bytes` at dst + i * bytes; dst must be the same for the whole wave.
__device__ __forceinline__ void pld_lds16(prsrc r, void* dst, uint32_t o) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)dst, 16, o, 0, 0, 0);
}
__device__ __forceinline__ void pld_lds4(prsrc r, void* dst, uint32_t o) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)dst, 4, o, 0, 0, 0);
}
// every vector memory access of this wave (LDS fills included) has completed
__device__ __forceinline__ void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
#else
struct prsrc {};
inline prsrc plane_rsrc(const void*, uint32_t) { return prsrc{}; }
inline float pld_f(prsrc, uint32_t) { return 0.f; }
inline c32 pld_c(prsrc, uint32_t) { return c32{}; }
inline c32x2 pld_c2(prsrc, uint32_t) { return c32x2{}; }
inline void pst_c2(c32x2, prsrc, uint32_t) {}
inline void pld_lds16(prsrc, void*, uint32_t) {}
inline void pld_lds4(prsrc, void*, uint32_t) {}
inline void wait_vmem() {}
#endif

// level vectors an Arnoldi stencil pass takes inner products with
struct VecPtrs {
  const c32* v[6];
};

//
// Arnoldi variant (NMEM + SELF > 0, plain H x only): the same pass also forms
// the workgroup's partial inner products s_t = sum conj(D_t) out over its
// points, for D_t = Vd.v[t] (t < NMEM, read from memory) and, with SELF, the
// stored input x itself as the last one; they go to
// part[(sblk0 + local) * PSTRIDE + 2t (+1)] (re, im).  This replaces a
// separate pass that would read the output back.  With npart, the input scale
// is derived in the kernel from the partial norms of the pass that wrote x
// (the Givens step of the previous column then runs later).  The plain
// operator (no inner products, no residual) keeps two planes of loads in
// flight (DEEP); the heavier variants one, to stay within their registers.
template <bool RESID, bool NORM, int NMEM, bool SELF, bool DEEP = (!RESID && !NORM && NMEM == 0 && !SELF)>
__global__ __launch_bounds__(256) void k_h7p(const Seg* __restrict__ segs, const int* __restrict__ smap,
                                             const int* __restrict__ slocal, const c32* __restrict__ x,
                                             const double* __restrict__ xs, const c32* __restrict__ b,
                                             const double* __restrict__ bs, c32* __restrict__ out,
                                             double* __restrict__ part, const int* __restrict__ active,
                                             VecPtrs Vd, const double* __restrict__ npart) {
  constexpr int ND = NMEM + (SELF ? 1 : 0);
  static_assert(!(ND > 0 && (RESID || NORM)), "inner products only with the plain operator");
  __shared__ double red[ND > 0 ? 4 * 2 * ND : 16];
  const int wg = xcd_logical(blockIdx.x, gridDim.x);
  const int sid = smap[wg];
  const int local = slocal[wg];
  const Seg& S = segs[sid];
  double* const pslot = (NORM || ND > 0) ? part + (int64_t)(S.sblk0 + local) * PSTRIDE : nullptr;
  if (active && !active[sid]) {
    if (NORM && threadIdx.x == 0) *pslot = 0.0;
    if (ND > 0 && threadIdx.x < 2 * ND) pslot[threadIdx.x] = 0.0;
    return;
  }
  const int nx = S.n[0], nz = S.n[2], pz = S.pz;
  const int plane = S.n[1] * pz;  // even
  const int npair = plane >> 1;
  const int xc = local / S.plane_blocks;
  const int pb = local - xc * S.plane_blocks;
  const int q0 = pb * 256 + threadIdx.x;
  const bool in = q0 < npair;
  const int e0 = 2 * (in ? q0 : npair - 1);
  const int j = e0 / pz, k0 = e0 - j * pz;  // k0 even, k0 + 1 < pz
  const bool pad1 = k0 + 1 >= nz;           // element 1 is a pitch pad
  const Tab7<float> tab = seg_tables<float>(S);
  const c32 ay = tab.al[1][j], by = tab.be[1][j], dy = tab.de[1][j];
  const c32 az0 = tab.al[2][k0], bz0 = tab.be[2][k0];
  const c32 d0 = dy + tab.de[2][k0];
  c32 az1 = czero<float>(), bz1 = czero<float>(), d1 = dy;
  if (!pad1) {
    az1 = tab.al[2][k0 + 1];
    bz1 = tab.be[2][k0 + 1];
    d1 = dy + tab.de[2][k0 + 1];
  }
  // neighbour element offsets inside the plane, clamped where the coupling is zero
  const int oym = e0 >= pz ? e0 - pz : e0;
  const int oyp = e0 + pz < plane ? e0 + pz : e0;
  const int ozm = e0 > 0 ? e0 - 1 : e0;
  const int ozp = e0 + 2 < plane ? e0 + 2 : e0 + 1;
  const float w2 = (float)S.w2;
  const HELM_GLOBAL float2* __restrict__ mp =
      (const HELM_GLOBAL float2*)(reinterpret_cast<const float*>(S.m) + e0);  // e0 even: 8-byte aligned
  const c32* __restrict__ xr = x + S.off;
  // input scale: given, or (npart) 1/||x|| from the partial norms of the
  // vector pass that produced x, summed exactly as the Givens step does
  float sx = xs ? (float)xs[sid] : 1.0f;
  if (npart) sx = (float)basis_scale(seg_sum0(npart, S.vblk0, S.vnblk, red));
  float sb = 1.0f;
  if (RESID) sb = bs ? (float)bs[sid] : 1.0f;
  auto L2 = [&](int ip, int e) { return *reinterpret_cast<const c32x2*>(xr + (int64_t)ip * plane + e); };
  const int i0 = xc * S.xchunk;
  const int i1 = min(nx, i0 + S.xchunk);
  double nrm = 0.0;
  const double wn = in ? 1.0 : 0.0;  // norm weight (duplicates count zero)
  double dr[ND > 0 ? ND : 1], di[ND > 0 ? ND : 1];
#pragma unroll
  for (int t = 0; t < ND; ++t) dr[t] = di[t] = 0.0;
  const float wf = in ? 1.0f : 0.0f;
  // Loads of plane i other than x's own column (issued one plane ahead).
  struct Yp {
    c32x2 ym, yp, bv;
    c32 zm, zp;
    float2 mv;
    c32x2 dv[NMEM > 0 ? NMEM : 1];
  };
  auto load = [&](int i, Yp& Y) {
    const int64_t pl = (int64_t)i * plane;
#pragma unroll
    for (int t = 0; t < NMEM; ++t) Y.dv[t] = *reinterpret_cast<const c32x2*>(Vd.v[t] + S.off + pl + e0);
    Y.ym = L2(i, oym);
    Y.yp = L2(i, oyp);
    Y.zm = xr[pl + ozm];
    Y.zp = xr[pl + ozp];
    Y.mv = mp[pl >> 1];
    if (RESID) Y.bv = *reinterpret_cast<const c32x2*>(b + S.off + pl + e0);
  };
  auto compute = [&](int i, const c32x2& qm, const c32x2& qc, const c32x2& qp, const Yp& Y) {
    const int64_t pl = (int64_t)i * plane;
    const c32 ax = uload(tab.al[0], i), bx = uload(tab.be[0], i), dx = uload(tab.de[0], i);
    const c32 x0 = mk(qc.a, qc.b), x1 = mk(qc.c, qc.d);
    c32 a0 = mk(w2 * Y.mv.x + dx.re + d0.re, dx.im + d0.im) * x0;
    a0 = cfma(ax, mk(qp.a, qp.b) - x0, a0);
    a0 = cfma(bx, mk(qm.a, qm.b) - x0, a0);
    a0 = cfma(ay, mk(Y.yp.a, Y.yp.b) - x0, a0);
    a0 = cfma(by, mk(Y.ym.a, Y.ym.b) - x0, a0);
    a0 = cfma(az0, x1 - x0, a0);
    a0 = cfma(bz0, Y.zm - x0, a0);
    c32 a1 = mk(w2 * Y.mv.y + dx.re + d1.re, dx.im + d1.im) * x1;
    a1 = cfma(ax, mk(qp.c, qp.d) - x1, a1);
    a1 = cfma(bx, mk(qm.c, qm.d) - x1, a1);
    a1 = cfma(ay, mk(Y.yp.c, Y.yp.d) - x1, a1);
    a1 = cfma(by, mk(Y.ym.c, Y.ym.d) - x1, a1);
    a1 = cfma(az1, Y.zp - x1, a1);
    a1 = cfma(bz1, x0 - x1, a1);
    a0 = sx * a0;
    a1 = sx * a1;
    if (RESID) {
      a0 = sb * mk(Y.bv.a, Y.bv.b) - a0;
      a1 = sb * mk(Y.bv.c, Y.bv.d) - a1;
    }
    if (pad1) a1 = czero<float>();
    c32x2 o;
    o.a = a0.re; o.b = a0.im; o.c = a1.re; o.d = a1.im;
    if (DEEP) {
      // the plain operator's output is not read back soon: stream it past
      // the caches (measured +4 % on 128^3 x 16; the Arnoldi variants keep
      // theirs cached for the update pass that follows)
      typedef float v4f __attribute__((ext_vector_type(4)));
      const v4f o4 = {o.a, o.b, o.c, o.d};
      __builtin_nontemporal_store(o4, reinterpret_cast<v4f*>(out + S.off + pl + e0));
    } else {
      *reinterpret_cast<c32x2*>(out + S.off + pl + e0) = o;
    }
    if (NORM)
      nrm += wn * ((double)a0.re * (double)a0.re + (double)a0.im * (double)a0.im +
                   ((double)a1.re * (double)a1.re + (double)a1.im * (double)a1.im));
    if (ND > 0) {
      const c32 u0 = wf * a0, u1 = wf * a1;
#pragma unroll
      for (int t = 0; t < ND; ++t) {
        const c32x2 v = (SELF && t == ND - 1) ? qc : Y.dv[t < NMEM ? t : 0];
        dr[t] += (double)v.a * u0.re + (double)v.b * u0.im + ((double)v.c * u1.re + (double)v.d * u1.im);
        di[t] += (double)v.a * u0.im - (double)v.b * u0.re + ((double)v.c * u1.im - (double)v.d * u1.re);
      }
    }
  };
  if (DEEP) {
    // Step i: the loads of plane i+2 and of x plane i+3 go out, then plane i
    // is computed from loads issued two steps earlier (six-register ring of x
    // planes, three load sets, unrolled by six: no loaded value is copied
    // between registers, since a copy would wait for the load).
    auto step = [&](int i, const c32x2& qm, const c32x2& qc, const c32x2& qp, c32x2& qn, const Yp& Yc, Yp& Yn) {
      load(min(i + 2, nx - 1), Yn);
      qn = L2(min(i + 3, nx - 1), e0);
      compute(i, qm, qc, qp, Yc);
    };
    c32x2 r0 = L2(max(i0 - 1, 0), e0), r1 = L2(i0, e0), r2 = L2(min(i0 + 1, nx - 1), e0),
          r3 = L2(min(i0 + 2, nx - 1), e0), r4, r5;
    Yp YA, YB, YC;
    load(i0, YA);
    load(min(i0 + 1, nx - 1), YB);
    int i = i0;
    for (; i + 6 <= i1; i += 6) {
      step(i, r0, r1, r2, r4, YA, YC);
      step(i + 1, r1, r2, r3, r5, YB, YA);
      step(i + 2, r2, r3, r4, r0, YC, YB);
      step(i + 3, r3, r4, r5, r1, YA, YC);
      step(i + 4, r4, r5, r0, r2, YB, YA);
      step(i + 5, r5, r0, r1, r3, YC, YB);
    }
    if (i < i1) step(i++, r0, r1, r2, r4, YA, YC);
    if (i < i1) step(i++, r1, r2, r3, r5, YB, YA);
    if (i < i1) step(i++, r2, r3, r4, r0, YC, YB);
    if (i < i1) step(i++, r3, r4, r5, r1, YA, YC);
    if (i < i1) step(i++, r4, r5, r0, r2, YB, YA);
  } else {
    // Step i: the loads of plane i+1 and of x plane i+2 go out, then plane i
    // is computed from loads issued one step earlier (four-register ring of x
    // planes, two load sets, unrolled by four).
    auto step = [&](int i, const c32x2& qm, const c32x2& qc, const c32x2& qp, c32x2& qn, const Yp& Yc, Yp& Yn) {
      load(min(i + 1, nx - 1), Yn);
      qn = L2(min(i + 2, nx - 1), e0);
      compute(i, qm, qc, qp, Yc);
    };
    c32x2 r0 = L2(max(i0 - 1, 0), e0), r1 = L2(i0, e0), r2 = L2(min(i0 + 1, nx - 1), e0), r3;
    Yp YA, YB;
    load(i0, YA);
    int i = i0;
    for (; i + 4 <= i1; i += 4) {
      step(i, r0, r1, r2, r3, YA, YB);
      step(i + 1, r1, r2, r3, r0, YB, YA);
      step(i + 2, r2, r3, r0, r1, YA, YB);
      step(i + 3, r3, r0, r1, r2, YB, YA);
    }
    if (i < i1) step(i++, r0, r1, r2, r3, YA, YB);
    if (i < i1) step(i++, r1, r2, r3, r0, YB, YA);
    if (i < i1) step(i++, r2, r3, r0, r1, YA, YB);
  }
  if (NORM) {
    const double s = block_sum(nrm, red);
    if (threadIdx.x == 0) *pslot = s;
  }
  if (ND > 0) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();  // red may still be read by the prologue's reduction
#pragma unroll
    for (int t = 0; t < ND; ++t) {
      const double sr = wave_sum(dr[t]);
      const double si = wave_sum(di[t]);
      if (lane == 0) {
        red[wid * 2 * ND + 2 * t] = sr;
        red[wid * 2 * ND + 2 * t + 1] = si;
      }
    }
    __syncthreads();
    if (threadIdx.x < 2 * ND)
      pslot[threadIdx.x] = red[threadIdx.x] + red[2 * ND + threadIdx.x] + red[4 * ND + threadIdx.x] +
                           red[6 * ND + threadIdx.x];
  }
}

// ---------------------------------------------------------------------------
// complex64 compact 27-point operator with pair tiles (same tiles, layout
// requirements and out-of-plane handling as k_h7p).  Each x plane is read
// once per lane -- the 3 x 4 (y, z) window around its pair -- and reduced to
// its contributions to the outputs of planes i-1, i and i+1.  With C the
// point, E the sum of its four in-plane face neighbours and F of its four
// in-plane diagonal neighbours:
//   same plane:       S0 = w0 C + w1 E + w2 F
//   neighbour planes: S1 = w1 C + w2 E + w3 F
// (class weights by the number of nonzero offsets), so a row of the compact
// Laplacian is S1(i-1) + S0(i) + S1(i+1) and the 27-point mass sum has the
// same form.  Layer rows take the 7-point stretched row from the tables.
//   forward:  out = (interior ? L27 x : L7 x) + omega^2 A (m . x)
//   adjoint:  out = L27 (mask . x) + L7^H ((1 - mask) . x) + omega^2 m . (A x)
// (mask = interior rows; L27 and A are symmetric).  Planes are consumed
// in order and each output is stored once its plane i+1 has been read.
// NMEM / SELF / npart: the Arnoldi inner products and input scale, as in
// k_h7p.
// ---------------------------------------------------------------------------
template <bool ADJ, bool RESID, bool NORM, int NMEM = 0, bool SELF = false>
__global__ __launch_bounds__(256) void k_h27p(const Seg* __restrict__ segs, const int* __restrict__ smap,
                                              const int* __restrict__ slocal, const c32* __restrict__ x,
                                              const double* __restrict__ xs, const c32* __restrict__ b,
                                              const double* __restrict__ bs, c32* __restrict__ out,
                                              double* __restrict__ part, const int* __restrict__ active,
                                              VecPtrs Vd = VecPtrs{}, const double* __restrict__ npart = nullptr,
                                              int stage = 0) {
  constexpr int ND = NMEM + (SELF ? 1 : 0);
  static_assert(!(ND > 0 && (RESID || NORM)), "inner products only with the plain operator");
  __shared__ double red[ND > 0 ? 4 * 2 * ND : 16];
  extern __shared__ __attribute__((aligned(16))) char stage_lds[];
  const int wg = xcd_logical(blockIdx.x, gridDim.x);
  const int sid = smap[wg];
  const int local = slocal[wg];
  const Seg& S = segs[sid];
  double* const pslot = (NORM || ND > 0) ? part + (int64_t)(S.sblk0 + local) * PSTRIDE : nullptr;
  if (active && !active[sid]) {
    if (NORM && threadIdx.x == 0) *pslot = 0.0;
    if (ND > 0 && threadIdx.x < 2 * ND) pslot[threadIdx.x] = 0.0;
    return;
  }
  const int nx = S.n[0], ny = S.n[1], nz = S.n[2], pz = S.pz;
  const int plane = ny * pz;  // even
  const int npair = plane >> 1;
  const int xc = local / S.plane_blocks;
  const int pb = local - xc * S.plane_blocks;
  const int q0 = pb * 256 + threadIdx.x;
  const bool in = q0 < npair;
  const int e0 = 2 * (in ? q0 : npair - 1);
  const int j = e0 / pz, k0 = e0 - j * pz;  // k0 even, k0 + 1 < pz
  const bool pad1 = k0 + 1 >= nz;
  const Int27& I27 = S.in27;
  const Tab7<float> tab = seg_tables<float>(S);
  // The window of a plane: rows j-1, j, j+1 by columns k0-1 .. k0+2, read
  // through byte offsets inside the plane (a plane holds fewer than 2^28
  // points) from a plane resource that is the same for the whole workgroup.
  // Entries outside the grid get an offset beyond every plane resource and
  // so read zero.  The pair k0, k0+1 is always inside a row (k0+1 may be a
  // pad column).
  constexpr uint32_t kOut = 0x80000000u;
  uint32_t obp[3], obl[3], obr[3];
  bool my[3], mz[4];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int jj = j + r - 1;
    const bool vr = jj >= 0 && jj < ny;
    my[r] = jj >= I27.lo[1] && jj <= I27.hi[1];
    const uint32_t rowp = (uint32_t)(jj * pz);
    obp[r] = vr ? (rowp + (uint32_t)k0) * 8u : kOut;
    obl[r] = vr && k0 > 0 ? (rowp + (uint32_t)k0 - 1u) * 8u : kOut;
    obr[r] = vr && k0 + 2 < nz ? (rowp + (uint32_t)k0 + 2u) * 8u : kOut;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int kk = k0 - 1 + c;
    mz[c] = kk >= I27.lo[2] && kk <= I27.hi[2];
  }
  const uint32_t obo = (uint32_t)e0 * 8u;  // the lane's output pair
  const float lw0 = (float)I27.lw[0], lw1 = (float)I27.lw[1], lw2 = (float)I27.lw[2], lw3 = (float)I27.lw[3];
  const float mw0 = (float)I27.mw[0], mw1 = (float)I27.mw[1], mw2 = (float)I27.mw[2], mw3 = (float)I27.mw[3];
  // layer rows: the stretched 7-point row with its diagonal folded,
  //   (d_x + d_y + d_z - sum of couplings) x_c + sum of couplings x_n;
  // the (y, z) part of the diagonal is fixed per lane, the x part per plane
  const c32 ay = tab.al[1][j], by = tab.be[1][j];
  c32 az[2], bz[2], cyz[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const bool pe = e == 1 && pad1;
    az[e] = pe ? czero<float>() : tab.al[2][k0 + e];
    bz[e] = pe ? czero<float>() : tab.be[2][k0 + e];
    const c32 dz = pe ? czero<float>() : tab.de[2][k0 + e];
    cyz[e] = (tab.de[1][j] + dz) - ((ay + by) + (az[e] + bz[e]));
  }
  const float w2 = (float)S.w2;
  const char* const xseg = reinterpret_cast<const char*>(x + S.off);
  const char* const mseg = reinterpret_cast<const char*>(S.m);
  // interior rows reach the edge of the grid (no layer on some side)
  const bool edge = I27.lo[0] == 0 || I27.lo[1] == 0 || I27.lo[2] == 0 || I27.hi[0] == nx - 1 ||
                    I27.hi[1] == ny - 1 || I27.hi[2] == nz - 1;
  float sx = xs ? (float)xs[sid] : 1.0f;
  if (npart) sx = (float)basis_scale(seg_sum0(npart, S.vblk0, S.vnblk, red));
  float sb = 1.0f;
  if (RESID) sb = bs ? (float)bs[sid] : 1.0f;
  const double wn = in ? 1.0 : 0.0;
  const float wf = in ? 1.0f : 0.0f;
  double dr[ND > 0 ? ND : 1], di[ND > 0 ? ND : 1];
#pragma unroll
  for (int t = 0; t < ND; ++t) dr[t] = di[t] = 0.0;
  c32x2 xself = {0.f, 0.f, 0.f, 0.f};  // stored input at the output plane (SELF)
  const int i0 = xc * S.xchunk;
  const int i1 = min(nx, i0 + S.xchunk);
  // running sums per element: output plane ip (cur) and ip+1 (next)
  c32 aL[2], aM[2], aP[2], nL[2], nM[2], xcp[2];
  float mcur[2] = {0.f, 0.f};
#pragma unroll
  for (int e = 0; e < 2; ++e) aL[e] = aM[e] = aP[e] = nL[e] = nM[e] = xcp[e] = czero<float>();
  double nrm = 0.0;
  // The pad column (k0 + 1 >= nz) holds zeros in every vector and model;
  // inputs whose pad entries reach a sum (the Laplacian of interior rows at
  // the grid edge, the adjoint's mass and layer inputs) are also zeroed
  // there explicitly.
  const bool zpad = pad1 && (ADJ || edge);
  // the window of one plane as read (zero outside the grid)
  struct Win {
    c32 X[3][4];
    float M[3][4];  // forward: the model at the window
    float mown[2];  // adjoint: the model at the pair
  };
  auto load = [&](const int ip) __attribute__((always_inline)) {
    Win w;
    const prsrc rx = plane_rsrc(xseg + (int64_t)ip * plane * 8, (uint32_t)plane * 8u);
    const prsrc rm = plane_rsrc(mseg + (int64_t)ip * plane * 4, (uint32_t)plane * 4u);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const c32x2 pr = pld_c2(rx, obp[r]);
      w.X[r][0] = pld_c(rx, obl[r]);
      w.X[r][1] = mk(pr.a, pr.b);
      w.X[r][2] = mk(pr.c, pr.d);
      w.X[r][3] = pld_c(rx, obr[r]);
      if (!ADJ) {
        const c32 mp = pld_c(rm, obp[r] >> 1);
        w.M[r][0] = pld_f(rm, obl[r] >> 1);
        w.M[r][1] = mp.re;
        w.M[r][2] = mp.im;
        w.M[r][3] = pld_f(rm, obr[r] >> 1);
      }
    }
    if (ADJ) {
      const c32 mp = pld_c(rm, obp[1] >> 1);
      w.mown[0] = mp.re;
      w.mown[1] = mp.im;
    }
    return w;
  };
  auto zero_win = [&]() __attribute__((always_inline)) {
    Win w;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        w.X[r][c] = czero<float>();
        w.M[r][c] = 0.0f;
      }
    w.mown[0] = w.mown[1] = 0.0f;
    return w;
  };
  // Consume plane ip from its window w.  OUT: the plane lies outside the
  // grid (all its values are zero); EMIT: output plane ip - 1 is complete
  // after it.
  // DEFER: leave the output pair in `pend` (stored by the caller after the
  // plane's barrier, so its store overlaps the next plane instead of the
  // barrier's wait for every outstanding memory operation).
  c32x2 pend = {0.f, 0.f, 0.f, 0.f};
  // the residual's right-hand side and the Arnoldi basis vectors at an output
  // plane, loaded ahead (staged path: before the next plane's fill, so that
  // waiting for them does not also wait for the fill)
  struct Pre {
    c32x2 bv;
    c32x2 dv[NMEM > 0 ? NMEM : 1];
  };
  auto preload = [&](const int ipo) __attribute__((always_inline)) {
    Pre pr;
    const int64_t pob = (int64_t)ipo * plane * 8;
    if (RESID) pr.bv = pld_c2(plane_rsrc(reinterpret_cast<const char*>(b + S.off) + pob, (uint32_t)plane * 8u), obo);
#pragma unroll
    for (int t = 0; t < NMEM; ++t)
      pr.dv[t] = *reinterpret_cast<const c32x2*>(reinterpret_cast<const char*>(Vd.v[t] + S.off) + pob + obo);
    return pr;
  };
  auto step = [&](const int ip, const Win& w, auto out_c, auto emit_c, auto defer_c,
                  const Pre* pre = nullptr) __attribute__((always_inline)) {
    constexpr bool OUT = decltype(out_c)::value;
    constexpr bool EMIT = decltype(emit_c)::value;
    constexpr bool DEFER = decltype(defer_c)::value;
    c32 X[3][4];
    float M[3][4];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        X[r][c] = OUT ? czero<float>() : w.X[r][c];
        M[r][c] = (OUT || ADJ) ? 0.0f : w.M[r][c];
      }
    c32x2 xcen;  // the stored pair of this plane (SELF)
    xcen.a = X[1][1].re; xcen.b = X[1][1].im; xcen.c = X[1][2].re; xcen.d = X[1][2].im;
    const float mown[2] = {OUT ? 0.0f : w.mown[0], OUT ? 0.0f : w.mown[1]};
#pragma unroll
    for (int r = 0; r < 3; ++r)
      if (zpad) X[r][2] = czero<float>();
    c32 bx = czero<float>(), dxx = czero<float>();
    bool mx = false;
    if (!OUT) {
      mx = (ip >= I27.lo[0]) & (ip <= I27.hi[0]);
      bx = uload(tab.be[0], ip);
      dxx = uload(tab.de[0], ip) - (uload(tab.al[0], ip) + bx);
    }
    // inputs of the Laplacian (XL), layer-row (XP) and mass (XA) parts
    c32 XL[3][4], XP[3][4], XA[3][4];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const bool inr = mx & my[r] & mz[c];  // bitwise: no branch on the uniform mx
        XL[r][c] = (!ADJ || inr) ? X[r][c] : czero<float>();
        XP[r][c] = ADJ ? X[r][c] - XL[r][c] : X[r][c];  // exact: X - X or X - 0
        XA[r][c] = ADJ ? X[r][c] : M[r][c] * X[r][c];
      }
    // column sums of rows j-1 and j+1 (shared by both elements)
    c32 VL[4], VA[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      VL[c] = XL[0][c] + XL[2][c];
      VA[c] = XA[0][c] + XA[2][c];
    }
    c32 ax = czero<float>();
    if (EMIT) ax = uload(tab.al[0], ip - 1);
    c32 fin[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const c32 CL = XL[1][e + 1];
      const c32 EL = (XL[1][e] + XL[1][e + 2]) + VL[e + 1];
      const c32 FL = VL[e] + VL[e + 2];
      const c32 CA = XA[1][e + 1];
      const c32 EA = (XA[1][e] + XA[1][e + 2]) + VA[e + 1];
      const c32 FA = VA[e] + VA[e + 2];
      const c32 S0L = lw0 * CL + lw1 * EL + lw2 * FL, S1L = lw1 * CL + lw2 * EL + lw3 * FL;
      const c32 S0M = mw0 * CA + mw1 * EA + mw2 * FA, S1M = mw1 * CA + mw2 * EA + mw3 * FA;
      // layer row ip: every term but the one of plane ip + 1
      const c32 xcn = XP[1][e + 1];
      c32 seed = (dxx + cyz[e]) * xcn;
      seed = cfma(ay, XP[2][e + 1], seed);
      seed = cfma(by, XP[0][e + 1], seed);
      seed = cfma(az[e], XP[1][e + 2], seed);
      seed = cfma(bz[e], XP[1][e], seed);
      seed = cfma(bx, xcp[e], seed);
      if (EMIT) {  // output ip - 1 is complete
        const c32 L = aL[e] + S1L, Mm = aM[e] + S1M;
        const c32 P = cfma(ax, xcn, aP[e]);
        c32 o;
        if (!ADJ) {
          const bool own = ((ip - 1) >= I27.lo[0]) & ((ip - 1) <= I27.hi[0]) & my[1] & mz[e + 1];
          o = (own ? L : P) + w2 * Mm;
        } else {
          o = L + P + (w2 * mcur[e]) * Mm;
        }
        fin[e] = sx * o;
      }
      // output ip starts; ip + 1 is seeded
      aP[e] = seed;
      xcp[e] = xcn;
      aM[e] = nM[e] + S0M;
      nM[e] = S1M;
      aL[e] = nL[e] + S0L;
      nL[e] = S1L;
    }
    if (EMIT) {
      c32 o0 = fin[0], o1 = fin[1];
      const int64_t pob = (int64_t)(ip - 1) * plane * 8;
      const uint32_t pbytes = (uint32_t)plane * 8u;
      if (RESID) {
        const c32x2 bv = pre ? pre->bv : pld_c2(plane_rsrc(reinterpret_cast<const char*>(b + S.off) + pob, pbytes), obo);
        o0 = sb * mk(bv.a, bv.b) - o0;
        o1 = sb * mk(bv.c, bv.d) - o1;
      }
      if (pad1) o1 = czero<float>();
      c32x2 ov;
      ov.a = o0.re; ov.b = o0.im; ov.c = o1.re; ov.d = o1.im;
      if (DEFER) pend = ov;
      else pst_c2(ov, plane_rsrc(reinterpret_cast<char*>(out + S.off) + pob, pbytes), obo);
      if (NORM)
        nrm += wn * ((double)o0.re * (double)o0.re + (double)o0.im * (double)o0.im +
                     ((double)o1.re * (double)o1.re + (double)o1.im * (double)o1.im));
      if (ND > 0) {
        const c32 u0 = wf * o0, u1 = wf * o1;  // duplicates count zero
#pragma unroll
        for (int t = 0; t < ND; ++t) {
          const c32x2 v =
              (SELF && t == ND - 1)
                  ? xself
                  : (pre ? pre->dv[t < NMEM ? t : 0]
                         : *reinterpret_cast<const c32x2*>(
                               reinterpret_cast<const char*>(Vd.v[t < NMEM ? t : 0] + S.off) + pob + obo));
          dr[t] += (double)v.a * u0.re + (double)v.b * u0.im + ((double)v.c * u1.re + (double)v.d * u1.im);
          di[t] += (double)v.a * u0.im - (double)v.b * u0.re + ((double)v.c * u1.im - (double)v.d * u1.re);
        }
      }
    }
    xself = xcen;
    if (ADJ) {
      mcur[0] = mown[0];
      mcur[1] = mown[1];
    }
  };
  // planes max(i0-1, 0) .. i1 complete outputs i0 .. i1-1; plane -1 is
  // outside the grid and adds nothing to the zero start, plane nx only
  // completes output nx - 1.
  const int ip0 = i0 > 0 ? i0 - 1 : 0;
  if (stage) {
    // Staged planes: the tile of a plane -- the workgroup's 512 points with
    // one row and two points of halo on each side -- is copied into LDS by
    // buffer loads that write LDS directly, one plane ahead into the other
    // of two buffers, while the current plane's sums run from LDS.  Tile
    // entries outside the plane read zero; window columns outside the row
    // read a zero slot.
    const int T0 = pb * 512 - pz - 2;  // first tile point (even)
    const int TL = 512 + 2 * pz + 4;   // tile points (even)
    const int Tm0 = T0 & ~3;           // model tile from a multiple of 4 (16-byte chunks)
    const int TLm = (T0 - Tm0 + TL + 3) & ~3;
    const uint32_t mt = (uint32_t)TL * 8u;  // model tile offset (16-byte aligned)
    const uint32_t zoff = (mt + (uint32_t)TLm * 4u + 15u) & ~15u;
    const uint32_t bstride = zoff + 16u;  // one buffer: x tile, m tile, zero slot
    const bool m16 = (plane & 3) == 0;    // no 16-byte model chunk straddles the plane's end
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (threadIdx.x < 2) *reinterpret_cast<c32x2*>(stage_lds + threadIdx.x * bstride + zoff) = c32x2{0.f, 0.f, 0.f, 0.f};
    uint32_t lxp[3], lxl[3], lxr[3], lmp[3], lml[3], lmr[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const uint32_t it = (uint32_t)(e0 - T0 + (r - 1) * pz);
      const uint32_t im = (uint32_t)(e0 - Tm0 + (r - 1) * pz);
      lxp[r] = it * 8u;
      lxl[r] = k0 > 0 ? (it - 1u) * 8u : zoff;
      lxr[r] = k0 + 2 < nz ? (it + 2u) * 8u : zoff;
      lmp[r] = mt + im * 4u;
      lml[r] = k0 > 0 ? mt + (im - 1u) * 4u : zoff;
      lmr[r] = k0 + 2 < nz ? mt + (im + 2u) * 4u : zoff;
    }
    auto fill = [&](const int ip, const uint32_t boff) __attribute__((always_inline)) {
      const prsrc rx = plane_rsrc(xseg + (int64_t)ip * plane * 8, (uint32_t)plane * 8u);
      const prsrc rm = plane_rsrc(mseg + (int64_t)ip * plane * 4, (uint32_t)plane * 4u);
      for (int c0 = 0; c0 < TL / 2; c0 += 256) {  // x: 16-byte chunks (two points)
        const int c = c0 + (int)threadIdx.x;
        if (c < TL / 2)
          pld_lds16(rx, stage_lds + boff + (uint32_t)(c0 + wave * 64) * 16u, (uint32_t)((T0 + 2 * c) * 8));
      }
      if (m16) {
        for (int c0 = 0; c0 < TLm / 4; c0 += 256) {  // m: 16-byte chunks (four points)
          const int c = c0 + (int)threadIdx.x;
          if (c < TLm / 4)
            pld_lds16(rm, stage_lds + boff + mt + (uint32_t)(c0 + wave * 64) * 16u, (uint32_t)((Tm0 + 4 * c) * 4));
        }
      } else {
        for (int c0 = 0; c0 < TLm; c0 += 256) {  // m: one point per lane
          const int c = c0 + (int)threadIdx.x;
          if (c < TLm)
            pld_lds4(rm, stage_lds + boff + mt + (uint32_t)(c0 + wave * 64) * 4u, (uint32_t)((Tm0 + c) * 4));
        }
      }
    };
    auto read_win = [&](const uint32_t boff) __attribute__((always_inline)) {
      Win w;
      const char* const lb = stage_lds + boff;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const c32x2 pr = *reinterpret_cast<const c32x2*>(lb + lxp[r]);
        w.X[r][0] = *reinterpret_cast<const c32*>(lb + lxl[r]);
        w.X[r][1] = mk(pr.a, pr.b);
        w.X[r][2] = mk(pr.c, pr.d);
        w.X[r][3] = *reinterpret_cast<const c32*>(lb + lxr[r]);
        if (!ADJ) {
          const c32 mp = *reinterpret_cast<const c32*>(lb + lmp[r]);
          w.M[r][0] = *reinterpret_cast<const float*>(lb + lml[r]);
          w.M[r][1] = mp.re;
          w.M[r][2] = mp.im;
          w.M[r][3] = *reinterpret_cast<const float*>(lb + lmr[r]);
        }
      }
      if (ADJ) {
        const c32 mp = *reinterpret_cast<const c32*>(lb + lmp[1]);
        w.mown[0] = mp.re;
        w.mown[1] = mp.im;
      }
      return w;
    };
    auto settle = [&]() __attribute__((always_inline)) {
      wait_vmem();
      __syncthreads();
    };
    auto flush = [&](const int ipo) __attribute__((always_inline)) {  // the deferred output plane ipo
      pst_c2(pend, plane_rsrc(reinterpret_cast<char*>(out + S.off) + (int64_t)ipo * plane * 8, (uint32_t)plane * 8u),
             obo);
    };
    // Each plane's window is read from LDS before the next plane's fill is
    // issued: an LDS read after the fill would wait for it (the fill may
    // write any LDS address as far as the compiler knows), so this order
    // lets the plane's arithmetic run while its wave's fill is in flight.
    uint32_t cur = 0;
    fill(ip0, cur);
    settle();
    int ip = ip0;
    for (; ip <= i0; ++ip) {
      const Win w = read_win(cur);
      if (ip + 1 < nx) fill(ip + 1, bstride - cur);
      step(ip, w, std::false_type{}, std::false_type{}, std::false_type{});
      settle();
      cur = bstride - cur;
    }
    for (; ip < i1; ++ip) {
      const Win w = read_win(cur);
      if (RESID || NMEM > 0) {
        const Pre pr = preload(ip - 1);
        if (ip + 1 < nx) fill(ip + 1, bstride - cur);
        step(ip, w, std::false_type{}, std::true_type{}, std::true_type{}, &pr);
      } else {
        if (ip + 1 < nx) fill(ip + 1, bstride - cur);
        step(ip, w, std::false_type{}, std::true_type{}, std::true_type{});
      }
      settle();
      flush(ip - 1);  // after the barrier
      cur = bstride - cur;
    }
    if (i1 < nx)
      step(i1, read_win(cur), std::false_type{}, std::true_type{}, std::false_type{});
    else
      step(i1, zero_win(), std::true_type{}, std::true_type{}, std::false_type{});
  } else {
    for (int ip = ip0; ip <= i0; ++ip) step(ip, load(ip), std::false_type{}, std::false_type{}, std::false_type{});
    for (int ip = i0 + 1; ip < i1; ++ip)
      step(ip, load(ip), std::false_type{}, std::true_type{}, std::false_type{});
    if (i1 < nx)
      step(i1, load(i1), std::false_type{}, std::true_type{}, std::false_type{});
    else
      step(i1, zero_win(), std::true_type{}, std::true_type{}, std::false_type{});
  }
  if (NORM) {
    const double s = block_sum(nrm, red);
    if (threadIdx.x == 0) *pslot = s;
  }
  if (ND > 0) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();  // red may still be read by the prologue's reduction
#pragma unroll
    for (int t = 0; t < ND; ++t) {
      const double sr = wave_sum(dr[t]);
      const double si = wave_sum(di[t]);
      if (lane == 0) {
        red[wid * 2 * ND + 2 * t] = sr;
        red[wid * 2 * ND + 2 * t + 1] = si;
      }
    }
    __syncthreads();
    if (threadIdx.x < 2 * ND)
      pslot[threadIdx.x] = red[threadIdx.x] + red[2 * ND + threadIdx.x] + red[4 * ND + threadIdx.x] +
                           red[6 * ND + threadIdx.x];
  }
}

// ---------------------------------------------------------------------------
// compact 27-point operator (one output point per lane, neighbours through
// the vector cache).  Interior rows: L27 = sum over the 27 offsets of the
// class weight; layer rows: the 7-point stretched row from the tables.  Mass
// term on every row: omega^2 sum_d wm(class d) m_{p+d} x_{p+d}.
// Adjoint: L27 (mask . x) + L7^H ((1 - mask) . x) + omega^2 m_p (A x)_p.
// Point-wise workgroups (tmap / tblk0).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool interior27(const Int27& in27, int i, int j, int k) {
  return i >= in27.lo[0] && i <= in27.hi[0] && j >= in27.lo[1] && j <= in27.hi[1] &&
         k >= in27.lo[2] && k <= in27.hi[2];
}

template <typename TC, typename TX, typename TM, typename TB, typename TO, bool RESID, bool NORM>
__global__ __launch_bounds__(256) void k_h27(const Seg* __restrict__ segs, const int* __restrict__ tmap,
                                             const cx<TX>* __restrict__ x, const double* __restrict__ xs,
                                             const cx<TB>* __restrict__ b, const double* __restrict__ bs,
                                             cx<TO>* __restrict__ out, double* __restrict__ part,
                                             const int* __restrict__ active) {
  __shared__ double red[16];
  const int wg = xcd_logical(blockIdx.x, gridDim.x);
  const int sid = tmap[wg];
  const Seg& S = segs[sid];
  if (active && !active[sid]) {
    if (NORM && threadIdx.x == 0) part[(int64_t)wg * PSTRIDE] = 0.0;
    return;
  }
  const int nx = S.n[0], ny = S.n[1], nz = S.n[2], pz = S.pz;
  const int64_t N = S.N;
  const int64_t p = (int64_t)(wg - S.tblk0) * 256 + threadIdx.x;
  const bool adj = S.dir != 0;
  const int64_t plane = (int64_t)ny * pz;
  double nrm = 0.0;
  if (p < N && (int)(p % pz) >= nz) {
    out[S.off + p] = czero<TO>();  // pitch pad
  } else if (p < N) {
    const Tab7<TC> tab = seg_tables<TC>(S);
    const TC w2 = (TC)S.w2;
    const TM* __restrict__ m = reinterpret_cast<const TM*>(S.m);
    const int k = (int)(p % pz);
    const int j = (int)((p / pz) % ny);
    const int i = (int)(p / plane);
    const cx<TX>* xr = x + S.off;
    const TC sx = xs ? (TC)xs[sid] : TC(1);
    const Int27& in27 = S.in27;
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
          const int64_t q = p + (int64_t)di * plane + (int64_t)dj * pz + dk;
          const cx<TC> xq = (cls == 0) ? xcur : ld<TX, TC>(xr + q);
          if (!adj) {
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
    if (!adj) {
      if (!own_int) {
        const cx<TC> xmx = i > 0 ? ld<TX, TC>(xr + p - plane) : czero<TC>();
        const cx<TC> xpx = i + 1 < nx ? ld<TX, TC>(xr + p + plane) : czero<TC>();
        const cx<TC> xmy = j > 0 ? ld<TX, TC>(xr + p - pz) : czero<TC>();
        const cx<TC> xpy = j + 1 < ny ? ld<TX, TC>(xr + p + pz) : czero<TC>();
        const cx<TC> xmz = k > 0 ? ld<TX, TC>(xr + p - 1) : czero<TC>();
        const cx<TC> xpz = k + 1 < nz ? ld<TX, TC>(xr + p + 1) : czero<TC>();
        const cx<TC> d = tab.de[0][i] + tab.de[1][j] + tab.de[2][k];
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
      const TC sb = bs ? (TC)bs[sid] : TC(1);
      acc = sb * ld<TB, TC>(b + S.off + p) - acc;
    }
    out[S.off + p] = cast<TO>(acc);
    if (NORM) nrm = (double)acc.re * (double)acc.re + (double)acc.im * (double)acc.im;
  }
  if (NORM) {
    const double s = block_sum(nrm, red);
    if (threadIdx.x == 0) part[(int64_t)wg * PSTRIDE] = s;
  }
}

}  // namespace helm
