// helm_apply_noalloc: the operator apply of helm_apply for callers that
// cannot allocate device memory (code under stream capture, serving loops,
// harnesses that forbid hipMalloc).
//
// helm_apply keeps a cached operator (layer tables, segment descriptors and
// stencil workgroup maps) in memory it allocates on a cache miss.  This
// variant puts that description into `scratch`, a fixed array in the
// library's code object (one copy per GPU, alive until the process ends),
// and builds it there with one setup kernel from by-value arguments: no
// allocation, no host-to-device copy and no synchronisation, so the call is
// two kernel launches on the caller's stream.  The stencil kernels, and the
// layer-table kernel, are the ones helm_apply runs, so both entry points give
// bitwise identical results.
//
// The array's name is a host-side stand-in in host code: its device address
// is taken once per device with hipGetSymbolAddress (at context creation)
// and only that address is ever passed to kernels.
#pragma once

#include <mutex>

#include "operator.hip"

namespace helm {

constexpr size_t kNoallocScratchBytes = (size_t)8 << 20;  // 8 MiB per GPU

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, resolved once per device with
// that device current (the caller makes it current).
inline void* scratch_address(int device) {
  HELM_REQUIRE(device >= 0 && device < kMaxDevices, "device ordinal out of range for the scratch table");
  std::lock_guard<std::mutex> guard(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    HELM_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    HELM_REQUIRE(p != nullptr, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

// Segment descriptors of the nrhs right-hand sides (copies of `tmpl` with
// their offsets and workgroup ranges), the stencil workgroup -> (segment,
// tile) maps in the order Hierarchy::layout_stencil uses (segment fastest
// when `interleave`), and the point-wise workgroup -> segment map (tmap may
// be null when the level's kernel does not read it).
__global__ void k_noalloc_layout(Seg* segs, int* smap, int* slocal, int* tmap, Seg tmpl, int nrhs, int interleave) {
  const int64_t nsblk = (int64_t)nrhs * tmpl.snblk;
  const int64_t ntblk = tmap ? (int64_t)nrhs * tmpl.tnblk : 0;
  const int64_t n = max(max((int64_t)nrhs, nsblk), ntblk);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < nrhs) {
      Seg s = tmpl;
      s.off = i * tmpl.N;
      s.sblk0 = (int)(i * tmpl.snblk);
      s.vblk0 = (int)(i * tmpl.vnblk);
      s.tblk0 = (int)(i * tmpl.tnblk);
      segs[i] = s;
    }
    if (i < nsblk) {
      smap[i] = interleave ? (int)(i % nrhs) : (int)(i / tmpl.snblk);
      slocal[i] = interleave ? (int)(i / nrhs) : (int)(i % tmpl.snblk);
    }
    if (i < ntblk) tmap[i] = (int)(i / tmpl.tnblk);
  }
}

// y = H x / H^H x for nrhs right-hand sides, the operator description in the
// device's scratch array.  Arguments are checked by the caller.
template <typename T>
void apply_noalloc(int device, const GridSpec& g, const void* m, double omega, int adjoint, int nrhs, const void* x,
                   void* y, hipStream_t st) {
  char* base = (char*)scratch_address(device);
  const bool f32 = sizeof(T) == 4;
  const bool pairs = Hierarchy::uses_pairs(g.stencil, sizeof(T));
  // the fine level of helm_apply: the caller's layout, one direction
  Seg S;
  std::memset(&S, 0, sizeof(Seg));
  for (int a = 0; a < 3; ++a) S.n[a] = g.n[a];
  S.dir = adjoint;
  S.pz = Hierarchy::z_pitch(S.n[2], 0, pairs, false);
  S.N = (int64_t)S.n[0] * S.n[1] * S.pz;
  const bool pair = pairs && (S.pz % 2 == 0) && (int64_t)S.n[1] * S.pz < ((int64_t)1 << 28);
  S.pair = pair ? 1 : 0;
  S.plane_blocks = (int)ceil_div((int64_t)S.n[1] * S.pz, pair ? 512 : 256);
  S.xchunk = choose_xchunk_for((int64_t)S.plane_blocks * nrhs, S.n[0], pair);
  S.nxc = (S.n[0] + S.xchunk - 1) / S.xchunk;
  S.snblk = (g.stencil == 0 || pair) ? S.plane_blocks * S.nxc : 0;
  S.vnblk = (int)std::min<int64_t>(vector_blocks_cap(), ceil_div(S.N, 256));
  S.tnblk = (int)ceil_div(S.N, 256);
  S.w2 = omega * omega;
  S.m = m;
  S.tdir = 3 * (S.n[0] + S.n[1] + S.n[2]);
  S.tpre[0] = 0;
  S.tpre[1] = 3 * S.n[0];
  S.tpre[2] = 3 * (S.n[0] + S.n[1]);
  S.in27 = interior27_desc(g, S.n, g.h, 1);
  const bool point27 = g.stencil == 1 && !pair;  // k_h27 walks the point-wise map
  const int64_t nsblk = (int64_t)nrhs * S.snblk, ntblk = point27 ? (int64_t)nrhs * S.tnblk : 0;
  // scratch layout, every part on a 256-byte boundary
  auto r256 = [](int64_t b) { return (b + 255) / 256 * 256; };
  const int64_t o_segs = 0;
  const int64_t o_smap = o_segs + r256((int64_t)nrhs * sizeof(Seg));
  const int64_t o_slocal = o_smap + r256(std::max<int64_t>(nsblk, 1) * sizeof(int));
  const int64_t o_tmap = o_slocal + r256(std::max<int64_t>(nsblk, 1) * sizeof(int));
  const int64_t o_tabd = o_tmap + r256(std::max<int64_t>(ntblk, 1) * sizeof(int));
  const int64_t o_tabf = o_tabd + r256(2 * (int64_t)S.tdir * sizeof(cx<double>));
  const int64_t need = o_tabf + r256(2 * (int64_t)S.tdir * sizeof(cx<float>));
  if (need > (int64_t)kNoallocScratchBytes)
    throw Error{-1, "helm_apply_noalloc: the operator description needs " + std::to_string(need) +
                        " bytes of scratch, more than the " + std::to_string(kNoallocScratchBytes) +
                        " bytes available (fewer right-hand sides or a smaller grid, or helm_apply)"};
  S.tabd = base + o_tabd;
  S.tabf = base + o_tabf;
  launch_layer_tables(g, omega, S.n, g.h, 1, (cx<double>*)(base + o_tabd), (cx<float>*)(base + o_tabf), st);
  const bool interleave = (g.stencil == 0 || pair) && nrhs > 1 && S.N <= ((int64_t)1 << 20);
  const int64_t nlay = std::max(std::max((int64_t)nrhs, nsblk), ntblk);
  hipLaunchKernelGGL(k_noalloc_layout, dim3(std::min<unsigned>(1024, ceil_div(nlay, 256))), dim3(256), 0, st,
                     (Seg*)(base + o_segs), (int*)(base + o_smap), (int*)(base + o_slocal),
                     point27 ? (int*)(base + o_tmap) : nullptr, S, nrhs, interleave ? 1 : 0);
  HELM_HIP_CHECK(hipGetLastError());
  const int stage = pair && g.stencil == 1 ? stage27_bytes_pz(S.pz) : 0;
  const LevelView L{(const Seg*)(base + o_segs), (const int*)(base + o_smap), (const int*)(base + o_slocal),
                    (const int*)(base + o_tmap), (int)nsblk, (int)(nrhs * (int64_t)S.tnblk), g.stencil, adjoint,
                    pair, stage};
  (void)f32;
  launch_h<T, T, T, T, T, false, false>(L, (const cx<T>*)x, nullptr, (const cx<T>*)nullptr, nullptr, (cx<T>*)y,
                                        nullptr, nullptr, st);
  HELM_HIP_CHECK(hipGetLastError());
}

}  // namespace helm
