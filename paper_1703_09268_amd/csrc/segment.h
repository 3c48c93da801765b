// Segment descriptors: one problem (grid, omega, model, direction) on one
// level of the multigrid hierarchy.  A solve advances a list of segments
// together; every kernel covers all of them in one launch and finds its
// segment through a workgroup -> segment map built on the host.  Several
// right-hand sides of one operator are segments that share the grid, the
// model and the layer tables; a batch of uneven problems is a list of
// segments with different grids.
#pragma once

#include "common.h"

namespace helm {

// 27-point interior description (compact stencil away from the layer).
struct Int27 {
  int lo[3], hi[3];  // rows with lo <= i <= hi on every axis are interior
  double lw[4];      // Laplacian weights: centre, face, edge, corner
  double mw[4];      // mass weights: centre, face, edge, corner
};

struct Seg {
  int n[3];
  int dir;            // 0: H, 1: H^H
  int pz;             // z pitch of the level's vectors: n2, or n2 + 1 to make it even
                      // (coarse levels of the pair-tiled 7-point path; the pad
                      // entries of every vector and model are kept at zero)
  int pair;           // stencil tiles of 256 lanes x 2 consecutive z-points
  int64_t N;          // n0*n1*pz (vector length including pads)
  int64_t off;        // element offset of this segment in a level vector
  // stencil launch: flattened (y,z) plane tiles of 256 lanes, x chunks
  int plane_blocks;   // ceil(n1*n2 / 256), or ceil(n1*pz / 512) with pair tiles
  int xchunk, nxc;    // x planes per workgroup, number of x chunks
  int sblk0, snblk;   // stencil workgroups [sblk0, sblk0 + snblk)
  int vblk0, vnblk;   // vector-kernel workgroups (grid-stride over N)
  int tblk0, tnblk;   // point-wise workgroups (one lane per point)
  double w2;          // omega^2
  const void* m;      // model on this level (float or double)
  const void* tabf;   // layer tables, complex<float>:  [dir][axis][alpha,beta,delta][n_axis]
  const void* tabd;   // layer tables, complex<double>
  int tpre[3];        // offset of axis a inside one direction: 3*(n0+..+n_{a-1})
  int tdir;           // size of one direction: 3*(n0+n1+n2)
  Int27 in27;
};

// XCD-aware workgroup order.  The hardware deals consecutive workgroup ids to
// the 8 XCDs round robin; this returns a logical id such that the ids one XCD
// executes form one contiguous range, so neighbouring tiles (which share
// halo planes and rows) are cached in the same L2.
__device__ __forceinline__ int xcd_logical(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

}  // namespace helm
