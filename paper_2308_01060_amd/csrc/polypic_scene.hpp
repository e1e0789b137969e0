// Where a processing slot's particle lives, and which chunks of the slot range
// a workgroup takes.
//
// Kernels that run over particles are templated on a scene policy:
//
// * OneScene  -- one grid for the whole launch (the single-scene entry
//   points); every lookup folds to kernel arguments at compile time.
// * SceneTable -- many independent scenes laid end to end: particle s of the
//   batch occupies flattened slots [p_begin, p_end) of its scene, and scene
//   grids occupy disjoint node ranges [node_off, node_off + nx*ny*nz) of the
//   flattened grid arrays.  A sort permutation from the batched sort keeps
//   every particle inside its scene's slot range, so the scene of slot i is
//   the scene of the particle read there.
#pragma once

#include "polypic_device.hpp"

namespace polypic {

// Device copy of one batch scene, written by polypic_batch_plan.
struct alignas(16) SceneDev {
  int32_t nx, ny, nz;
  float inv_dx;
  float ox, oy, oz;
  float dx;
  float lo[3];       // advection clamp bounds
  float hi[3];
  int64_t p_begin;   // flattened particle range [p_begin, p_end)
  int64_t p_end;
  int64_t node_off;  // first node of the scene in the flattened grid arrays
};

// What a kernel needs to know about the grid of one scene.
struct SceneGrid {
  int nx, ny, nz;
  float inv_dx;
  float ox, oy, oz;
  float dx;
  float lo[3], hi[3];
  int64_t node_off;
};

struct OneScene {
  static constexpr bool kMany = false;
  SceneGrid sg;
  __device__ __forceinline__ int first(int64_t) const { return 0; }
  __device__ __forceinline__ int of(int64_t, int) const { return 0; }
  __device__ __forceinline__ SceneGrid grid(int) const { return sg; }
};

struct SceneTable {
  static constexpr bool kMany = true;
  const SceneDev* t;
  int n;
  // Scene holding slot i (0 <= i < total particles): the last scene whose
  // range starts at or before i.  Empty scenes share their start with the
  // next one, so the last such scene is the one that holds i.
  __device__ __forceinline__ int first(int64_t i) const {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (t[mid].p_begin <= i)
        lo = mid;
      else
        hi = mid - 1;
    }
    return lo;
  }
  // Scene of slot i >= the first slot of scene s.
  __device__ __forceinline__ int of(int64_t i, int s) const {
    while (s + 1 < n && i >= t[s].p_end) ++s;
    return s;
  }
  __device__ __forceinline__ SceneGrid grid(int s) const {
    const SceneDev& d = t[s];
    SceneGrid g;
    g.nx = d.nx;
    g.ny = d.ny;
    g.nz = d.nz;
    g.inv_dx = d.inv_dx;
    g.ox = d.ox;
    g.oy = d.oy;
    g.oz = d.oz;
    g.dx = d.dx;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      g.lo[k] = d.lo[k];
      g.hi[k] = d.hi[k];
    }
    g.node_off = d.node_off;
    return g;
  }
};

// ------------------------------------------------------------ chunk schedule
// A launch over C chunks of slots (one chunk = one workgroup's worth).
//   kSchedLinear: one chunk per workgroup, chunk = workgroup index.
//   kSchedXcd:    one chunk per workgroup, renumbered so that the workgroups
//                 the dispatcher sends to one XCD (index mod 8) take one
//                 contiguous eighth of the chunks: neighbouring chunks (in
//                 sorted order: neighbouring cells) then share that XCD's L2.
//   kSchedPersistent: G < C workgroups, each a contiguous share of the
//                 chunks, shares ordered by XCD as above.
constexpr int kSchedLinear = 0;
constexpr int kSchedXcd = 1;
constexpr int kSchedPersistent = 2;
constexpr int kXcds = 8;

struct ChunkRange {
  int64_t begin, end;
};

__device__ __forceinline__ ChunkRange block_chunks(int mode, int64_t n_chunks) {
  const int64_t b = blockIdx.x;
  const int64_t G = gridDim.x;
  if (mode == kSchedLinear) return {b, b + 1};
  const int64_t x = b % kXcds;
  const int64_t k = b / kXcds;
  const int64_t q = G / kXcds;
  const int64_t r = G % kXcds;
  const int64_t rank = x * q + (x < r ? x : r) + k;  // a bijection of [0, G)
  if (mode == kSchedXcd) return {rank, rank + 1};
  return {rank * n_chunks / G, (rank + 1) * n_chunks / G};
}

}  // namespace polypic
