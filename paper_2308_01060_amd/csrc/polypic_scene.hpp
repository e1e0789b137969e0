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
//   the scene of the particle read there.  A workgroup's chunk of kSceneChunk
//   slots may straddle scenes.
// * SceneChunks -- the same layout, but every workgroup takes a chunk inside one
//   scene (each scene is cut into chunks of its own, the last one partial), so
//   that the scene's grid is uniform over the workgroup and lives in scalar
//   registers.  The launch has (total particles) / kSceneChunk + (scenes) + 1
//   workgroups at most; those past the last chunk return at once.
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
  int64_t chunk_begin;  // chunks of kSceneChunk slots of the scenes before this one
  int64_t region_begin; // active regions of the scenes before this one
};

// slots per workgroup chunk of the SceneChunks schedule
constexpr int kSceneChunk = 256;

// Slots a workgroup processes: [i0, i0 + n) (n <= 0: none), in scene s (the scene
// of slot i0).
struct Chunk {
  int64_t i0;
  int n;
  int s;
};

// What a kernel needs to know about the grid of one scene.
struct SceneGrid {
  int nx, ny, nz;
  float inv_dx;
  float ox, oy, oz;
  float dx;
  float lo[3], hi[3];
  int64_t node_off;
  int64_t region_off;  // first region flag of the scene
};

struct OneScene {
  static constexpr bool kMany = false;
  SceneGrid sg;
  // chunk b of the launch (b < the launch's workgroups)
  template <int BS>
  __device__ __forceinline__ Chunk chunk(int64_t P, int64_t b) const {
    const int64_t i0 = b * BS;
    return {i0, (int)min((int64_t)BS, P - i0), 0};
  }
  __device__ __forceinline__ int first(int64_t) const { return 0; }
  __device__ __forceinline__ int of(int64_t, int) const { return 0; }
  __device__ __forceinline__ SceneGrid grid(int) const { return sg; }
};

struct SceneTable {
  static constexpr bool kMany = true;
  const SceneDev* t;
  int n;
  template <int BS>
  __device__ __forceinline__ Chunk chunk(int64_t P, int64_t b) const {
    const int64_t i0 = b * BS;
    return {i0, (int)min((int64_t)BS, P - i0), first(i0)};
  }
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
    g.region_off = d.region_begin;
    return g;
  }
};

struct SceneChunks {
  static constexpr bool kMany = false;  // one scene per workgroup
  const SceneDev* t;
  int n;
  // Chunk b: the last scene whose first chunk is at or before b (empty scenes share
  // their first chunk with the next scene, so the last such is the one holding it),
  // and the chunk's slots in that scene.
  template <int BS>
  __device__ __forceinline__ Chunk chunk(int64_t, int64_t b) const {
    static_assert(BS == kSceneChunk, "chunks are planned for kSceneChunk slots");
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (t[mid].chunk_begin <= b)
        lo = mid;
      else
        hi = mid - 1;
    }
    const SceneDev& d = t[lo];
    const int64_t i0 = d.p_begin + (b - d.chunk_begin) * BS;
    const int64_t left = d.p_end - i0;
    return {i0, (int)(left < 0 ? 0 : (left < BS ? left : BS)), lo};
  }
  __device__ __forceinline__ int of(int64_t, int s) const { return s; }
  __device__ __forceinline__ SceneGrid grid(int s) const { return SceneTable{t, n}.grid(s); }
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
