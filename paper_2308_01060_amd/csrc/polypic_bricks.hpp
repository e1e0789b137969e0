// Brick plan shared by the scatter kernels of the staggered-grid, affine-map and
// mixture transfers.
//
// A workgroup processes a chunk of consecutive slots of the cell-key sorted order.
// Equal 4^3 tiles of stencil base nodes form runs of consecutive slots; the tiles of
// the chunk's first kWave runs are deduplicated in order of appearance, and the first
// K distinct tiles get an FP64 LDS brick each.  Slots of later tiles (and every slot
// of a chunk in arbitrary order beyond its first K tiles) add to HBM instead.
#pragma once

#include "polypic_device.hpp"

namespace polypic {

template <int BS>
struct BrickPlan {
  uint64_t tile_of[BS];     // tile of slot t
  int run_of[BS];           // run index of slot t (-1 before the first valid slot)
  uint64_t run_tile[kWave]; // tiles of the first kWave runs
  int run_brick[kWave];     // distinct-tile index of each of those runs
  int wave_heads[BS / kWave];
  int n_bricks;             // distinct tiles among the first kWave runs
};

// Called by every thread of the workgroup (it holds barriers), with the tile of the
// slot the thread processes (kNoTile if none).  Returns that slot's brick: in [0, K)
// for an LDS brick, >= K for HBM, -1 for no tile.  seg_tile[d] receives the tile of
// brick d < K; plan.n_bricks the number of distinct tiles seen.
template <int BS, int K>
__device__ __forceinline__ int plan_bricks(BrickPlan<BS>& plan, uint64_t* seg_tile, int tid,
                                           int slot, uint64_t tile) {
  constexpr int NW = BS / kWave;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  plan.tile_of[slot] = tile;
  __syncthreads();
  {
    const uint64_t tt = plan.tile_of[tid];
    const bool head = tt != kNoTile && (tid == 0 || plan.tile_of[tid - 1] != tt);
    const unsigned long long hb = __ballot(head);
    if (lane == 0) plan.wave_heads[wv] = __popcll(hb);
    __syncthreads();
    int pre = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) pre += (w < wv) ? plan.wave_heads[w] : 0;
    const int run = pre + lanes_below(hb) + (head ? 1 : 0) - 1;
    plan.run_of[tid] = run;
    if (head && run < kWave) plan.run_tile[run] = tt;
  }
  __syncthreads();
  if (wv == 0) {
    int nruns = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) nruns += plan.wave_heads[w];
    const int nr = nruns < kWave ? nruns : kWave;
    const uint64_t mine = lane < nr ? plan.run_tile[lane] : kNoTile;
    int first_same = lane;  // first run with this run's tile
    for (int q = nr - 1; q >= 0; --q)
      if (q < lane && plan.run_tile[q] == mine) first_same = q;
    const bool first = lane < nr && first_same == lane;
    const unsigned long long fb = __ballot(first);
    const int d_first = lanes_below(fb);
    const int d = __shfl(d_first, first_same, kWave);
    if (lane < nr) plan.run_brick[lane] = d;
    if (first && d < K) seg_tile[d] = mine;
    if (lane == 0) plan.n_bricks = __popcll(fb);
  }
  __syncthreads();
  const int run = plan.run_of[slot];
  // a run past the first kWave keeps a value of its own (never below K)
  return run < 0 ? -1 : (run < kWave ? plan.run_brick[run] : K + run);
}

// Slot of a thread for lane-pair scatters: pairs of consecutive sorted slots (which in
// cell order usually share a cell, hence a stencil), the pairs of a wavefront spread
// over the chunk NW pairs apart so that they sit in different cells.
template <int NW>
__device__ __forceinline__ int pair_slot(int tid) {
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  return ((((lane >> 1) * NW + wv)) << 1) | (lane & 1);
}

// Lane-pair fold of a scatter: `key` identifies what a lane scatters to (its stencil
// base, and anything else that must match; unique per lane when it scatters nothing),
// `seg` its brick.  Both lanes of a pair call it (it exchanges through DPP).  The even
// lane of a matching pair emits the sum of both lanes' node values, every other
// scattering lane its own.
struct PairFold {
  float f;    // 1 where the partner's values are added, else 0
  bool emit;  // this lane does the atomics
};
__device__ __forceinline__ PairFold pair_fold_plan(int key, int seg, bool scatters, int lane) {
  const bool pair = key == pair_swap_i(key) && seg == pair_swap_i(seg);
  PairFold pf;
  pf.f = pair ? 1.0f : 0.0f;
  pf.emit = scatters && (!pair || (lane & 1) == 0);
  return pf;
}

// Origin (first node) of the brick of tile `tl` along each axis, for bricks that start
// `below` nodes under the tile's first base node.
__device__ __forceinline__ void brick_origin(uint64_t tl, int below, int& o0, int& o1, int& o2) {
  o0 = 4 * (int)(tl & 1023u) - below;
  o1 = 4 * (int)((tl >> 10) & 1023u) - below;
  o2 = 4 * (int)((tl >> 20) & 1023u) - below;
}

}  // namespace polypic
