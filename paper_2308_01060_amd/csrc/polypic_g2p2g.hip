// G2P of one step fused with the P2G of the next, for gfx950.
//
// G2P reads no coefficients: the new ones come from the grid velocity alone
// (Eq. 6-8, section 3.3), and the next step's P2G (Eq. 1, 4, 13) is their only
// reader.  One thread per output slot i (particle perm[i]) therefore does:
//
//   * G2P at the particle's position: gather the 27 node velocities per
//     component, project them onto the first n_modes modes, write the new
//     coefficients, the advected position x' (and F', mass) at slot i;
//   * P2G at x' with the coefficients still in registers: the stencil of x',
//     the weighted mode rows, and the nodal mass and momentum streamed node by
//     node into FP64 LDS bricks of 4^3-node tiles (lane pairs that share a
//     base node add across lanes first), then one float atomic per brick node
//     and channel into the next grid.
//
// The coefficient array is written once and never read back, instead of being
// written by G2P and read again by the next step's P2G: the particle stream
// drops from 40 + 24 n_modes to 28 + 12 n_modes bytes per particle.  The result
// is the G2P call followed by the P2G call on its outputs, up to the order of
// the floating-point sums.
#include "polypic_internal.hpp"

namespace polypic {

namespace {

// Slot of a thread: lane groups of G = 2^LG consecutive slots (which in cell
// order usually share a cell, hence a base node), the groups of a wavefront
// spread over the workgroup's chunk so that they sit in different cells and
// their brick atomics do not collide.
template <int LG, int NW>
__device__ __forceinline__ int fused_slot(int tid) {
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  return (((lane >> LG) * NW + wv) << LG) | (lane & ((1 << LG) - 1));
}

// Position of slot s in a staging row (a permutation of each 32 slots).  The 64
// slots one wavefront writes agree in their wavefront-index bits (LG, LG + 1) and
// differ in bits 5-7, which a plain index drops from the bank number.  XORing bit 6,
// and bits 5 ^ 7, into the wavefront-index bits puts the writes of each half
// wavefront on 32 distinct banks and those of the whole wavefront on 64, while a
// read of 64 consecutive slots only permutes each half.  (Written for 256-thread
// workgroups; any size stays a bijection.)
template <int LG>
__device__ __forceinline__ int stage_pos(int s) {
  return s ^ (((s >> 6) & 1) << LG) ^ ((((s >> 7) ^ (s >> 5)) & 1) << (LG + 1));
}

// LDS (about 40 KB per 256-thread workgroup) allows 4 waves per SIMD; the launch
// bound holds the registers to the 128 that allow them too.  At 27 modes that
// spills 6 registers and still wins (measured, 4.19 M particles: 0.40 ms at 3
// waves per SIMD without spills, 0.38 ms at 4).
// LG: log2 of the lane-group size.  Pairs (LG = 1) are the default: where the vector
// ALU is the tighter limit, one DPP fold per node value beats the two of quads
// (measured, 27 modes, 4.19 M particles at 8 per cell: 0.369 -> 0.359 ms).  Quads
// (LG = 2) spread a wavefront's groups 16 slots apart instead of 8, so that at 16
// particles per cell two groups of a wavefront do not share a cell and its LDS
// addresses; the fused autotuner picks between them on the caller's data.
template <int NR, int BS, class Scenes, int LG>
__global__ __launch_bounds__(BS, 4) void g2p2g_kernel(G2P2GArgs a, Scenes sc) {
  constexpr int NW = BS / kWave;
  static_assert(LG == 1 || LG == 2, "lane pairs or quads");
  static_assert(!Scenes::kMany, "a workgroup's slots lie in one scene (OneScene, SceneChunks)");
  __shared__ double brick[kBrickKMAX * 4 * kBrickV];  // [brick][channel][node]
  __shared__ uint64_t tile_of[BS];                    // by processing slot
  __shared__ int seg_of[BS];
  __shared__ uint64_t seg_tile[kBrickKMAX];
  __shared__ int wave_heads[NW];
  __shared__ uint64_t run_tile[kWave];  // tile of each of the first 64 runs
  __shared__ int run_brick[kWave];      // brick (distinct-tile index) of each run
  __shared__ int n_bricks;

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  const int slot = fused_slot<LG, NW>(tid);
  const size_t Ps = (size_t)a.P;
  // this workgroup's chunk (in launch order, or XCD-contiguous), its slots
  // [i0, i0 + n_slots) and the scene of the first
  const Chunk ck = sc.template chunk<BS>(a.P, block_chunks(a.sched, gridDim.x).begin);
  if (ck.n <= 0) return;  // (whole workgroup: past the last chunk of a scene-chunked launch)
  const int64_t i0 = ck.i0;
  const int n_slots = ck.n;
  const int64_t i = i0 + slot;
  const bool in = slot < n_slots;
  const SceneGrid g = sc.grid(ck.s);  // uniform over the workgroup
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int nxny = nx * ny;
  // a caller permutation is clamped into [0, P): a bad one gives wrong results, never a fault
  const int p = in ? (a.perm ? min(max(a.perm[i], 0), (int)(a.P - 1)) : (int)i) : 0;

  // ---------------------------------------------------------------- G2P
  float xp[3] = {0.f, 0.f, 0.f};
  if (in) {
    xp[0] = a.x_in[p];
    xp[1] = a.x_in[Ps + p];
    xp[2] = a.x_in[2 * Ps + p];
  }
  int b0, b1, b2;
  float t0, t1, t2;
  bool ok = stencil_axis(xp[0], g.ox, g.inv_dx, nx, b0, t0);
  ok &= stencil_axis(xp[1], g.oy, g.inv_dx, ny, b1, t1);
  ok &= stencil_axis(xp[2], g.oz, g.inv_dx, nz, b2, t2);
  if (in && !ok) raise_flag(a.status, kFlagRange);
  const bool gather = in && ok;

  float c[3][27];  // the new coefficients, kept for the P2G half
  float xn[3];     // the advected position
  // Output rows go through LDS (the bricks are not in use yet) so that every
  // wavefront writes 64 consecutive slots (measured, 27 modes, 4.19 M particles:
  // 2.0 ms with the rows written from the spread slots, 0.47 ms staged): row k of
  // a round is stage[k * BS + stage_pos(slot)], read back at stage_pos(tid).
  float* const stage = reinterpret_cast<float*>(brick);
  static_assert(28 * BS * sizeof(float) <= sizeof(brick), "staging fits in the bricks");
  const int64_t i_out = i0 + tid;  // slot this thread writes out
  const int put = stage_pos<LG>(slot), get = stage_pos<LG>(tid);
  // floats of this workgroup's rows that exist, and this thread's byte in a row
  const int row_n = n_slots;
  const int out_off = tid * (int)sizeof(float);
  const bool out_ok = tid < n_slots;
  {
    const Proj1D px = proj_g2p(t0);
    const Proj1D py = proj_g2p(t1);
    const Proj1D pz = proj_g2p(t2);
    const int64_t gbase = g.node_off + (int64_t)(b2 * ny + b1) * nx + b0;
    // every lane's stencil lies in the grid (a flagged or idle lane has base node
    // 0 and the grid at least 3 nodes per axis), so the gathers need no branch;
    // such lanes are zeroed afterwards, only in the wavefronts that hold one
    const bool any_idle = __ballot(!gather) != 0ull;
    auto gather_nodes = [&](int ax, float(&v)[27]) {
      const float* vg = a.gv + (size_t)ax * a.gstride + gbase;
#pragma unroll
      for (int jz = 0; jz < 3; ++jz)
#pragma unroll
        for (int jy = 0; jy < 3; ++jy)
#pragma unroll
          for (int jx = 0; jx < 3; ++jx) v[jx + 3 * jy + 9 * jz] = vg[jz * nxny + jy * nx + jx];
    };
    float v[27];
    gather_nodes(0, v);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      project_modes<NR>(v, px, py, pz, c[ax]);
      // the next component's gathers go out now, ahead of this component's
      // staging barriers and stores (v is free once projected)
      if (ax < 2) gather_nodes(ax + 1, v);
      if (any_idle) {
#pragma unroll
        for (int r = 0; r < NR; ++r) c[ax][r] = gather ? c[ax][r] : 0.0f;
      }
#pragma unroll
      for (int r = NR; r < 27; ++r) c[ax][r] = 0.0f;
      float x1 = fmaf(a.dt, c[ax][0], xp[ax]);
      x1 = fmaxf(x1, g.lo[ax]);
      xn[ax] = fminf(x1, g.hi[ax]);
      // rows of this component: the NR coefficients and x'; written once, never
      // re-read here, so streamed past the caches the gathers use
      float* const co = a.coeff_out + (size_t)ax * NR * Ps + i0;  // this workgroup's slots
      float* const xo = a.x_out + (size_t)ax * Ps + i0;
#pragma unroll
      for (int r = 0; r < NR; ++r) stage[r * BS + put] = c[ax][r];
      stage[NR * BS + put] = xn[ax];
      __syncthreads();
      if (out_ok) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
          row_store_nt(stage[r * BS + get], co + (size_t)r * Ps, row_n, out_off);
        row_store_nt(stage[NR * BS + get], xo, row_n, out_off);
      }
      __syncthreads();  // the next component overwrites the stage
    }
  }
  float m = 0.0f;
  if (in) m = a.mass_in ? a.mass_in[p] : a.uniform_mass;
  if (a.F_in || a.mass_out) {  // (uniform: kernel arguments)
    // F' = F + dt C F with C_ab = c[a][1 + b] / dx; rows 0-8 F', row 9 the mass
    float Fn[9];
    if (in && a.F_in) {
      float F[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) F[e] = a.F_in[(size_t)e * Ps + p];
      const float sdt = a.dt / g.dx;
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int col = 0; col < 3; ++col) {
          float acc = 0.0f;
          if constexpr (NR >= 4) {
#pragma unroll
            for (int k = 0; k < 3; ++k) acc = fmaf(c[r][1 + k], F[3 * k + col], acc);
          }
          Fn[3 * r + col] = fmaf(sdt, acc, F[3 * r + col]);
        }
    } else {
#pragma unroll
      for (int e = 0; e < 9; ++e) Fn[e] = 0.0f;
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) stage[e * BS + put] = Fn[e];
    stage[9 * BS + put] = m;
    __syncthreads();
    if (out_ok) {
      if (a.F_out) {
#pragma unroll
        for (int e = 0; e < 9; ++e)
          row_store_nt(stage[e * BS + get], a.F_out + (size_t)e * Ps + i0, row_n, out_off);
      }
      if (a.mass_out) row_store_nt(stage[9 * BS + get], a.mass_out + i0, row_n, out_off);
    }
    __syncthreads();  // the bricks are cleared next
  }

  // ---------------------------------------------------------------- P2G of x'
  bool valid = in;
  int c0 = 0, c1 = 0, c2 = 0;
  float u0 = 0.f, u1 = 0.f, u2 = 0.f;
  if (valid) {
    bool ok2 = stencil_axis(xn[0], g.ox, g.inv_dx, nx, c0, u0);
    ok2 &= stencil_axis(xn[1], g.oy, g.inv_dx, ny, c1, u1);
    ok2 &= stencil_axis(xn[2], g.oz, g.inv_dx, nz, c2, u2);
    if (!ok2) {  // (x' is clamped into the grid: only for a grid too small for a stencil)
      raise_flag(a.status, kFlagRange);
      valid = false;
    }
  }
  if (!valid) m = 0.0f;
  tile_of[slot] = valid ? brick_tile_id(0, c0, c1, c2) : kNoTile;
  static_assert(kBrickNodes <= BS, "one brick node per thread");
  const BrickNode bn = brick_node(tid);
  if (tid < kBrickNodes) {
#pragma unroll
    for (int k = 0; k < kBrickKMAX * 4; ++k) brick[k * kBrickV + bn.lds] = 0.0;
  }
  __syncthreads();

  // Bricks are given per distinct tile, not per run: the chunk is in the order of
  // the previous positions, so a particle that changed cell can split a run of
  // equal tiles, and per-run segments would then spill the rest of the chunk to
  // HBM.  Runs of equal tiles in slot order (thread t looks at slot t), then the
  // first kRuns runs' tiles deduplicated in order of appearance by wavefront 0.
  constexpr int kRuns = kWave;
  {
    const uint64_t tt = tile_of[tid];
    const bool head = tt != kNoTile && (tid == 0 || tile_of[tid - 1] != tt);
    const unsigned long long hb = __ballot(head);
    if (lane == 0) wave_heads[wv] = __popcll(hb);
    __syncthreads();
    int pre = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) pre += (w < wv) ? wave_heads[w] : 0;
    const int run = pre + lanes_below(hb) + (head ? 1 : 0) - 1;
    seg_of[tid] = run;  // run index for now (-1 before the first valid slot)
    if (head && run < kRuns) run_tile[run] = tt;
  }
  __syncthreads();
  int nruns = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) nruns += wave_heads[w];
  const int nr = nruns < kRuns ? nruns : kRuns;
  if (wv == 0) {
    const uint64_t mine = lane < nr ? run_tile[lane] : kNoTile;
    int first_same = lane;  // first run with this run's tile
    for (int q = nr - 1; q >= 0; --q)
      if (q < lane && run_tile[q] == mine) first_same = q;
    const bool first = lane < nr && first_same == lane;
    const unsigned long long fb = __ballot(first);
    // distinct index of a first run = first runs before it; a later run takes its
    // first run's index (all lanes hold a value, so the shuffle is well defined)
    const int d_first = lanes_below(fb);
    const int d = __shfl(d_first, first_same, kWave);
    if (lane < nr) run_brick[lane] = d;
    if (first && d < kBrickKMAX) seg_tile[d] = mine;
    if (lane == 0) n_bricks = __popcll(fb);
  }
  __syncthreads();
  const int run_slot = seg_of[slot];
  // brick of this slot's run; runs past kRuns, and tiles past the brick budget, go to HBM.
  // A run past kRuns keeps a value of its own (kBrickKMAX + run index, above every
  // distinct-tile index d < kRuns), so that two lanes of different runs never compare
  // equal below.
  const int seg = run_slot < 0 ? -1
                               : (run_slot < kRuns ? run_brick[run_slot] : kBrickKMAX + run_slot);
  const int nseg = n_bricks;
  if (a.regions) {
    // the regions the scatter lands in: each brick's 6^3 nodes, and the 6^3 nodes of
    // the tile of every slot that went to HBM directly (a box holding its stencil);
    // from the run bookkeeping, before the scatter holds its node values (plain stores)
    const int nb = nseg < kBrickKMAX ? nseg : kBrickKMAX;
    if (tid < 8 * nb) {
      const uint32_t tc = (uint32_t)seg_tile[tid >> 3];
      flag_box_corner(a.regions, g.region_off, (uint32_t)ck.s, nx, ny, nz,
                      (int)(tc & 1023u) * kBrickT, (int)((tc >> 10) & 1023u) * kBrickT,
                      (int)(tc >> 20) * kBrickT, kBrickN, tid & 7);
    }
    const int run_t = seg_of[tid];
    if (run_t >= 0 && (run_t >= kRuns || run_brick[run_t] >= kBrickKMAX)) {
      const uint32_t tc = (uint32_t)tile_of[tid];
#pragma unroll
      for (int corner = 0; corner < 8; ++corner)
        flag_box_corner(a.regions, g.region_off, (uint32_t)ck.s, nx, ny, nz,
                        (int)(tc & 1023u) * kBrickT, (int)((tc >> 10) & 1023u) * kBrickT,
                        (int)(tc >> 20) * kBrickT, kBrickN, corner);
    }
  }
  // the lane pair (lane ^ 1), and with quads the other pair of the quad, share this
  // lane's segment and base node: every lane runs the exchanges (an invalid one with
  // zero mass), since a DPP read from a lane that did not execute it is undefined
  const int mykey = valid ? ((c2 * 1024 + c1) * 1024 + c0) : -1 - lane;
  const int pair_key = pair_swap_i(mykey), pair_seg = pair_swap_i(seg);
  const bool pair = mykey == pair_key && seg == pair_seg;
  bool quad = false;
  if constexpr (LG == 2) {
    const int quad_pair = quad_swap_i((int)pair), quad_key = quad_swap_i(mykey);
    const int quad_seg = quad_swap_i(seg);
    quad = pair && quad_pair != 0 && mykey == quad_key && seg == quad_seg;
  }
  const bool emit = valid && (quad ? (lane & 3) == 0 : (!pair || (lane & 1) == 0));
  const float pair_f = pair ? 1.0f : 0.0f;
  const float quad_f = quad ? 1.0f : 0.0f;
  {
    const Rows Rx = p2g_rows_scaled(basis_p2g(u0), m);
    const Rows Ry = p2g_rows_scaled(basis_p2g(u1), 1.0f);
    const Rows Rz = p2g_rows_scaled(basis_p2g(u2), 1.0f);
    const bool lds = seg < kBrickKMAX;
    const int lbase = (c0 & 3) + kBrickSY * (c1 & 3) + kBrickSZ * (c2 & 3);
    const int64_t gbase = g.node_off + (int64_t)(c2 * ny + c1) * nx + c0;
    double* const lb = brick + (lds ? max(seg, 0) : 0) * 4 * kBrickV + lbase;
    // one plane of 9 node values at a time: the folds run on every lane, then a
    // single predicated block per plane does the atomics
    auto emitter = [&](int ch) {
      double* const lbc = lb + ch * kBrickV;
      // (the HBM base is formed only on that rare path, to keep registers free)
      float* const gc = ch == 0 ? a.gm : ch == 1 ? a.gp0 : ch == 2 ? a.gp1 : a.gp2;
      return [=](int jz, float (&v)[9]) {
        float w[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          w[k] = pair_fold(v[k], pair_f);
          if constexpr (LG == 2) w[k] = quad_fold(w[k], quad_f);
        }
        if (!emit) return;
        if (lds) {
#pragma unroll
          for (int jy = 0; jy < 3; ++jy)
#pragma unroll
            for (int jx = 0; jx < 3; ++jx)
              atomicAdd(lbc + jx + kBrickSY * jy + kBrickSZ * jz, (double)w[jx + 3 * jy]);
        } else {
#pragma unroll
          for (int jy = 0; jy < 3; ++jy)
#pragma unroll
            for (int jx = 0; jx < 3; ++jx)
              atomicAdd(gc + gbase + (jz * nxny + jy * nx + jx), w[jx + 3 * jy]);
        }
      };
    };
    {  // mass: m W_ip
      float one[27];
#pragma unroll
      for (int r = 0; r < 27; ++r) one[r] = r == 0 ? 1.0f : 0.0f;
      stream_modes_planes<1>(one, Rx, Ry, Rz, emitter(0));
    }
    stream_modes_planes<NR>(c[0], Rx, Ry, Rz, emitter(1));
    stream_modes_planes<NR>(c[1], Rx, Ry, Rz, emitter(2));
    stream_modes_planes<NR>(c[2], Rx, Ry, Rz, emitter(3));
  }
  __syncthreads();

  // flush: one global float atomic per channel per non-zero brick node, by the
  // node's owner thread
  const int nb = nseg < kBrickKMAX ? nseg : kBrickKMAX;

  if (tid < kBrickNodes) {
    for (int sb = 0; sb < nb; ++sb) {
      const uint32_t tc = (uint32_t)seg_tile[sb];
      const int gx = (int)(tc & 1023u) * kBrickT + bn.lx;
      const int gy = (int)((tc >> 10) & 1023u) * kBrickT + bn.ly;
      const int gz = (int)(tc >> 20) * kBrickT + bn.lz;
      if (gx >= nx || gy >= ny || gz >= nz) continue;
      const int64_t node = g.node_off + ((int64_t)(gz * ny + gy) * nx + gx);
      const double* const src = brick + sb * 4 * kBrickV + bn.lds;
      float* const dst[4] = {a.gm, a.gp0, a.gp1, a.gp2};
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) {
        const float v = (float)src[ch * kBrickV];
        if (v != 0.0f) atomicAdd(dst[ch] + node, v);
      }
    }
  }
}

template <int NR, class Scenes>
hipError_t launch_nr(const G2P2GArgs& a, const Scenes& sc, unsigned blocks, hipStream_t stream) {
  constexpr int BS = kSceneChunk;
  if (a.lane_group == 4)
    g2p2g_kernel<NR, BS, Scenes, 2><<<blocks, BS, 0, stream>>>(a, sc);
  else
    g2p2g_kernel<NR, BS, Scenes, 1><<<blocks, BS, 0, stream>>>(a, sc);
  return hipGetLastError();
}

// blocks: workgroups of kSceneChunk threads that cover every chunk
template <class Scenes>
hipError_t launch_modes(const G2P2GArgs& a, const Scenes& sc, int n_modes, int64_t n_nodes,
                        unsigned blocks, hipStream_t stream) {
  if (!a.accumulate) {
    hipError_t e = launch_grid_clear(a.gm, a.gp0, n_nodes, nullptr, stream);
    if (e != hipSuccess) return e;
  }
  if (a.P == 0) return hipSuccess;
  switch (n_modes) {
    case 1: return launch_nr<1>(a, sc, blocks, stream);
    case 4: return launch_nr<4>(a, sc, blocks, stream);
    case 8: return launch_nr<8>(a, sc, blocks, stream);
    case 27: return launch_nr<27>(a, sc, blocks, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_g2p2g(const G2P2GArgs& a, int n_modes, hipStream_t stream) {
  OneScene one;
  one.sg.nx = a.g.nx;
  one.sg.ny = a.g.ny;
  one.sg.nz = a.g.nz;
  one.sg.inv_dx = a.g.inv_dx;
  one.sg.ox = a.g.ox;
  one.sg.oy = a.g.oy;
  one.sg.oz = a.g.oz;
  one.sg.dx = a.dx;
  for (int k = 0; k < 3; ++k) {
    one.sg.lo[k] = a.lo[k];
    one.sg.hi[k] = a.hi[k];
  }
  one.sg.node_off = 0;
  one.sg.region_off = 0;
  const unsigned blocks = (unsigned)((a.P + kSceneChunk - 1) / kSceneChunk);
  return launch_modes(a, one, n_modes, (int64_t)a.g.nx * a.g.ny * a.g.nz, blocks, stream);
}

hipError_t launch_g2p2g_batch(const G2P2GArgs& a, const SceneDev* table, int n_scenes,
                              int n_modes, hipStream_t stream) {
  // each scene in chunks of its own: at most one partial chunk per scene
  SceneChunks sc{table, n_scenes};
  const unsigned blocks = (unsigned)(a.P / kSceneChunk + n_scenes + 1);
  return launch_modes(a, sc, n_modes, a.gstride, blocks, stream);
}

}  // namespace polypic
