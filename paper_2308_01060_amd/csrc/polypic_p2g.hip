// P2G scatter (Eq. 1, 4 and 13) for gfx950.
//
// Per particle, in registers: the stencil, the quadratic B-spline weights and
// the 1-D mode factors of Eq. 11 / Eq. 14, then the nodal values
// sum_r c_r s_r at the 27 stencil nodes by a separable 3-stage contraction
// that skips the modes beyond n_modes at compile time.
//
// Two accumulation strategies:
//
// * Cell runs (sorted input: perm and sorted keys from polypic_sort).  One
//   workgroup per occupied tile of 4^3 cells (a Morton-aligned run of 64 cell
//   keys); each of its 4 wavefronts owns one channel (mass, 3 momentum
//   components) and walks the tile's particles in rounds of 64, one particle
//   per lane (coalesced loads).  Per round a wave writes its channel's 27
//   nodal values to a wave-private LDS buffer, finds the runs of equal cells
//   (particles of a cell are contiguous in sorted order and share one base
//   node) with ballots, sums each (run, stencil node) pair and adds it to an
//   FP64 brick of 6^3 nodes with one LDS double atomic -- eight times fewer
//   atomics than per particle, and mostly on distinct addresses, where
//   gfx950's LDS double atomics are fast (float ones are not: about 190
//   cycles per wavefront instruction).  The waves of a workgroup meet only at
//   the end of the tile, where the bricks go to HBM with one coalesced float
//   atomic per node and channel.
//
// * Brick scatter (any order; perm from polypic_sort makes it effective).  One
//   thread per particle, the lanes of a wavefront spread over the workgroup's
//   chunk of the processing order so that they fall in different cells; runs
//   of particles in the same tile (of 2^3, 4^3 or 8^3 cells, as configured)
//   accumulate into FP64 LDS bricks with LDS double atomics, and the bricks are
//   added to HBM with one float atomic per node and channel.  Runs beyond the
//   LDS budget (unsorted input) add straight to HBM.
#include "polypic_internal.hpp"

namespace polypic {

namespace {

// Brick geometry for tiles of T = 2^TL cells per axis: (T + 2)^3 nodes stored as FP64
// with strides (1, SY, SZ) doubles (V per channel, padding included), and K bricks per
// workgroup, so that the bricks take 29 to 37 KB of LDS at every edge.  The 4^3 tile is
// the one the fused kernel and the batched paths use; the autotuner may pick another.
template <int TL>
struct BrickGeom;
template <>
struct BrickGeom<1> {
  static constexpr int T = 2, N = 4, SY = 4, SZ = 20, K = 12;
};
template <>
struct BrickGeom<2> {
  static constexpr int T = kBrickT, N = kBrickN, SY = kBrickSY, SZ = kBrickSZ, K = kBrickKMAX;
};
template <>
struct BrickGeom<3> {
  static constexpr int T = 8, N = 10, SY = 10, SZ = 104, K = 1;
};

// Occupancy is bounded by LDS to 4 waves per SIMD (about 40 KB per 256-thread
// workgroup); the launch bound holds the registers to the 128 that allow it.
template <int NR, int BS, class Scenes, int TL>
__global__ __launch_bounds__(BS, BS == 256 ? 4 : 2) void p2g_brick_kernel(P2GArgs a, Scenes sc) {
  constexpr int NW = BS / kWave;
  using Geo = BrickGeom<TL>;
  constexpr int T = Geo::T, NB = Geo::N, SY = Geo::SY, SZ = Geo::SZ, K = Geo::K;
  constexpr int V = (NB - 1) * (1 + SY + SZ) + 1;  // doubles per channel of a brick
  constexpr int NB3 = NB * NB * NB;
  static_assert(SY >= NB && SZ >= SY * NB, "brick strides hold a brick");
  // LDS double atomics run at about 8 cycles per wavefront instruction on
  // gfx950 when their addresses avoid bank conflicts; float ones at about 190
  // whatever the addresses.
  __shared__ double brick[K * 4 * V];  // [brick][channel][node]
  __shared__ uint64_t tile_of[BS];     // by processing slot
  __shared__ int seg_of[BS];           // by processing slot
  __shared__ uint64_t seg_tile[K];
  __shared__ int wave_heads[NW];
  // grid of each brick's scene (batches only; one scene folds to constants)
  __shared__ int seg_dims[K][3];
  __shared__ int64_t seg_node_off[K];

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  // Slot of this thread's particle.  Lane groups of G (4 at 8 or more modes,
  // else 2) take G consecutive slots, which in sorted order (about 8 particles
  // per cell) usually share a cell, hence a base node: the group adds its nodal
  // values across lanes (DPP) and one lane does the atomic.  Groups of a
  // wavefront take every NW-th group of slots, so that they sit in different
  // cells and their brick atomics do not collide.
  constexpr int LG = NR >= 8 ? 2 : 1;  // log2 G
  const int slot = (((lane >> LG) * NW + wv) << LG) | (lane & ((1 << LG) - 1));
  const size_t Ps = (size_t)a.P;
  const int64_t n_chunks = (a.P + BS - 1) / BS;
  const ChunkRange cr = block_chunks(a.sched, n_chunks);
  // brick node q of the workgroup's bricks (q < K * NB3): its brick, and its offset in
  // a channel of that brick
  auto brick_of = [](int q) { return q / NB3; };
  auto node_lds = [](int q, int& lx, int& ly, int& lz) {
    const int n = q % NB3;
    lz = n / (NB * NB);
    ly = (n / NB) % NB;
    lx = n % NB;
    return lx + SY * ly + SZ * lz;
  };

  for (int64_t chunk = cr.begin; chunk < cr.end; ++chunk) {
    const int64_t i0 = chunk * BS;
    const int s0 = sc.first(i0);  // uniform over the workgroup
    const int64_t i = i0 + slot;
    bool valid = i < a.P;
    const int s = valid ? sc.of(i, s0) : s0;
    // one wave-uniform lookup unless the wavefront straddles a scene boundary
    SceneGrid sg = sc.grid(s0);
    if constexpr (Scenes::kMany) {
      if (__ballot(s != s0) != 0ull) sg = sc.grid(s);
    }
    int p = 0;
    // a caller permutation is clamped into [0, P) so that a bad one cannot read
    // out of bounds (results are then wrong, never a fault)
    if (valid) p = a.perm ? min(max(a.perm[i], 0), (int)(a.P - 1)) : (int)i;
    int b0 = 0, b1 = 0, b2 = 0;
    float t0 = 0.f, t1 = 0.f, t2 = 0.f;
    if (valid) {
      bool ok = stencil_axis(a.x[p], sg.ox, sg.inv_dx, sg.nx, b0, t0);
      ok &= stencil_axis(a.x[Ps + p], sg.oy, sg.inv_dx, sg.ny, b1, t1);
      ok &= stencil_axis(a.x[2 * Ps + p], sg.oz, sg.inv_dx, sg.nz, b2, t2);
      if (!ok) {
        raise_flag(a.status, kFlagRange);
        valid = false;
      }
    }
    // The first momentum component's coefficients are requested before the
    // workgroup barriers, so that their HBM latency overlaps the segment set-up
    // and the mass channel; later components are double-buffered (measured:
    // 0.49 -> 0.43 ms at 27 modes, 4.19 M particles).
    float cfa[27], cfb[27];
    {
      const float* cp = a.coeff + p;
#pragma unroll
      for (int r = 0; r < 27; ++r) cfa[r] = (r < NR) ? cp[(size_t)r * Ps] : 0.0f;
    }
    // tile of the base node: T^3-cell tile coordinates (10 bits per axis), plus the
    // scene relative to the chunk's first scene in the high word
    tile_of[slot] = valid ? (((uint64_t)(uint32_t)(s - s0) << 32) |
                             (uint64_t)((uint32_t)(b0 >> TL) | ((uint32_t)(b1 >> TL) << 10) |
                                        ((uint32_t)(b2 >> TL) << 20)))
                          : kNoTile;
    for (int q = tid; q < K * NB3; q += BS) {
      int lx, ly, lz;
      double* const dst = brick + brick_of(q) * 4 * V + node_lds(q, lx, ly, lz);
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) dst[ch * V] = 0.0;
    }
    __syncthreads();

    // runs of equal tiles in slot order (thread t looks at slot t) -> segments
    {
      const uint64_t tt = tile_of[tid];
      const bool head = tt != kNoTile && (tid == 0 || tile_of[tid - 1] != tt);
      const unsigned long long hb = __ballot(head);
      if (lane == 0) wave_heads[wv] = __popcll(hb);
      __syncthreads();
      int pre = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) pre += (w < wv) ? wave_heads[w] : 0;
      const int sgi = pre + lanes_below(hb) + (head ? 1 : 0) - 1;
      seg_of[tid] = sgi;
      if (head && sgi < K) {
        seg_tile[sgi] = tt;
        if constexpr (Scenes::kMany) {
          const SceneGrid fg = sc.grid(s0 + (int)(tt >> 32));
          seg_dims[sgi][0] = fg.nx;
          seg_dims[sgi][1] = fg.ny;
          seg_dims[sgi][2] = fg.nz;
          seg_node_off[sgi] = fg.node_off;
        }
      }
    }
    __syncthreads();
    int nseg = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) nseg += wave_heads[w];
    const int seg = seg_of[slot];

    // Lanes that share this lane's segment and base node: the pair (lane ^ 1)
    // and, with G = 4, the whole quad.  Every lane runs the evaluation below
    // (an invalid one with zero mass), since the DPP exchanges need them all.
    // (All exchanges run unconditionally: a DPP read from a lane that did not
    // execute it would return an undefined value.)
    const int mykey = valid ? ((b2 * 1024 + b1) * 1024 + b0) : -1 - lane;
    const int pair_key = pair_swap_i(mykey), pair_seg = pair_swap_i(seg);
    const bool pair = mykey == pair_key && seg == pair_seg;
    bool quad = false;
    if constexpr (LG == 2) {
      const int quad_pair = quad_swap_i((int)pair), quad_key = quad_swap_i(mykey);
      const int quad_seg = quad_swap_i(seg);
      quad = pair && quad_pair != 0 && mykey == quad_key && seg == quad_seg;
    }
    const bool emit = valid && (quad ? (lane & 3) == 0 : (!pair || (lane & 1) == 0));
    const float pair_f = pair ? 1.0f : 0.0f, quad_f = quad ? 1.0f : 0.0f;
    {
      const float m = valid ? (a.mass ? a.mass[p] : a.uniform_mass) : 0.0f;
      // rows s w_j phi_k(j) per axis; the particle mass rides on the x rows
      const Rows Rx = p2g_rows_scaled(basis_p2g(t0), m);
      const Rows Ry = p2g_rows_scaled(basis_p2g(t1), 1.0f);
      const Rows Rz = p2g_rows_scaled(basis_p2g(t2), 1.0f);
      const bool lds = seg < K;
      const int nx = sg.nx, ny = sg.ny;
      const int lbase = (b0 & (T - 1)) + SY * (b1 & (T - 1)) + SZ * (b2 & (T - 1));
      const int64_t gbase = sg.node_off + (int64_t)(b2 * ny + b1) * nx + b0;
      double* const lb = brick + (lds ? max(seg, 0) : 0) * 4 * V + lbase;
      float* const gch[4] = {a.gm + gbase, a.gp0 + gbase, a.gp1 + gbase, a.gp2 + gbase};
      const int nxny = nx * ny;
      // each nodal value goes straight to its brick (or, past the LDS budget, to HBM)
      auto emitter = [&](int ch) {
        double* const lbc = lb + ch * V;
        float* const gc = gch[ch];
        return [=](int jx, int jy, int jz, float v) {
          float w = pair_fold(v, pair_f);
          if constexpr (LG == 2) w = quad_fold(w, quad_f);
          if (!emit) return;
          if (lds)
            atomicAdd(lbc + jx + SY * jy + SZ * jz, (double)w);
          else
            atomicAdd(gc + jz * nxny + jy * nx + jx, w);
        };
      };
      {  // mass: m W_ip
        float one[27];
#pragma unroll
        for (int r = 0; r < 27; ++r) one[r] = r == 0 ? 1.0f : 0.0f;
        stream_modes<1>(one, Rx, Ry, Rz, emitter(0));
      }
      const float* cp = a.coeff + p;
#pragma unroll
      for (int r = 0; r < 27; ++r) cfb[r] = (r < NR) ? cp[(size_t)(NR + r) * Ps] : 0.0f;
      stream_modes<NR>(cfa, Rx, Ry, Rz, emitter(1));
#pragma unroll
      for (int r = 0; r < 27; ++r) cfa[r] = (r < NR) ? cp[(size_t)(2 * NR + r) * Ps] : 0.0f;
      stream_modes<NR>(cfb, Rx, Ry, Rz, emitter(2));
      stream_modes<NR>(cfa, Rx, Ry, Rz, emitter(3));
    }
    __syncthreads();

    // flush: one global float atomic per channel per non-zero brick node, the bricks'
    // nodes shared out over the threads
    const int nb = nseg < K ? nseg : K;
    for (int q = tid; q < nb * NB3; q += BS) {
      const int sb = brick_of(q);
      int lx, ly, lz;
      const int lo = node_lds(q, lx, ly, lz);
      const uint32_t tc = (uint32_t)seg_tile[sb];
      int fnx = sg.nx, fny = sg.ny, fnz = sg.nz;  // one scene: constants
      int64_t foff = sg.node_off;
      if constexpr (Scenes::kMany) {
        fnx = seg_dims[sb][0];
        fny = seg_dims[sb][1];
        fnz = seg_dims[sb][2];
        foff = seg_node_off[sb];
      }
      const int gx = (int)(tc & 1023u) * T + lx;
      const int gy = (int)((tc >> 10) & 1023u) * T + ly;
      const int gz = (int)(tc >> 20) * T + lz;
      if (gx >= fnx || gy >= fny || gz >= fnz) continue;
      const int64_t node = foff + ((int64_t)(gz * fny + gy) * fnx + gx);
      const double* const src = brick + sb * 4 * V + lo;
      float* const dst[4] = {a.gm, a.gp0, a.gp1, a.gp2};
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) {
        const float v = (float)src[ch * V];
        if (v != 0.0f) atomicAdd(dst[ch] + node, v);
      }
    }
    __syncthreads();  // the next chunk reuses tile_of, seg_tile and the bricks
  }
}

__global__ __launch_bounds__(256) void grid_clear_kernel(float* __restrict__ gm,
                                                         float* __restrict__ gp, int64_t n,
                                                         uint32_t* __restrict__ counter) {
  if (counter && blockIdx.x == 0 && threadIdx.x == 0) *counter = 0u;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    gm[k] = 0.0f;
    gp[k] = 0.0f;
    gp[n + k] = 0.0f;
    gp[2 * n + k] = 0.0f;
  }
}


__global__ __launch_bounds__(64) void zero_counter_kernel(uint32_t* __restrict__ counter) {
  if (threadIdx.x == 0) *counter = 0u;
}

// Start index (in sorted order) of every occupied 4^3-cell tile, appended in
// arbitrary order.  A tile is a run of 64 consecutive cell keys.
__global__ __launch_bounds__(256) void p2g_tiles_kernel(const uint32_t* __restrict__ keys,
                                                        int64_t P, uint32_t* __restrict__ list,
                                                        uint32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool head = i < P && (i == 0 || (keys[i - 1] >> 6) != (keys[i] >> 6));
  // one counter atomic per wavefront; heads take consecutive slots after it
  const unsigned long long hb = __ballot(head);
  if (hb == 0ull) return;
  const int leader = __builtin_ctzll(hb);
  const int lane = threadIdx.x & (kWave - 1);
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(hb));
  base = __shfl(base, leader, kWave);
  if (head) list[base + (uint32_t)lanes_below(hb)] = (uint32_t)i;
}

// local Morton index of a cell inside its 4^3 tile
__device__ __forceinline__ int morton_local4(int cx, int cy, int cz) {
  return (cx & 1) | ((cy & 1) << 1) | ((cz & 1) << 2) | ((cx >> 1) << 3) | ((cy >> 1) << 4) |
         ((cz >> 1) << 5);
}

constexpr int kCellT = 4;                         // tile edge in cells
constexpr int kCellC = kCellT * kCellT * kCellT;  // cells per tile
constexpr int kCellE = kCellT + 2;                // brick edge in nodes
constexpr int kCellBV = kCellE * kCellE * kCellE;
constexpr int kCellThreads = 4 * kWave;           // one wave per channel
constexpr int kRow = kWave + 1;                   // padded LDS row (conflict-free writes)

// Orders this wavefront's LDS accesses: LDS operations of one wave complete in
// issue order, so a compiler-level fence between writes and reads by other
// lanes of the same wave is all that is needed.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NR>
__global__ __launch_bounds__(kCellThreads) void p2g_cell_kernel(P2GArgs a) {
  __shared__ float buf[4][27 * kRow];      // per wave: one channel's nodal values of a round
  __shared__ double brick[4][kCellBV];     // per channel: the tile's 6^3 brick, FP64
  __shared__ int run_lo[4][kWave + 1];     // per wave: first lane of each run (+ end)
  __shared__ int run_cell[4][kWave];       // per wave: cell (local Morton index) of each run

  const int lane = threadIdx.x & (kWave - 1);
  const int ch = threadIdx.x / kWave;  // 0 mass, 1..3 momentum components
  float* const wbuf = buf[ch];
  double* const wbrick = brick[ch];
  const size_t Ps = (size_t)a.P;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const uint32_t ntiles = *a.tile_count;

  for (uint32_t w = blockIdx.x; w < ntiles; w += gridDim.x) {
    const int64_t ts = a.tile_list[w];
    const uint32_t key0 = a.keys[ts] & ~(uint32_t)(kCellC - 1);
    const uint32_t tkey = key0 >> 6;
    const int ox = (int)compact_bits3(key0);  // tile origin (base-node coordinates)
    const int oy = (int)compact_bits3(key0 >> 1);
    const int oz = (int)compact_bits3(key0 >> 2);
    for (int n = lane; n < kCellBV; n += kWave) wbrick[n] = 0.0;

    for (int64_t r0 = ts;; r0 += kWave) {
      const int64_t k = r0 + lane;
      const uint32_t kk = k < a.P ? a.keys[k] : 0xFFFFFFFFu;
      const bool inside = k < a.P && (kk >> 6) == tkey;  // a prefix of the wave
      const uint32_t kprev = (lane > 0 && k < a.P) ? a.keys[k - 1] : 0xFFFFFFFFu;
      const bool head = inside && (lane == 0 || kprev != kk);
      const unsigned long long hb = __ballot(head);
      const int n_runs = __popcll(hb);
      const int n_in = __popcll(__ballot(inside));
      const bool more = __ballot(lane == kWave - 1 && inside) != 0ull;
      if (head) {
        const int r = lanes_below(hb);
        run_lo[ch][r] = lane;
        run_cell[ch][r] = (int)(kk & (kCellC - 1));
      }
      if (lane == 0) run_lo[ch][n_runs] = n_in;

      bool valid = inside;
      int p = 0;
      int b0 = 0, b1 = 0, b2 = 0;
      float t0 = 0.f, t1 = 0.f, t2 = 0.f;
      if (valid) {
        p = a.perm ? min(max(a.perm[k], 0), (int)(a.P - 1)) : (int)k;
        bool ok = stencil_axis(a.x[p], a.g.ox, a.g.inv_dx, nx, b0, t0);
        ok &= stencil_axis(a.x[Ps + p], a.g.oy, a.g.inv_dx, ny, b1, t1);
        ok &= stencil_axis(a.x[2 * Ps + p], a.g.oz, a.g.inv_dx, nz, b2, t2);
        // the particle's base node must be the cell its key names
        const int cl = (int)(kk & (kCellC - 1));
        const int cx = (cl & 1) | (((cl >> 3) & 1) << 1);
        const int cy = ((cl >> 1) & 1) | (((cl >> 4) & 1) << 1);
        const int cz = ((cl >> 2) & 1) | (((cl >> 5) & 1) << 1);
        if (!ok || b0 != ox + cx || b1 != oy + cy || b2 != oz + cz) {
          if (ch == 0) raise_flag(a.status, kFlagRange);
          valid = false;
        }
      }
      const Basis1D bx = basis_p2g(t0);
      const Basis1D by = basis_p2g(t1);
      const Basis1D bz = basis_p2g(t2);
      const float m = valid ? (a.mass ? a.mass[p] : a.uniform_mass) : 0.0f;
      float wyz[9];
#pragma unroll
      for (int jz = 0; jz < 3; ++jz)
#pragma unroll
        for (int jy = 0; jy < 3; ++jy) wyz[jy + 3 * jz] = m * by.w[jy] * bz.w[jz];
      float val[27];
      if (ch == 0) {
#pragma unroll
        for (int jz = 0; jz < 3; ++jz)
#pragma unroll
          for (int jy = 0; jy < 3; ++jy)
#pragma unroll
            for (int jx = 0; jx < 3; ++jx) val[jx + 3 * jy + 9 * jz] = wyz[jy + 3 * jz] * bx.w[jx];
      } else {
        float cf[27];
        const float* cp = a.coeff + (size_t)(ch - 1) * NR * Ps + p;
#pragma unroll
        for (int r = 0; r < 27; ++r) cf[r] = (r < NR && valid) ? cp[(size_t)r * Ps] : 0.0f;
        float V[27];
        eval_modes<NR>(cf, bx, by, bz, V);
#pragma unroll
        for (int jz = 0; jz < 3; ++jz)
#pragma unroll
          for (int jy = 0; jy < 3; ++jy)
#pragma unroll
            for (int jx = 0; jx < 3; ++jx) {
              const int j = jx + 3 * jy + 9 * jz;
              val[j] = (wyz[jy + 3 * jz] * bx.w[jx]) * V[j];
            }
      }
#pragma unroll
      for (int j = 0; j < 27; ++j) wbuf[j * kRow + lane] = val[j];
      wave_lds_sync();

      // (run, stencil node) pairs: sum the run's lanes, add to the brick node
      for (int q = lane; q < n_runs * 27; q += kWave) {
        const int r = q / 27;
        const int j = q - r * 27;
        const int lo = run_lo[ch][r];
        const int hi = run_lo[ch][r + 1];
        const float* row = wbuf + j * kRow;
        float sum = 0.0f;
        for (int i0 = lo; i0 < hi; i0 += 8) {
#pragma unroll
          for (int d = 0; d < 8; ++d) {
            const int i = i0 + d;
            const float v = row[min(i, kWave - 1)];
            sum += (i < hi) ? v : 0.0f;
          }
        }
        const int cl = run_cell[ch][r];
        const int jz = j / 9, jy = (j / 3) % 3, jx = j % 3;
        const int lx = ((cl & 1) | (((cl >> 3) & 1) << 1)) + jx;
        const int ly = (((cl >> 1) & 1) | (((cl >> 4) & 1) << 1)) + jy;
        const int lz = (((cl >> 2) & 1) | (((cl >> 5) & 1) << 1)) + jz;
        atomicAdd(wbrick + (lz * kCellE + ly) * kCellE + lx, (double)sum);
      }
      wave_lds_sync();
      if (!more) break;
    }
    __syncthreads();

    // flush the four channel bricks with one global atomic per non-zero node
    float* const dst[4] = {a.gm, a.gp0, a.gp1, a.gp2};
    for (int q = threadIdx.x; q < 4 * kCellBV; q += kCellThreads) {
      const int chq = q / kCellBV;
      const int n = q - chq * kCellBV;
      const float v = (float)brick[chq][n];
      if (v != 0.0f) {
        const int lz = n / (kCellE * kCellE);
        const int ly = (n / kCellE) % kCellE;
        const int lx = n % kCellE;
        const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
        if (gx < nx && gy < ny && gz < nz) atomicAdd(dst[chq] + ((gz * ny + gy) * nx + gx), v);
      }
    }
    __syncthreads();  // the bricks are cleared by the next tile
  }
}

template <int NR, int BS, class Scenes>
hipError_t launch_cfg(const P2GArgs& a0, const Scenes& sc, const P2GConfig& c, hipStream_t stream) {
  P2GArgs a = a0;
  const int64_t chunks = (a.P + BS - 1) / BS;
  int64_t blocks = chunks;
  a.sched = c.sched;
  if (c.sched == kSchedPersistent) {
    const int64_t cap = (int64_t)c.persist_per_cu * kComputeUnits;
    if (cap < chunks) blocks = cap;
    else a.sched = kSchedXcd;  // as many workgroups as chunks: one chunk each
  }
  switch (c.tile_log2) {
    case 1: p2g_brick_kernel<NR, BS, Scenes, 1><<<(unsigned)blocks, BS, 0, stream>>>(a, sc); break;
    case 2: p2g_brick_kernel<NR, BS, Scenes, 2><<<(unsigned)blocks, BS, 0, stream>>>(a, sc); break;
    case 3: p2g_brick_kernel<NR, BS, Scenes, 3><<<(unsigned)blocks, BS, 0, stream>>>(a, sc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int NR, class Scenes>
hipError_t launch_nr(const P2GArgs& a, const Scenes& sc, const P2GConfig& c, hipStream_t stream) {
  switch (c.block) {
    case 256: return launch_cfg<NR, 256>(a, sc, c, stream);
    case 512: return launch_cfg<NR, 512>(a, sc, c, stream);
    default: return hipErrorInvalidValue;
  }
}

template <class Scenes>
hipError_t launch_modes(const P2GArgs& a, const Scenes& sc, int n_modes, const P2GConfig& cfg,
                        hipStream_t stream) {
  if (a.P == 0) return hipSuccess;
  switch (n_modes) {
    case 1: return launch_nr<1>(a, sc, cfg, stream);
    case 4: return launch_nr<4>(a, sc, cfg, stream);
    case 8: return launch_nr<8>(a, sc, cfg, stream);
    case 27: return launch_nr<27>(a, sc, cfg, stream);
    default: return hipErrorInvalidValue;
  }
}

template <int NR>
hipError_t launch_cell_nr(const P2GArgs& a, int blocks, hipStream_t stream) {
  p2g_cell_kernel<NR><<<blocks, kCellThreads, 0, stream>>>(a);
  return hipGetLastError();
}

}  // namespace

P2GConfig p2g_default_config() { return P2GConfig{2, 256, kSchedLinear, 0}; }

bool p2g_config_supported(const P2GConfig& c) {
  if (c.tile_log2 < 1 || c.tile_log2 > 3 || (c.block != 256 && c.block != 512)) return false;
  if (c.sched == kSchedLinear || c.sched == kSchedXcd) return true;
  return c.sched == kSchedPersistent && c.persist_per_cu >= 1 && c.persist_per_cu <= 64;
}

hipError_t launch_grid_clear(float* gm, float* gp, int64_t n_nodes, uint32_t* counter,
                             hipStream_t stream) {
  int64_t blocks = (n_nodes + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  grid_clear_kernel<<<(unsigned)blocks, 256, 0, stream>>>(gm, gp, n_nodes, counter);
  return hipGetLastError();
}

int64_t p2g_max_tiles(const GridDev& g, int64_t P) {
  // tiles are indexed by base node >> 2 per axis, base node in [0, n - 3]
  const int64_t t = (int64_t)(((g.nx - 3) >> 2) + 1) * (((g.ny - 3) >> 2) + 1) *
                    (((g.nz - 3) >> 2) + 1);
  return P < t ? P : t;
}

size_t p2g_workspace_bytes(const GridDev& g, int64_t P) {
  return align_up(sizeof(uint32_t)) + align_up((size_t)p2g_max_tiles(g, P) * sizeof(uint32_t));
}

hipError_t launch_p2g_sorted(const P2GArgs& a0, int n_modes, void* ws, bool counter_zeroed,
                             hipStream_t stream) {
  if (a0.P == 0) return hipSuccess;
  P2GArgs a = a0;
  uint32_t* count = (uint32_t*)ws;
  uint32_t* list = (uint32_t*)((char*)ws + align_up(sizeof(uint32_t)));
  a.tile_count = count;
  a.tile_list = list;
  if (!counter_zeroed) {
    zero_counter_kernel<<<1, 64, 0, stream>>>(count);
  }
  p2g_tiles_kernel<<<(unsigned)((a.P + 255) / 256), 256, 0, stream>>>(a.keys, a.P, list, count);
  // persistent grid over the occupied tiles (their number is only known on the device)
  int64_t blocks = p2g_max_tiles(a.g, a.P);
  if (blocks > 2048) blocks = 2048;
  switch (n_modes) {
    case 1: return launch_cell_nr<1>(a, (int)blocks, stream);
    case 4: return launch_cell_nr<4>(a, (int)blocks, stream);
    case 8: return launch_cell_nr<8>(a, (int)blocks, stream);
    case 27: return launch_cell_nr<27>(a, (int)blocks, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_p2g(const P2GArgs& a, int n_modes, const P2GConfig& cfg, hipStream_t stream) {
  OneScene one;
  one.sg.nx = a.g.nx;
  one.sg.ny = a.g.ny;
  one.sg.nz = a.g.nz;
  one.sg.inv_dx = a.g.inv_dx;
  one.sg.ox = a.g.ox;
  one.sg.oy = a.g.oy;
  one.sg.oz = a.g.oz;
  one.sg.dx = 0.0f;  // unused by P2G
  for (int k = 0; k < 3; ++k) one.sg.lo[k] = one.sg.hi[k] = 0.0f;
  one.sg.node_off = 0;
  return launch_modes(a, one, n_modes, cfg, stream);
}

hipError_t launch_p2g_batch(const P2GArgs& a, const SceneDev* table, int n_scenes, int n_modes,
                            const P2GConfig& cfg, hipStream_t stream) {
  SceneTable st{table, n_scenes};
  return launch_modes(a, st, n_modes, cfg, stream);
}

}  // namespace polypic
