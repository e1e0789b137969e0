// Grid update: v = (mv) / m (Eq. 5) where m > 0, plus gravity and separating
// slip walls, for gfx950.  One thread per node of a flat launch (x fastest), so
// every wavefront streams 64 consecutive nodes whatever the row length.
// Optionally the pass also zeroes the mass and momentum it has read, so that the
// next step's scatter can accumulate into them without a separate clear; and the
// active form visits only the regions of nodes a scatter has flagged.
#include "polypic_internal.hpp"

namespace polypic {

namespace {

// The update of node n, at (ix, iy, iz) of an nx x ny x nz grid (channels N apart),
// from its mass m and momentum (p0, p1, p2), already read.
__device__ __forceinline__ void update_node_values(const GridUpdateArgs& a, int ix, int iy,
                                                   int iz, int nx, int ny, int nz, size_t n,
                                                   size_t N, float m, float p0, float p1,
                                                   float p2) {
  // v = fl(fl(p / m) + fl(dt g)) in every pass that updates nodes: no multiply-add
  // contraction, which the compiler would otherwise choose per kernel
#pragma clang fp contract(off)
  float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f;
  if (m > 0.0f) {
    v0 = p0 / m + a.dt * a.g0;
    v1 = p1 / m + a.dt * a.g1;
    v2 = p2 / m + a.dt * a.g2;
  }
  if (a.bc_layers > 0) {
    const int L = a.bc_layers;
    if (ix <= 1 + L) v0 = fmaxf(v0, 0.0f);
    if (ix >= nx - 1 - L) v0 = fminf(v0, 0.0f);
    if (iy <= 1 + L) v1 = fmaxf(v1, 0.0f);
    if (iy >= ny - 1 - L) v1 = fminf(v1, 0.0f);
    if (iz <= 1 + L) v2 = fmaxf(v2, 0.0f);
    if (iz >= nz - 1 - L) v2 = fminf(v2, 0.0f);
  }
  a.gv[n] = v0;
  a.gv[N + n] = v1;
  a.gv[2 * N + n] = v2;
  if (a.clear_gm) {  // the sums are consumed: leave them zero for the next accumulation
    a.clear_gm[n] = 0.0f;
    a.clear_gp[n] = 0.0f;
    a.clear_gp[N + n] = 0.0f;
    a.clear_gp[2 * N + n] = 0.0f;
  }
}

// The same, reading the node's mass and momentum.
__device__ __forceinline__ void update_node(const GridUpdateArgs& a, int ix, int iy, int iz,
                                            int nx, int ny, int nz, size_t n, size_t N) {
  const float m = a.gm[n];
  float p0 = 0.0f, p1 = 0.0f, p2 = 0.0f;
  if (m > 0.0f) {
    p0 = a.gp[n];
    p1 = a.gp[N + n];
    p2 = a.gp[2 * N + n];
  }
  update_node_values(a, ix, iy, iz, nx, ny, nz, n, N, m, p0, p1, p2);
}

__global__ __launch_bounds__(256) void grid_update_kernel(GridUpdateArgs a) {
  uint32_t n;
  int ix, iy, iz;
  if (!flat_node(a.nx, a.ny, a.nz, n, ix, iy, iz)) return;
  const size_t N = (size_t)a.nx * a.ny * a.nz;
  update_node(a, ix, iy, iz, a.nx, a.ny, a.nz, n, N);
}

// One row of workgroups per scene (blockIdx.y), striding over its nodes.
__global__ __launch_bounds__(256) void grid_update_batch_kernel(GridUpdateArgs a,
                                                                const SceneDev* __restrict__ t,
                                                                int64_t stride) {
  const SceneDev& d = t[blockIdx.y];
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  // a scene grid has at most 1026^3 nodes: 32-bit node indices and divisions
  const uint32_t nn = (uint32_t)nx * (uint32_t)ny * (uint32_t)nz;
  const uint32_t step = gridDim.x * blockDim.x;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < nn; k += step) {
    const uint32_t r = k / (uint32_t)nx;
    const int ix = (int)(k - r * (uint32_t)nx);
    const int iz = (int)(r / (uint32_t)ny);
    const int iy = (int)(r - (uint32_t)iz * (uint32_t)ny);
    update_node(a, ix, iy, iz, nx, ny, nz, (size_t)(d.node_off + k), (size_t)stride);
  }
}

// The flagged regions (16 x 4 x 4 nodes, one per thread).  Workgroup w reads the
// flags w, w + G, w + 2G, ... (G workgroups; 256 at a time, one per thread), so that
// every workgroup samples the whole grid and the flagged regions, which cluster where
// the particles are, spread evenly over the workgroups.  It resets the set flags it
// finds and gathers them in LDS (a flag holds 1 + the region's scene), then updates and
// clears those regions kGroup at a time, every load of a group issued before the first
// store, so that the memory latency of one region overlaps the others'.
constexpr int kGroup = 4;

template <bool kBatch>
__global__ __launch_bounds__(256) void grid_update_flagged_kernel(GridUpdateArgs a,
                                                                  const SceneDev* __restrict__ t,
                                                                  int n_scenes, int64_t stride) {
  static_assert(kRegX * kRegY * kRegZ == 256, "one node per thread");
  __shared__ uint32_t todo[256];
  __shared__ uint32_t todo_scene[256];
  __shared__ int wave_count[256 / kWave];
  uint32_t* const flags = a.regions;
  const int64_t R = a.n_regions;
  const int64_t G = gridDim.x;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int lx = tid % kRegX, ly = (tid / kRegX) % kRegY, lz = tid / (kRegX * kRegY);
  for (int64_t base = blockIdx.x; base < R; base += G * 256) {
    const int64_t q = base + (int64_t)tid * G;
    uint32_t f = 0u;
    if (q < R) {
      f = flags[q];
      if (f != 0u) flags[q] = 0u;
    }
    const bool set = f != 0u;
    const unsigned long long bal = __ballot(set);
    if (lane == 0) wave_count[wv] = __popcll(bal);
    __syncthreads();
    int pre = 0, n_todo = 0;
#pragma unroll
    for (int w = 0; w < 256 / kWave; ++w) {
      pre += (w < wv) ? wave_count[w] : 0;
      n_todo += wave_count[w];
    }
    if (set) {
      todo[pre + lanes_below(bal)] = (uint32_t)q;
      todo_scene[pre + lanes_below(bal)] = f - 1u;
    }
    __syncthreads();
    for (int j0 = 0; j0 < n_todo; j0 += kGroup) {
      // this thread's node in each region of the group, and its mass and momentum
      int ix[kGroup], iy[kGroup], iz[kGroup], nxs[kGroup], nys[kGroup], nzs[kGroup];
      size_t node[kGroup], Ns[kGroup];
      bool live[kGroup];
      float m[kGroup], p0[kGroup], p1[kGroup], p2[kGroup];
#pragma unroll
      for (int u = 0; u < kGroup; ++u) {
        live[u] = false;
        m[u] = p0[u] = p1[u] = p2[u] = 0.0f;
        if (j0 + u >= n_todo) continue;
        const int64_t r_id = todo[j0 + u];
        int nx = a.nx, ny = a.ny, nz = a.nz;
        int64_t node_off = 0, q_local = r_id;
        size_t N = (size_t)nx * ny * nz;
        if constexpr (kBatch) {
          const int sc = (int)min(todo_scene[j0 + u], (uint32_t)(n_scenes - 1));
          const SceneDev& d = t[sc];
          nx = d.nx;
          ny = d.ny;
          nz = d.nz;
          node_off = d.node_off;
          q_local = r_id - d.region_begin;
          N = (size_t)stride;
        }
        const int rx = regions_along(nx, kRegX), ry = regions_along(ny, kRegY);
        const int64_t rr = q_local / rx;
        ix[u] = (int)(q_local % rx) * kRegX + lx;
        iy[u] = (int)(rr % ry) * kRegY + ly;
        iz[u] = (int)(rr / ry) * kRegZ + lz;
        nxs[u] = nx;
        nys[u] = ny;
        nzs[u] = nz;
        Ns[u] = N;
        live[u] = q_local >= 0 && ix[u] < nx && iy[u] < ny && iz[u] < nz;
        node[u] = (size_t)(node_off + ((int64_t)iz[u] * ny + iy[u]) * nx + ix[u]);
        if (live[u]) {
          m[u] = a.gm[node[u]];
          p0[u] = a.gp[node[u]];
          p1[u] = a.gp[Ns[u] + node[u]];
          p2[u] = a.gp[2 * Ns[u] + node[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < kGroup; ++u)
        if (live[u])
          update_node_values(a, ix[u], iy[u], iz[u], nxs[u], nys[u], nzs[u], node[u], Ns[u],
                             m[u], p0[u], p1[u], p2[u]);
    }
    __syncthreads();  // todo and wave_count are rewritten by the next round
  }
}

// workgroups of the flagged update: enough to fill the chip, no more than regions
unsigned flagged_blocks(int64_t n_regions) {
  const int64_t most = 8 * (int64_t)kComputeUnits;
  return (unsigned)(n_regions < most ? (n_regions < 1 ? 1 : n_regions) : most);
}

__global__ __launch_bounds__(256) void zero_kernel(float* __restrict__ p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = 0.0f;
}

}  // namespace

hipError_t launch_zero(float* p, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  zero_kernel<<<(unsigned)blocks, 256, 0, stream>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_grid_update(const GridUpdateArgs& a, hipStream_t stream) {
  grid_update_kernel<<<node_blocks(a.nx, a.ny, a.nz), 256, 0, stream>>>(a);
  return hipGetLastError();
}

hipError_t launch_grid_update_active(const GridUpdateArgs& a, hipStream_t stream) {
  grid_update_flagged_kernel<false><<<flagged_blocks(a.n_regions), 256, 0, stream>>>(
      a, nullptr, 0, 0);
  return hipGetLastError();
}

hipError_t launch_grid_update_active_batch(const GridUpdateArgs& a, const SceneDev* table,
                                           int n_scenes, int64_t stride, hipStream_t stream) {
  grid_update_flagged_kernel<true><<<flagged_blocks(a.n_regions), 256, 0, stream>>>(
      a, table, n_scenes, stride);
  return hipGetLastError();
}

hipError_t launch_grid_update_batch(const GridUpdateArgs& a, const SceneDev* table, int n_scenes,
                                    int max_nodes, int64_t stride, hipStream_t stream) {
  if (n_scenes <= 0) return hipSuccess;
  int64_t bx = ((int64_t)max_nodes + 255) / 256;
  if (bx > 1024) bx = 1024;
  if (bx < 1) bx = 1;
  dim3 grid((unsigned)bx, (unsigned)n_scenes, 1);
  grid_update_batch_kernel<<<grid, 256, 0, stream>>>(a, table, stride);
  return hipGetLastError();
}

}  // namespace polypic
