// Grid update: v = (mv) / m (Eq. 5) where m > 0, plus gravity and separating
// slip walls, for gfx950.  One thread per node of a flat launch (x fastest), so
// every wavefront streams 64 consecutive nodes whatever the row length.  Optionally the pass also zeroes
// the mass and momentum it has read, so that the next step's scatter can
// accumulate into them without a separate clear.
#include "polypic_internal.hpp"

namespace polypic {

namespace {

// Node n of a grid with nx x ny x nz nodes at (ix, iy, iz); channels N apart.
__device__ __forceinline__ void update_node(const GridUpdateArgs& a, int ix, int iy, int iz,
                                            int nx, int ny, int nz, size_t n, size_t N) {
  const float m = a.gm[n];
  float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f;
  if (m > 0.0f) {
    v0 = a.gp[n] / m + a.dt * a.g0;
    v1 = a.gp[N + n] / m + a.dt * a.g1;
    v2 = a.gp[2 * N + n] / m + a.dt * a.g2;
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
