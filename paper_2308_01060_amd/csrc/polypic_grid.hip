// Grid update: v = (mv) / m (Eq. 5) where m > 0, plus gravity and separating
// slip walls, for gfx950.  One thread per node along x; y and z come from the
// block grid, so the wall tests need no division.
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
}

__global__ __launch_bounds__(256) void grid_update_kernel(GridUpdateArgs a) {
  const int ix = blockIdx.x * blockDim.x + threadIdx.x;
  const int iy = blockIdx.y;
  const int iz = blockIdx.z;
  if (ix >= a.nx) return;
  const size_t N = (size_t)a.nx * a.ny * a.nz;
  const size_t n = ((size_t)iz * a.ny + iy) * a.nx + ix;
  update_node(a, ix, iy, iz, a.nx, a.ny, a.nz, n, N);
}

// One row of workgroups per scene (blockIdx.y), striding over its nodes.
__global__ __launch_bounds__(256) void grid_update_batch_kernel(GridUpdateArgs a,
                                                                const SceneDev* __restrict__ t,
                                                                int64_t stride) {
  const SceneDev& d = t[blockIdx.y];
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const int64_t nn = (int64_t)nx * ny * nz;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nn; k += step) {
    const int64_t r = k / nx;
    const int ix = (int)(k - r * nx);
    const int iz = (int)(r / ny);
    const int iy = (int)(r - (int64_t)iz * ny);
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
  dim3 grid((unsigned)((a.nx + 255) / 256), (unsigned)a.ny, (unsigned)a.nz);
  grid_update_kernel<<<grid, 256, 0, stream>>>(a);
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
