// P2G scatter (Eq. 1, 4 and 13) for gfx950.
//
// One thread per particle, particles taken in the caller's processing order
// (a cell sort makes neighbours adjacent).  Per particle, in registers:
// the stencil, the quadratic B-spline weights and the 1-D mode factors of
// Eq. 11 / Eq. 14, then the nodal values sum_r c_r s_r at the 27 stencil nodes
// by a separable 3-stage contraction (z, then y, then x) that skips the
// modes beyond n_modes at compile time.
//
// Accumulation: the block's particles are split into runs that share a brick
// tile (an aligned cube of 2^tile_log2 cells, keyed by the base node).  Each
// run accumulates mass and momentum into an LDS brick of (T + 2)^3 nodes with
// LDS float atomics; a block-wide flush then adds every non-zero brick node to
// HBM with one global atomic per channel.  Runs beyond the LDS brick budget
// (unsorted input) add straight to HBM.
#include "polypic_internal.hpp"

namespace polypic {

namespace {

template <int NR>
__device__ constexpr bool any_kz(int kx, int ky) {
  return has_mode<NR>(kx, ky, 0) || has_mode<NR>(kx, ky, 1) || has_mode<NR>(kx, ky, 2);
}

template <int NR>
__device__ constexpr bool any_kykz(int kx) {
  return any_kz<NR>(kx, 0) || any_kz<NR>(kx, 1) || any_kz<NR>(kx, 2);
}

__device__ __forceinline__ float phi(const Basis1D& B, int k, int j) {
  return k == 0 ? 1.0f : (k == 1 ? B.z[j] : B.g[j]);
}

// V[jx + 3 jy + 9 jz] = sum_{r < NR} c[r] s_r(node j)
template <int NR>
__device__ __forceinline__ void eval_modes(const float (&c)[27], const Basis1D& bx,
                                           const Basis1D& by, const Basis1D& bz, float (&V)[27]) {
  float A[3][3][3];  // [kx][ky][jz]
#pragma unroll
  for (int kx = 0; kx < 3; ++kx)
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
      if (!any_kz<NR>(kx, ky)) continue;
#pragma unroll
      for (int jz = 0; jz < 3; ++jz) {
        float s = 0.0f;
        bool first = true;
#pragma unroll
        for (int kz = 0; kz < 3; ++kz) {
          if (!has_mode<NR>(kx, ky, kz)) continue;
          const float term = c[mode_index(kx, ky, kz)];
          s = first ? (kz == 0 ? term : term * phi(bz, kz, jz))
                    : (kz == 0 ? s + term : fmaf(term, phi(bz, kz, jz), s));
          first = false;
        }
        A[kx][ky][jz] = s;
      }
    }
  float Bm[3][3][3];  // [kx][jy][jz]
#pragma unroll
  for (int kx = 0; kx < 3; ++kx) {
    if (!any_kykz<NR>(kx)) continue;
#pragma unroll
    for (int jy = 0; jy < 3; ++jy)
#pragma unroll
      for (int jz = 0; jz < 3; ++jz) {
        float s = 0.0f;
        bool first = true;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
          if (!any_kz<NR>(kx, ky)) continue;
          const float term = A[kx][ky][jz];
          s = first ? (ky == 0 ? term : term * phi(by, ky, jy))
                    : (ky == 0 ? s + term : fmaf(term, phi(by, ky, jy), s));
          first = false;
        }
        Bm[kx][jy][jz] = s;
      }
  }
#pragma unroll
  for (int jx = 0; jx < 3; ++jx)
#pragma unroll
    for (int jy = 0; jy < 3; ++jy)
#pragma unroll
      for (int jz = 0; jz < 3; ++jz) {
        float s = 0.0f;
        bool first = true;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
          if (!any_kykz<NR>(kx)) continue;
          const float term = Bm[kx][jy][jz];
          s = first ? (kx == 0 ? term : term * phi(bx, kx, jx))
                    : (kx == 0 ? s + term : fmaf(term, phi(bx, kx, jx), s));
          first = false;
        }
        V[jx + 3 * jy + 9 * jz] = s;
      }
}

template <int TB>
constexpr int kmax_for() {
  return TB == 1 ? 16 : (TB == 2 ? 6 : 2);
}

template <int NR, int TB, int BS>
__global__ __launch_bounds__(BS) void p2g_kernel(P2GArgs a) {
  constexpr int T = 1 << TB;
  constexpr int E = T + 2;          // brick edge in nodes
  constexpr int BV = E * E * E;     // brick volume in nodes
  constexpr int KMAX = kmax_for<TB>();
  constexpr int NW = BS / kWave;
  __shared__ float brick[4 * KMAX * BV];  // [channel][brick][node]
  __shared__ uint32_t tile_of[BS];
  __shared__ uint32_t seg_tile[KMAX];
  __shared__ int wave_heads[NW];

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  const int64_t i = (int64_t)blockIdx.x * BS + tid;
  const size_t Ps = (size_t)a.P;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;

  bool valid = i < a.P;
  int p = 0;
  // a caller permutation is clamped into [0, P) so that a bad one cannot read
  // out of bounds (results are then wrong, never a fault)
  if (valid) p = a.perm ? min(max(a.perm[i], 0), (int)(a.P - 1)) : (int)i;
  int b0 = 0, b1 = 0, b2 = 0;
  float t0 = 0.f, t1 = 0.f, t2 = 0.f;
  if (valid) {
    bool ok = stencil_axis(a.x[p], a.g.ox, a.g.inv_dx, nx, b0, t0);
    ok &= stencil_axis(a.x[Ps + p], a.g.oy, a.g.inv_dx, ny, b1, t1);
    ok &= stencil_axis(a.x[2 * Ps + p], a.g.oz, a.g.inv_dx, nz, b2, t2);
    if (!ok) {
      raise_flag(a.status, kFlagRange);
      valid = false;
    }
  }
  const uint32_t tile = valid ? ((uint32_t)(b0 >> TB) | ((uint32_t)(b1 >> TB) << 10) |
                                 ((uint32_t)(b2 >> TB) << 20))
                              : 0xFFFFFFFFu;
  tile_of[tid] = tile;
  for (int k = tid; k < 4 * KMAX * BV; k += BS) brick[k] = 0.0f;
  __syncthreads();

  // runs of equal tiles in processing order -> segment index per particle
  const bool head = valid && (tid == 0 || tile_of[tid - 1] != tile);
  const unsigned long long hb = __ballot(head);
  if (lane == 0) wave_heads[wv] = __popcll(hb);
  __syncthreads();
  int pre = 0, nseg = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int h = wave_heads[w];
    pre += (w < wv) ? h : 0;
    nseg += h;
  }
  const int seg = pre + lanes_below(hb) + (head ? 1 : 0) - 1;
  if (head && seg < KMAX) seg_tile[seg] = tile;
  __syncthreads();

  if (valid) {
    const Basis1D bx = basis_p2g(t0);
    const Basis1D by = basis_p2g(t1);
    const Basis1D bz = basis_p2g(t2);
    const float m = a.mass ? a.mass[p] : a.uniform_mass;
    const bool lds = seg < KMAX;
    const int lbase = lds ? ((((b2 & (T - 1)) * E) + (b1 & (T - 1))) * E + (b0 & (T - 1))) : 0;
    float* lb = brick + (lds ? seg : 0) * BV + lbase;
    const int nxny = nx * ny;
    const int gbase = (b2 * ny + b1) * nx + b0;
    float* gch[4] = {a.gm + gbase, a.gp0 + gbase, a.gp1 + gbase, a.gp2 + gbase};

    float wyz[9];
#pragma unroll
    for (int jz = 0; jz < 3; ++jz)
#pragma unroll
      for (int jy = 0; jy < 3; ++jy) wyz[jy + 3 * jz] = m * by.w[jy] * bz.w[jz];

    // mass channel (Eq. 1, 4)
#pragma unroll
    for (int jz = 0; jz < 3; ++jz)
#pragma unroll
      for (int jy = 0; jy < 3; ++jy)
#pragma unroll
        for (int jx = 0; jx < 3; ++jx) {
          const float val = wyz[jy + 3 * jz] * bx.w[jx];
          if (lds)
            atomicAdd(lb + (jz * E + jy) * E + jx, val);
          else
            atomicAdd(gch[0] + jz * nxny + jy * nx + jx, val);
        }

    // momentum channels (Eq. 13)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      float c[27];
      const float* cp = a.coeff + (size_t)ax * NR * Ps + p;
#pragma unroll
      for (int r = 0; r < 27; ++r) c[r] = (r < NR) ? cp[(size_t)r * Ps] : 0.0f;
      float V[27];
      eval_modes<NR>(c, bx, by, bz, V);
      float* lbc = lb + (1 + ax) * KMAX * BV;
#pragma unroll
      for (int jz = 0; jz < 3; ++jz)
#pragma unroll
        for (int jy = 0; jy < 3; ++jy)
#pragma unroll
          for (int jx = 0; jx < 3; ++jx) {
            const float val = wyz[jy + 3 * jz] * bx.w[jx] * V[jx + 3 * jy + 9 * jz];
            if (lds)
              atomicAdd(lbc + (jz * E + jy) * E + jx, val);
            else
              atomicAdd(gch[1 + ax] + jz * nxny + jy * nx + jx, val);
          }
    }
  }
  __syncthreads();

  // flush the bricks: one global atomic per channel per non-zero node
  const int nb = nseg < KMAX ? nseg : KMAX;
  for (int k = tid; k < nb * BV; k += BS) {
    const int s = k / BV;
    const int loc = k - s * BV;
    const float vm = brick[(0 * KMAX + s) * BV + loc];
    const float v0 = brick[(1 * KMAX + s) * BV + loc];
    const float v1 = brick[(2 * KMAX + s) * BV + loc];
    const float v2 = brick[(3 * KMAX + s) * BV + loc];
    if (vm != 0.0f || v0 != 0.0f || v1 != 0.0f || v2 != 0.0f) {
      const uint32_t tl = seg_tile[s];
      const int lz = loc / (E * E);
      const int rem = loc - lz * E * E;
      const int ly = rem / E;
      const int lx = rem - ly * E;
      const int gx = (int)(tl & 1023u) * T + lx;
      const int gy = (int)((tl >> 10) & 1023u) * T + ly;
      const int gz = (int)(tl >> 20) * T + lz;
      if (gx < nx && gy < ny && gz < nz) {
        const int node = (gz * ny + gy) * nx + gx;
        atomicAdd(a.gm + node, vm);
        atomicAdd(a.gp0 + node, v0);
        atomicAdd(a.gp1 + node, v1);
        atomicAdd(a.gp2 + node, v2);
      }
    }
  }
}

__global__ __launch_bounds__(256) void grid_clear_kernel(float* __restrict__ gm,
                                                         float* __restrict__ gp, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    gm[k] = 0.0f;
    gp[k] = 0.0f;
    gp[n + k] = 0.0f;
    gp[2 * n + k] = 0.0f;
  }
}

template <int NR, int TB, int BS>
hipError_t launch_cfg(const P2GArgs& a, hipStream_t stream) {
  const unsigned blocks = (unsigned)((a.P + BS - 1) / BS);
  p2g_kernel<NR, TB, BS><<<blocks, BS, 0, stream>>>(a);
  return hipGetLastError();
}

template <int NR>
hipError_t launch_nr(const P2GArgs& a, const P2GConfig& c, hipStream_t stream) {
  switch (c.tile_log2 * 1000 + c.block) {
    case 1128: return launch_cfg<NR, 1, 128>(a, stream);
    case 1256: return launch_cfg<NR, 1, 256>(a, stream);
    case 2128: return launch_cfg<NR, 2, 128>(a, stream);
    case 2256: return launch_cfg<NR, 2, 256>(a, stream);
    case 2512: return launch_cfg<NR, 2, 512>(a, stream);
    case 3256: return launch_cfg<NR, 3, 256>(a, stream);
    case 3512: return launch_cfg<NR, 3, 512>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

P2GConfig p2g_default_config() { return P2GConfig{2, 256}; }

bool p2g_config_supported(const P2GConfig& c) {
  const int code = c.tile_log2 * 1000 + c.block;
  return code == 1128 || code == 1256 || code == 2128 || code == 2256 || code == 2512 ||
         code == 3256 || code == 3512;
}

hipError_t launch_grid_clear(float* gm, float* gp, int64_t n_nodes, hipStream_t stream) {
  if (n_nodes == 0) return hipSuccess;
  int64_t blocks = (n_nodes + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  grid_clear_kernel<<<(unsigned)blocks, 256, 0, stream>>>(gm, gp, n_nodes);
  return hipGetLastError();
}

hipError_t launch_p2g(const P2GArgs& a, int n_modes, const P2GConfig& cfg, hipStream_t stream) {
  if (a.P == 0) return hipSuccess;
  switch (n_modes) {
    case 1: return launch_nr<1>(a, cfg, stream);
    case 4: return launch_nr<4>(a, cfg, stream);
    case 8: return launch_nr<8>(a, cfg, stream);
    case 27: return launch_nr<27>(a, cfg, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace polypic
