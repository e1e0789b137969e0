// PolyPIC transfers on a staggered (marker-and-cell) grid, for gfx950.
//
// The paper applies its transfers on MAC grids (section 3, Table 1): velocity
// component a lives on the faces at origin + (i + (1 - e_a) / 2) dx, each face with
// its own mass, momentum and velocity, and Eq. 1-8 and Eq. 13 hold per face.  Every
// component is thus a scalar transfer on its own lattice, shifted by half a spacing
// along the two other axes.  Along an axis a particle has two stencils: the node
// one (b = floor(u - 1/2), used by the component normal to that axis) and the
// shifted one (u' = u - 1/2, b' = floor(u' - 1/2) = b or b - 1, used by the two
// other components).  Their union spans 4 faces per axis, [b - 1, b + 2].
//
// P2G: one thread per sorted slot; lane pairs take consecutive slots (which usually
// share a cell) and the pairs of a wavefront are spread over the workgroup's chunk.
// Per distinct 4^3 tile of node bases (the cell-key sort makes them contiguous) a
// workgroup keeps an FP64 LDS brick of 7^3 faces x 6 channels (3 face masses, 3 face
// momenta), one face below the tile and two above.  A component's 27 face values per
// channel are added across a pair whose stencils of that component coincide (one DPP
// fold each), and one lane of the pair adds them to the brick with LDS atomics, one z
// plane at a time; the brick is flushed with one float atomic per non-zero face
// value.  Tiles past the brick budget add straight to HBM.
// G2P: one thread per output slot, gathering each component's 27 face velocities
// and projecting them with that component's rows (section 3.3), then advection and
// the F update, as on the collocated grid.
#include "polypic_bricks.hpp"
#include "polypic_internal.hpp"

namespace polypic {

namespace {

constexpr int kMacN = 7;                                       // brick edge in faces
constexpr int kMacNodes = kMacN * kMacN * kMacN;               // 343
constexpr int kMacSY = 7;                                      // y stride (doubles)
constexpr int kMacSZ = 49;                                     // z stride (doubles)
constexpr int kMacV = kMacNodes;                               // 343 doubles per channel:
                                                               // 36 KB of LDS, 4 groups per CU
constexpr int kMacCh = 6;                                      // m_x m_y m_z p_x p_y p_z
constexpr int kMacK = 2;                                       // bricks per workgroup
constexpr int kMacBS = 256;

// u = (x - o) inv_dx with two float32 roundings; the node stencil (b, t) and the
// stencil of the lattice shifted by +dx/2 (bs, ts); false if either leaves [0, n - 3].
__device__ __forceinline__ bool face_axes(float x, float o, float inv_dx, int n, int& b, float& t,
                                          int& bs, float& ts) {
  const float u = __fmul_rn(__fsub_rn(x, o), inv_dx);
  const float f = floorf(__fsub_rn(u, 0.5f));
  const float us = __fsub_rn(u, 0.5f);  // exact for u < 2^22
  const float fs = floorf(__fsub_rn(us, 0.5f));
  const bool ok = (f >= 0.0f) && (f <= (float)(n - 3)) && (fs >= 0.0f) && (fs <= (float)(n - 3));
  b = ok ? (int)f : 0;
  t = ok ? __fsub_rn(u, f + 1.0f) : 0.0f;
  bs = ok ? (int)fs : 0;
  ts = ok ? __fsub_rn(us, fs + 1.0f) : 0.0f;
  return ok;
}

template <int NR>
__global__ __launch_bounds__(kMacBS) void mac_p2g_kernel(MacP2GArgs a) {
  constexpr int BS = kMacBS;
  constexpr int NW = BS / kWave;
  __shared__ double brick[kMacK * kMacCh * kMacV];
  __shared__ BrickPlan<BS> plan;
  __shared__ uint64_t seg_tile[kMacK];

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int slot = pair_slot<NW>(tid);
  const int64_t i = (int64_t)blockIdx.x * BS + slot;
  const bool in = i < a.P;
  const size_t Ps = (size_t)a.P;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const size_t N = (size_t)nx * ny * nz;
  int p = 0;
  if (in) p = a.perm ? min(max(a.perm[i], 0), (int)(a.P - 1)) : (int)i;

  int b[3] = {0, 0, 0}, bs[3] = {0, 0, 0};
  float t[3] = {0.f, 0.f, 0.f}, ts[3] = {0.f, 0.f, 0.f};
  bool valid = in;
  if (in) {
    bool ok = face_axes(a.x[p], a.g.ox, a.g.inv_dx, nx, b[0], t[0], bs[0], ts[0]);
    ok &= face_axes(a.x[Ps + p], a.g.oy, a.g.inv_dx, ny, b[1], t[1], bs[1], ts[1]);
    ok &= face_axes(a.x[2 * Ps + p], a.g.oz, a.g.inv_dx, nz, b[2], t[2], bs[2], ts[2]);
    if (!ok) {
      raise_flag(a.status, kFlagRange);
      valid = false;
    }
  }
  const float m = valid ? (a.mass ? a.mass[p] : a.uniform_mass) : 0.0f;
  for (int n = tid; n < kMacNodes; n += BS) {
    const int lz = n / (kMacN * kMacN), ly = (n / kMacN) % kMacN, lx = n % kMacN;
    const int off = lx + kMacSY * ly + kMacSZ * lz;
#pragma unroll
    for (int k = 0; k < kMacK * kMacCh; ++k) brick[k * kMacV + off] = 0.0;
  }
  const int seg = plan_bricks<BS, kMacK>(plan, seg_tile, tid, slot,
                                         valid ? brick_tile_id(0, b[0], b[1], b[2]) : kNoTile);
  const bool lds = valid && seg >= 0 && seg < kMacK;
  // brick origin: one face below the tile of node bases, on every axis
  const int o0 = (b[0] & ~3) - 1, o1 = (b[1] & ~3) - 1, o2 = (b[2] & ~3) - 1;

  // Every lane runs the component loop (an idle one with zero mass and coefficients),
  // since the pair folds read the partner lane through DPP.
#pragma unroll 1
  for (int ax = 0; ax < 3; ++ax) {
    // component ax: node stencil along axis ax, shifted stencil along the others
    const int c0 = ax == 0 ? b[0] : bs[0], c1 = ax == 1 ? b[1] : bs[1],
              c2 = ax == 2 ? b[2] : bs[2];
    const Rows Rx = p2g_rows_scaled(basis_p2g(ax == 0 ? t[0] : ts[0]), m);
    const Rows Ry = p2g_rows_scaled(basis_p2g(ax == 1 ? t[1] : ts[1]), 1.0f);
    const Rows Rz = p2g_rows_scaled(basis_p2g(ax == 2 ? t[2] : ts[2]), 1.0f);
    float c[27];
#pragma unroll
    for (int r = 0; r < 27; ++r) c[r] = 0.0f;
    if (valid) {
      const float* cp = a.coeff + (size_t)ax * NR * Ps + p;
#pragma unroll
      for (int r = 0; r < NR; ++r) c[r] = cp[(size_t)r * Ps];
    }
    // a pair folds when both lanes' stencils of this component coincide
    const PairFold pf = pair_fold_plan(valid ? ((c2 * 1024 + c1) * 1024 + c0) : -1 - lane, seg,
                                       valid, lane);
    const int lbase = (c0 - o0) + kMacSY * (c1 - o1) + kMacSZ * (c2 - o2);
    const size_t gb = ((size_t)c2 * ny + c1) * nx + c0;
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
    auto emitter = [&](int ch) {
      double* const lbc = brick + ((lds ? seg : 0) * kMacCh + ch) * kMacV + lbase;
      float* const gc = (ch < 3 ? a.fm : a.fp) + (size_t)(ch % 3) * N + gb;
      return [=](int jz, float (&v)[9]) {
        float w[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) w[k] = pair_fold(v[k], pf.f);
        if (!pf.emit) return;
        if (lds) {
#pragma unroll
          for (int jy = 0; jy < 3; ++jy)
#pragma unroll
            for (int jx = 0; jx < 3; ++jx)
              atomicAdd(lbc + jx + kMacSY * jy + kMacSZ * jz, (double)w[jx + 3 * jy]);
        } else {
#pragma unroll
          for (int jy = 0; jy < 3; ++jy)
#pragma unroll
            for (int jx = 0; jx < 3; ++jx)
              atomicAdd(gc + jx + sy * jy + sz * jz, w[jx + 3 * jy]);
        }
      };
    };
    {  // face mass of this component: m W
      float one[27];
#pragma unroll
      for (int r = 0; r < 27; ++r) one[r] = r == 0 ? 1.0f : 0.0f;
      stream_modes_planes<1>(one, Rx, Ry, Rz, emitter(ax));
    }
    stream_modes_planes<NR>(c, Rx, Ry, Rz, emitter(3 + ax));
  }
  __syncthreads();

  // flush: thread t owns faces t, t + BS, ... of every brick
  const int nb = plan.n_bricks < kMacK ? plan.n_bricks : kMacK;
  for (int n = tid; n < kMacNodes; n += BS) {
    const int lz = n / (kMacN * kMacN), ly = (n / kMacN) % kMacN, lx = n % kMacN;
    const int off = lx + kMacSY * ly + kMacSZ * lz;
    for (int k = 0; k < nb; ++k) {
      int gx, gy, gz;
      brick_origin(seg_tile[k], 1, gx, gy, gz);
      gx += lx;
      gy += ly;
      gz += lz;
      if (gx < 0 || gy < 0 || gz < 0 || gx >= nx || gy >= ny || gz >= nz) continue;
      const size_t f = ((size_t)gz * ny + gy) * nx + gx;
#pragma unroll
      for (int ch = 0; ch < kMacCh; ++ch) {
        const double v = brick[(k * kMacCh + ch) * kMacV + off];
        if (v != 0.0) {
          float* dst = (ch < 3 ? a.fm : a.fp) + (size_t)(ch % 3) * N + f;
          atomicAdd(dst, (float)v);
        }
      }
    }
  }
}

// 512 threads: each output row is written in 2 KB runs per workgroup (the plain G2P's
// measured choice)
constexpr int kMacG2PBS = 512;

template <int NR>
__global__ __launch_bounds__(kMacG2PBS) void mac_g2p_kernel(MacG2PArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.P) return;
  const size_t Ps = (size_t)a.P;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const size_t N = (size_t)nx * ny * nz;
  const int p = a.perm ? min(max(a.perm[i], 0), (int)(a.P - 1)) : (int)i;
  const float xp[3] = {a.x_in[p], a.x_in[Ps + p], a.x_in[2 * Ps + p]};
  int b[3], bs[3];
  float t[3], ts[3];
  bool ok = face_axes(xp[0], a.g.ox, a.g.inv_dx, nx, b[0], t[0], bs[0], ts[0]);
  ok &= face_axes(xp[1], a.g.oy, a.g.inv_dx, ny, b[1], t[1], bs[1], ts[1]);
  ok &= face_axes(xp[2], a.g.oz, a.g.inv_dx, nz, b[2], t[2], bs[2], ts[2]);
  if (!ok) raise_flag(a.status, kFlagRange);
  float F[9];
  if (a.F_in) {
#pragma unroll
    for (int e = 0; e < 9; ++e) F[e] = a.F_in[(size_t)e * Ps + p];
  }
  float lin[3][3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    float c[27];
    if (ok) {
      const int c0 = ax == 0 ? b[0] : bs[0], c1 = ax == 1 ? b[1] : bs[1],
                c2 = ax == 2 ? b[2] : bs[2];
      const Proj1D px = proj_g2p(ax == 0 ? t[0] : ts[0]);
      const Proj1D py = proj_g2p(ax == 1 ? t[1] : ts[1]);
      const Proj1D pz = proj_g2p(ax == 2 ? t[2] : ts[2]);
      const float* vg = a.fv + (size_t)ax * N + ((size_t)c2 * ny + c1) * nx + c0;
      float v[27];
#pragma unroll
      for (int jz = 0; jz < 3; ++jz)
#pragma unroll
        for (int jy = 0; jy < 3; ++jy)
#pragma unroll
          for (int jx = 0; jx < 3; ++jx)
            v[jx + 3 * jy + 9 * jz] = vg[(size_t)jz * nx * ny + (size_t)jy * nx + jx];
      project_modes<NR>(v, px, py, pz, c);
    } else {
#pragma unroll
      for (int r = 0; r < 27; ++r) c[r] = 0.0f;
    }
    float* co = a.coeff_out + (size_t)ax * NR * Ps + i;
#pragma unroll
    for (int r = 0; r < NR; ++r) __builtin_nontemporal_store(c[r], co + (size_t)r * Ps);
    if (a.x_out) {
      float xn = fmaf(a.dt, c[0], xp[ax]);
      xn = fmaxf(xn, a.lo[ax]);
      xn = fminf(xn, a.hi[ax]);
      __builtin_nontemporal_store(xn, a.x_out + (size_t)ax * Ps + i);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) lin[ax][q] = (NR >= 4) ? c[1 + q] : 0.0f;
  }
  if (a.F_out) {
    const float s = a.dt / a.dx;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int col = 0; col < 3; ++col) {
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) acc = fmaf(lin[r][k], F[3 * k + col], acc);
        __builtin_nontemporal_store(fmaf(s, acc, F[3 * r + col]),
                                     a.F_out + (size_t)(3 * r + col) * Ps + i);
      }
  }
  if (a.mass_out) __builtin_nontemporal_store(a.mass_in[p], a.mass_out + i);
}

// Face velocities from face sums: per component, its own mass and walls normal to its axis.
__global__ __launch_bounds__(256) void mac_grid_update_kernel(MacUpdateArgs a) {
  uint32_t n32;
  int ix, iy, iz;
  if (!flat_node(a.nx, a.ny, a.nz, n32, ix, iy, iz)) return;
  const size_t N = (size_t)a.nx * a.ny * a.nz;
  const size_t n = n32;
  const int idx[3] = {ix, iy, iz};
  const int dims[3] = {a.nx, a.ny, a.nz};
  const float g[3] = {a.g0, a.g1, a.g2};
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const float m = a.fm[ax * N + n];
    float v = 0.0f;
    if (m > 0.0f) v = a.fp[ax * N + n] / m + a.dt * g[ax];
    if (a.bc_layers > 0) {
      if (idx[ax] <= 1 + a.bc_layers) v = fmaxf(v, 0.0f);
      if (idx[ax] >= dims[ax] - 1 - a.bc_layers) v = fminf(v, 0.0f);
    }
    a.fv[ax * N + n] = v;
  }
}

template <int NR>
hipError_t mac_p2g_nr(const MacP2GArgs& a, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.P + kMacBS - 1) / kMacBS);
  mac_p2g_kernel<NR><<<blocks, kMacBS, 0, s>>>(a);
  return hipGetLastError();
}

template <int NR>
hipError_t mac_g2p_nr(const MacG2PArgs& a, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.P + kMacG2PBS - 1) / kMacG2PBS);
  mac_g2p_kernel<NR><<<blocks, kMacG2PBS, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_mac_p2g(const MacP2GArgs& a, int n_modes, bool accumulate, hipStream_t s) {
  const int64_t N = (int64_t)a.g.nx * a.g.ny * a.g.nz;
  if (!accumulate) {
    hipError_t e = launch_zero(a.fm, 3 * N, s);
    if (e != hipSuccess) return e;
    if ((e = launch_zero(a.fp, 3 * N, s)) != hipSuccess) return e;
  }
  if (a.P == 0) return hipSuccess;
  switch (n_modes) {
    case 1: return mac_p2g_nr<1>(a, s);
    case 4: return mac_p2g_nr<4>(a, s);
    case 8: return mac_p2g_nr<8>(a, s);
    case 27: return mac_p2g_nr<27>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mac_grid_update(const MacUpdateArgs& a, hipStream_t s) {
  mac_grid_update_kernel<<<node_blocks(a.nx, a.ny, a.nz), 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_mac_g2p(const MacG2PArgs& a, int n_modes, hipStream_t s) {
  if (a.P == 0) return hipSuccess;
  switch (n_modes) {
    case 1: return mac_g2p_nr<1>(a, s);
    case 4: return mac_g2p_nr<4>(a, s);
    case 8: return mac_g2p_nr<8>(a, s);
    case 27: return mac_g2p_nr<27>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace polypic
