// Liquid and fabric particles on one grid (section 3.4), for gfx950.
//
// One particle array holds both phases, tagged per particle (0 fluid, 1 solid).  Every
// grid node carries two sets of channels: the fluid mass and momentum of Eq. 15-16,
// scattered by the fluid particles with their mass m_f, and the solid mixture mass and
// momentum of Eq. 18-19, scattered by the solid particles with m_s + m_f (the fabric
// point and its absorbed fluid).  The velocity of each set is its momentum over its
// own grid-summed mass (Eq. 17, 20), and G2P fits each particle from its own phase.
//
// P2G: one thread per sorted slot; lane pairs take consecutive slots and the pairs of
// a wavefront are spread over the workgroup's chunk.  FP64 LDS bricks of 6^3 nodes x 8
// channels for the first two distinct 4^3 tiles of the chunk -- fluid and solid
// particles of a tile share its brick -- take the node values, added first across a
// pair with the same stencil and phase (one DPP fold each), one z plane at a time;
// one float atomic per non-zero brick value at the flush; other tiles add to HBM.
// The nodal values are the separable three-stage contraction of the plain P2G.
#include "polypic_bricks.hpp"
#include "polypic_internal.hpp"

namespace polypic {

namespace {

constexpr int kMixK = 2;
constexpr int kMixCh = 8;  // fluid m, p_x, p_y, p_z, then solid m, p_x, p_y, p_z
constexpr int kMixBS = 256;
// dense 6^3 bricks (27 KB of LDS for two bricks of 8 channels: 5 groups per CU)
constexpr int kMixSY = 6;
constexpr int kMixSZ = 36;
constexpr int kMixV = kBrickNodes;

template <int NR>
__global__ __launch_bounds__(kMixBS) void mixture_p2g_kernel(MixtureP2GArgs a) {
  constexpr int BS = kMixBS;
  constexpr int NW = BS / kWave;
  __shared__ double brick[kMixK * kMixCh * kMixV];
  __shared__ BrickPlan<BS> plan;
  __shared__ uint64_t seg_tile[kMixK];

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

  int b[3] = {0, 0, 0};
  float t[3] = {0.f, 0.f, 0.f};
  bool valid = in;
  int ph = 0;
  float m = 0.0f;
  if (in) {
    bool ok = stencil_axis(a.x[p], a.g.ox, a.g.inv_dx, nx, b[0], t[0]);
    ok &= stencil_axis(a.x[Ps + p], a.g.oy, a.g.inv_dx, ny, b[1], t[1]);
    ok &= stencil_axis(a.x[2 * Ps + p], a.g.oz, a.g.inv_dx, nz, b[2], t[2]);
    if (!ok) raise_flag(a.status, kFlagRange);
    ph = a.phase[p];
    const bool ph_ok = ph == 0 || ph == 1;
    if (!ph_ok) raise_flag(a.status, kFlagPhase);
    valid = ok && ph_ok;
    if (valid) m = a.mass_f[p] + (ph == 1 && a.mass_s ? a.mass_s[p] : 0.0f);
  }
  if (!valid) {
    ph = 0;
    b[0] = b[1] = b[2] = 0;
    t[0] = t[1] = t[2] = 0.0f;
  }

  for (int n = tid; n < kBrickNodes; n += BS) {
    const BrickNode bn = brick_node(n);
    const int off = bn.lx + kMixSY * bn.ly + kMixSZ * bn.lz;
#pragma unroll
    for (int k = 0; k < kMixK * kMixCh; ++k) brick[k * kMixV + off] = 0.0;
  }
  const int seg = plan_bricks<BS, kMixK>(plan, seg_tile, tid, slot,
                                         valid ? brick_tile_id(0, b[0], b[1], b[2]) : kNoTile);
  const bool lds = valid && seg >= 0 && seg < kMixK;
  // a pair folds when both lanes share stencil, brick and phase; every lane runs the
  // scatter below (an idle one with zero mass), since the folds read the partner lane
  const PairFold pf = pair_fold_plan(valid ? ((ph << 30) | ((b[2] * 1024 + b[1]) * 1024 + b[0]))
                                           : -1 - lane,
                                     seg, valid, lane);
  {
    const Rows Rx = p2g_rows_scaled(basis_p2g(t[0]), m);
    const Rows Ry = p2g_rows_scaled(basis_p2g(t[1]), 1.0f);
    const Rows Rz = p2g_rows_scaled(basis_p2g(t[2]), 1.0f);
    const int lbase = (b[0] & 3) + kMixSY * (b[1] & 3) + kMixSZ * (b[2] & 3);
    const size_t gbase = ((size_t)b[2] * ny + b[1]) * nx + b[0];
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
    // channel ch of this particle's phase: 0 mass, 1-3 momentum
    auto emitter = [&](int ch) {
      double* const lbc = brick + ((lds ? seg : 0) * kMixCh + 4 * ph + ch) * kMixV + lbase;
      float* const gc = ch == 0 ? a.gm + (size_t)ph * N + gbase
                                : a.gp + ((size_t)ph * 3 + (ch - 1)) * N + gbase;
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
              atomicAdd(lbc + jx + kMixSY * jy + kMixSZ * jz, (double)w[jx + 3 * jy]);
        } else {
#pragma unroll
          for (int jy = 0; jy < 3; ++jy)
#pragma unroll
            for (int jx = 0; jx < 3; ++jx)
              atomicAdd(gc + jx + sy * jy + sz * jz, w[jx + 3 * jy]);
        }
      };
    };
    {
      float one[27];
#pragma unroll
      for (int r = 0; r < 27; ++r) one[r] = r == 0 ? 1.0f : 0.0f;
      stream_modes_planes<1>(one, Rx, Ry, Rz, emitter(0));
    }
#pragma unroll 1
    for (int al = 0; al < 3; ++al) {
      float c[27];
#pragma unroll
      for (int r = 0; r < 27; ++r) c[r] = 0.0f;
      if (valid) {
#pragma unroll
        for (int r = 0; r < NR; ++r) c[r] = a.coeff[((size_t)al * NR + r) * Ps + p];
      }
      stream_modes_planes<NR>(c, Rx, Ry, Rz, emitter(1 + al));
    }
  }
  __syncthreads();

  const int nb = plan.n_bricks < kMixK ? plan.n_bricks : kMixK;
  for (int n = tid; n < kBrickNodes; n += BS) {
    const BrickNode bn = brick_node(n);
    const int off = bn.lx + kMixSY * bn.ly + kMixSZ * bn.lz;
    for (int k = 0; k < nb; ++k) {
      int o0, o1, o2;
      brick_origin(seg_tile[k], 0, o0, o1, o2);
      const int gx = o0 + bn.lx, gy = o1 + bn.ly, gz = o2 + bn.lz;
      if (gx >= nx || gy >= ny || gz >= nz) continue;
      const size_t f = ((size_t)gz * ny + gy) * nx + gx;
#pragma unroll
      for (int ch = 0; ch < kMixCh; ++ch) {
        const double v = brick[(k * kMixCh + ch) * kMixV + off];
        if (v == 0.0) continue;
        const int k4 = ch & 3, phase = ch >> 2;
        float* dst = k4 == 0 ? a.gm + (size_t)phase * N + f
                             : a.gp + ((size_t)phase * 3 + (k4 - 1)) * N + f;
        atomicAdd(dst, (float)v);
      }
    }
  }
}

// 512 threads: each output row is written in 2 KB runs per workgroup
constexpr int kMixG2PBS = 512;

template <int NR>
__global__ __launch_bounds__(kMixG2PBS) void mixture_g2p_kernel(MixtureG2PArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.P) return;
  const size_t Ps = (size_t)a.P;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const size_t N = (size_t)nx * ny * nz;
  const int p = a.perm ? min(max(a.perm[i], 0), (int)(a.P - 1)) : (int)i;
  const float xp[3] = {a.x_in[p], a.x_in[Ps + p], a.x_in[2 * Ps + p]};
  int b0, b1, b2;
  float t0, t1, t2;
  bool ok = stencil_axis(xp[0], a.g.ox, a.g.inv_dx, nx, b0, t0);
  ok &= stencil_axis(xp[1], a.g.oy, a.g.inv_dx, ny, b1, t1);
  ok &= stencil_axis(xp[2], a.g.oz, a.g.inv_dx, nz, b2, t2);
  if (!ok) raise_flag(a.status, kFlagRange);
  const int ph = a.phase_in[p];
  if (ph != 0 && ph != 1) {
    raise_flag(a.status, kFlagPhase);
    ok = false;
  }
  const Proj1D px = proj_g2p(t0), py = proj_g2p(t1), pz = proj_g2p(t2);
  const size_t gbase = ((size_t)b2 * ny + b1) * nx + b0;
  const float* const gv = a.gv + (size_t)(ok ? ph : 0) * 3 * N;
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
      const float* vg = gv + (size_t)ax * N + gbase;
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
  if (a.phase_out) a.phase_out[i] = ph;
  if (a.mass_f_out) a.mass_f_out[i] = a.mass_f_in[p];
  if (a.mass_s_out) a.mass_s_out[i] = a.mass_s_in[p];
}

template <int NR>
hipError_t mix_p2g_nr(const MixtureP2GArgs& a, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.P + kMixBS - 1) / kMixBS);
  mixture_p2g_kernel<NR><<<blocks, kMixBS, 0, s>>>(a);
  return hipGetLastError();
}

template <int NR>
hipError_t mix_g2p_nr(const MixtureG2PArgs& a, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.P + kMixG2PBS - 1) / kMixG2PBS);
  mixture_g2p_kernel<NR><<<blocks, kMixG2PBS, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_mixture_p2g(const MixtureP2GArgs& a, int n_modes, bool accumulate,
                              hipStream_t s) {
  if (!accumulate) {
    const int64_t N = (int64_t)a.g.nx * a.g.ny * a.g.nz;
    hipError_t e = launch_zero(a.gm, 2 * N, s);
    if (e != hipSuccess) return e;
    if ((e = launch_zero(a.gp, 6 * N, s)) != hipSuccess) return e;
  }
  if (a.P == 0) return hipSuccess;
  switch (n_modes) {
    case 1: return mix_p2g_nr<1>(a, s);
    case 4: return mix_p2g_nr<4>(a, s);
    case 8: return mix_p2g_nr<8>(a, s);
    case 27: return mix_p2g_nr<27>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mixture_g2p(const MixtureG2PArgs& a, int n_modes, hipStream_t s) {
  if (a.P == 0) return hipSuccess;
  switch (n_modes) {
    case 1: return mix_g2p_nr<1>(a, s);
    case 4: return mix_g2p_nr<4>(a, s);
    case 8: return mix_g2p_nr<8>(a, s);
    case 27: return mix_g2p_nr<27>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace polypic
