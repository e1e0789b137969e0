// P2G with the affine back-map of Eq. 12, for gfx950.
//
// A particle's coefficients were fitted at its previous position x_fit, in the basis
// orthogonalised there; Eq. 12 maps the present configuration back to that one, so the
// modes of Eq. 13 are evaluated at
//     z'_i = B (x_i - x_p) / dx,   B = (I + dt C)^-1,   C_ab = c_{a, 1+b} / dx,
// with the quadratic factor of Eq. 14 of the fitting position,
//     ghat(z) = z^2 - a z - 1/4,   a = t_fit (1 - 4 t_fit^2),
// and the weights of the present position.  z' mixes the three axes, so the node
// values no longer factor into three 1-D contractions: per node and component the
// 27 modes cost 27 + 9 + 3 multiply-adds on the per-axis factors (1, z', ghat(z')),
// against 3 x 81 per component for the whole separable stencil of the plain P2G.
//
// Scatter: one thread per sorted slot, lane pairs on consecutive slots and the pairs
// of a wavefront spread over the chunk; a pair with the same stencil adds its node
// values across lanes (one DPP fold each), and one lane adds them, one z plane at a
// time, to FP64 LDS bricks of 6^3 nodes x 4 channels for the first three distinct 4^3
// tiles of the chunk; one float atomic per non-zero brick value at the flush; other
// tiles add straight to HBM.
#include "polypic_bricks.hpp"
#include "polypic_internal.hpp"

namespace polypic {

namespace {

constexpr int kAffK = 3;
constexpr int kAffBS = 256;

template <int NR>
__global__ __launch_bounds__(kAffBS) void affine_p2g_kernel(AffineP2GArgs a) {
  constexpr int BS = kAffBS;
  constexpr int NW = BS / kWave;
  __shared__ double brick[kAffK * 4 * kBrickV];
  __shared__ BrickPlan<BS> plan;
  __shared__ uint64_t seg_tile[kAffK];

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  const int slot = pair_slot<NW>(tid);
  const int64_t i = (int64_t)blockIdx.x * BS + slot;
  const bool in = i < a.P;
  const size_t Ps = (size_t)a.P;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  int p = 0;
  if (in) p = a.perm ? min(max(a.perm[i], 0), (int)(a.P - 1)) : (int)i;

  int b[3] = {0, 0, 0};
  float t[3] = {0.f, 0.f, 0.f};
  float afit[3] = {0.f, 0.f, 0.f};
  bool valid = in;
  if (in) {
    bool ok = stencil_axis(a.x[p], a.g.ox, a.g.inv_dx, nx, b[0], t[0]);
    ok &= stencil_axis(a.x[Ps + p], a.g.oy, a.g.inv_dx, ny, b[1], t[1]);
    ok &= stencil_axis(a.x[2 * Ps + p], a.g.oz, a.g.inv_dx, nz, b[2], t[2]);
    if (!ok) {
      raise_flag(a.status, kFlagRange);
      valid = false;
    }
    float tf[3] = {t[0], t[1], t[2]};
    if (valid && a.x_fit) {
      int bf;
      bool okf = stencil_axis(a.x_fit[p], a.g.ox, a.g.inv_dx, nx, bf, tf[0]);
      okf &= stencil_axis(a.x_fit[Ps + p], a.g.oy, a.g.inv_dx, ny, bf, tf[1]);
      okf &= stencil_axis(a.x_fit[2 * Ps + p], a.g.oz, a.g.inv_dx, nz, bf, tf[2]);
      if (!okf) {
        raise_flag(a.status, kFlagRange);
        valid = false;
      }
    }
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) afit[ax] = tf[ax] * (1.0f - 4.0f * tf[ax] * tf[ax]);
  }
  // B = (I + dt C)^-1 from the linear coefficients (identity below 4 modes)
  float B[3][3] = {{1.f, 0.f, 0.f}, {0.f, 1.f, 0.f}, {0.f, 0.f, 1.f}};
  if (NR >= 4 && valid) {
    const float s = a.dt * a.g.inv_dx;
    float A[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        A[r][q] = (r == q ? 1.0f : 0.0f) + s * a.coeff[((size_t)r * NR + 1 + q) * Ps + p];
    const float c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    const float c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
    const float c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    const float det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
    if (!(fabsf(det) > 1e-20f) || !isfinite(det)) {
      raise_flag(a.status, kFlagMap);
      valid = false;
    } else {
      const float inv = 1.0f / det;
      B[0][0] = c00 * inv;
      B[1][0] = c01 * inv;
      B[2][0] = c02 * inv;
      B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * inv;
      B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * inv;
      B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * inv;
      B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * inv;
      B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * inv;
      B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * inv;
    }
  }
  const float m = valid ? (a.mass ? a.mass[p] : a.uniform_mass) : 0.0f;

  for (int n = tid; n < kBrickNodes; n += BS) {
    const int off = brick_node(n).lds;
#pragma unroll
    for (int k = 0; k < kAffK * 4; ++k) brick[k * kBrickV + off] = 0.0;
  }
  const int seg = plan_bricks<BS, kAffK>(plan, seg_tile, tid, slot,
                                         valid ? brick_tile_id(0, b[0], b[1], b[2]) : kNoTile);
  const bool lds = valid && seg >= 0 && seg < kAffK;
  // a pair folds when both lanes share stencil and brick; every lane runs the scatter
  // below (an idle one with zero mass and coefficients), since the folds read the
  // partner lane through DPP
  const PairFold pf = pair_fold_plan(valid ? ((b[2] * 1024 + b[1]) * 1024 + b[0]) : -1 - lane,
                                     seg, valid, lane);
  {
    const Basis1D bx = basis_p2g(t[0]), by = basis_p2g(t[1]), bz = basis_p2g(t[2]);
    const int lbase = (b[0] & 3) + kBrickSY * (b[1] & 3) + kBrickSZ * (b[2] & 3);
    const size_t N = (size_t)nx * ny * nz;
    const size_t gbase = ((size_t)b[2] * ny + b[1]) * nx + b[0];
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
    // fold a plane of node values over the pair and add it to channel ch
    auto emit_plane = [&](int ch, int jz, float (&v)[9]) {
      float w[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) w[k] = pair_fold(v[k], pf.f);
      if (!pf.emit) return;
      if (lds) {
        double* const bb = brick + ((lds ? seg : 0) * 4 + ch) * kBrickV + lbase + kBrickSZ * jz;
#pragma unroll
        for (int jy = 0; jy < 3; ++jy)
#pragma unroll
          for (int jx = 0; jx < 3; ++jx)
            atomicAdd(bb + jx + kBrickSY * jy, (double)w[jx + 3 * jy]);
      } else {
        float* const gc = (ch == 0 ? a.gm : a.gp + (size_t)(ch - 1) * N) + gbase + sz * jz;
#pragma unroll
        for (int jy = 0; jy < 3; ++jy)
#pragma unroll
          for (int jx = 0; jx < 3; ++jx) atomicAdd(gc + jx + sy * jy, w[jx + 3 * jy]);
      }
    };
#pragma unroll 1
    for (int al = 0; al < 3; ++al) {
      float c[27];
#pragma unroll
      for (int r = 0; r < 27; ++r) c[r] = 0.0f;
      if (valid) {
#pragma unroll
        for (int r = 0; r < NR; ++r) c[r] = a.coeff[((size_t)al * NR + r) * Ps + p];
      }
      // one z plane at a time keeps the node values' temporaries few (not unrolled)
#pragma unroll 1
      for (int jz = 0; jz < 3; ++jz) {
        const float zz = jz == 0 ? bz.z[0] : (jz == 1 ? bz.z[1] : bz.z[2]);
        const float wz = jz == 0 ? bz.w[0] : (jz == 1 ? bz.w[1] : bz.w[2]);
        float wv[9], vv[9];
#pragma unroll
        for (int jy = 0; jy < 3; ++jy)
#pragma unroll
          for (int jx = 0; jx < 3; ++jx) {
            const float zh[3] = {bx.z[jx], by.z[jy], zz};
            float phi[3][3];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
              const float zp = fmaf(B[ax][2], zh[2], fmaf(B[ax][1], zh[1], B[ax][0] * zh[0]));
              phi[ax][0] = 1.0f;
              phi[ax][1] = zp;
              phi[ax][2] = fmaf(zp, zp - afit[ax], -0.25f);
            }
            float V = 0.0f;
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
              if (!any_kykz<NR>(kx)) continue;
              float sxy = 0.0f;
#pragma unroll
              for (int ky = 0; ky < 3; ++ky) {
                if (!any_kz<NR>(kx, ky)) continue;
                float s_z = 0.0f;
#pragma unroll
                for (int kz = 0; kz < 3; ++kz)
                  if (has_mode<NR>(kx, ky, kz))
                    s_z = kz == 0 ? s_z + c[mode_index(kx, ky, kz)]
                                  : fmaf(c[mode_index(kx, ky, kz)], phi[2][kz], s_z);
                sxy = ky == 0 ? sxy + s_z : fmaf(s_z, phi[1][ky], sxy);
              }
              V = kx == 0 ? V + sxy : fmaf(sxy, phi[0][kx], V);
            }
            const float W = m * bx.w[jx] * by.w[jy] * wz;
            wv[jx + 3 * jy] = W;
            vv[jx + 3 * jy] = W * V;
          }
        if (al == 0) emit_plane(0, jz, wv);
        emit_plane(1 + al, jz, vv);
      }
    }
  }
  __syncthreads();

  const int nb = plan.n_bricks < kAffK ? plan.n_bricks : kAffK;
  const size_t N = (size_t)nx * ny * nz;
  for (int n = tid; n < kBrickNodes; n += BS) {
    const BrickNode bn = brick_node(n);
    for (int k = 0; k < nb; ++k) {
      int o0, o1, o2;
      brick_origin(seg_tile[k], 0, o0, o1, o2);
      const int gx = o0 + bn.lx, gy = o1 + bn.ly, gz = o2 + bn.lz;
      if (gx >= nx || gy >= ny || gz >= nz) continue;
      const size_t f = ((size_t)gz * ny + gy) * nx + gx;
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) {
        const double v = brick[(k * 4 + ch) * kBrickV + bn.lds];
        if (v != 0.0) atomicAdd(ch == 0 ? a.gm + f : a.gp + (size_t)(ch - 1) * N + f, (float)v);
      }
    }
  }
}

template <int NR>
hipError_t affine_nr(const AffineP2GArgs& a, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.P + kAffBS - 1) / kAffBS);
  affine_p2g_kernel<NR><<<blocks, kAffBS, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_p2g_affine(const AffineP2GArgs& a, int n_modes, bool accumulate,
                             hipStream_t s) {
  if (!accumulate) {
    const int64_t N = (int64_t)a.g.nx * a.g.ny * a.g.nz;
    hipError_t e = launch_zero(a.gm, N, s);
    if (e != hipSuccess) return e;
    if ((e = launch_zero(a.gp, 3 * N, s)) != hipSuccess) return e;
  }
  if (a.P == 0) return hipSuccess;
  switch (n_modes) {
    case 1: return affine_nr<1>(a, s);
    case 4: return affine_nr<4>(a, s);
    case 8: return affine_nr<8>(a, s);
    case 27: return affine_nr<27>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace polypic
