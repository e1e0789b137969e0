// Hand-written adjoint of one transfer step, for gfx950.
//
// Forward (per particle p, normalised units, t = u - b - 1 per axis):
//   P2G      M_i = sum_p m_p W_ip,   Q_ai = sum_p m_p W_ip V_pa(i),
//            V_pa(i) = sum_r c_par s_r(i)           (Eq. 1, 4, 13)
//   update   v_ai = Q_ai / M_i + dt g_a  (M_i > 0), then the wall clamps (Eq. 5)
//   G2P      c'_par = sum_i P_r(i) v_ai             (section 3.3 projection)
//   advect   x'_pa = clamp(x_pa + dt c'_pa0)
// Reverse, given dL/dc' and dL/dx':
//   advect   passes dL/dx' to x and dt dL/dx' to c'_0 where the clamp is inactive
//   G2P      v_bar_ai  += sum_p sum_r P_r(i) c'_bar_par           (scatter)
//            x_bar_pb  += inv_dx sum_a sum_r c'_bar_par sum_i dP_r(i)/dt_b v_ai
//   update   Q_bar = v_bar / M,  M_bar = -sum_a v_bar_a Q_a / M^2 on unclamped
//            components of occupied nodes
//   P2G      c_bar_par  = m_p sum_i R_r(i) Q_bar_ai,  R_r = W s_r   (gather)
//            x_bar_pb  += inv_dx m_p [sum_i dW/dt_b M_bar_i
//                                     + sum_a sum_r c_par sum_i dR_r(i)/dt_b Q_bar_ai]
//            m_bar_p    = sum_i W M_bar_i + sum_a sum_r c_par (c_bar_par / m_p)
// Every row product is separable, so each sum over the 27 nodes is a 3-stage
// contraction with 1-D rows (and their t-derivatives) in registers.
#include "polypic_internal.hpp"

namespace polypic {

namespace {

// ---------------------------------------------------------------- grid update
__global__ __launch_bounds__(256) void grid_update_backward_kernel(GridUpdateBackArgs a) {
  uint32_t n32;
  int ix, iy, iz;
  if (!flat_node(a.nx, a.ny, a.nz, n32, ix, iy, iz)) return;
  const size_t N = (size_t)a.nx * a.ny * a.nz;
  const size_t n = n32;
  const float m = a.gm[n];
  float mb = 0.0f, pb0 = 0.0f, pb1 = 0.0f, pb2 = 0.0f;
  if (m > 0.0f) {
    const float p[3] = {a.gp[n], a.gp[N + n], a.gp[2 * N + n]};
    const float g[3] = {a.g0, a.g1, a.g2};
    const int idx[3] = {ix, iy, iz};
    const int dims[3] = {a.nx, a.ny, a.nz};
    float pb[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      // the forward's rounding: fl(fl(p / m) + fl(dt g)), not contracted
      const float v = __fadd_rn(p[ax] / m, __fmul_rn(a.dt, g[ax]));
      bool pass = true;  // derivative of the wall clamp
      if (a.bc_layers > 0) {
        if (idx[ax] <= 1 + a.bc_layers && v < 0.0f) pass = false;
        if (idx[ax] >= dims[ax] - 1 - a.bc_layers && v > 0.0f) pass = false;
      }
      const float vb = pass ? a.gvb[(size_t)ax * N + n] : 0.0f;
      pb[ax] = vb / m;
      mb -= pb[ax] * (p[ax] / m);
    }
    pb0 = pb[0];
    pb1 = pb[1];
    pb2 = pb[2];
  }
  a.gmb[n] = mb;
  a.gpb[n] = pb0;
  a.gpb[N + n] = pb1;
  a.gpb[2 * N + n] = pb2;
}

// ---------------------------------------------------------------- P2G adjoint (gather)
template <int NR>
__global__ __launch_bounds__(256) void p2g_backward_kernel(P2GBackArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.P) return;
  const size_t Ps = (size_t)a.P;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int p = a.perm ? min(max(a.perm[i], 0), (int)(a.P - 1)) : (int)i;
  int b0, b1, b2;
  float t0, t1, t2;
  bool ok = stencil_axis(a.x[p], a.g.ox, a.g.inv_dx, nx, b0, t0);
  ok &= stencil_axis(a.x[Ps + p], a.g.oy, a.g.inv_dx, ny, b1, t1);
  ok &= stencil_axis(a.x[2 * Ps + p], a.g.oz, a.g.inv_dx, nz, b2, t2);
  if (!ok) {
    // skipped in the forward pass: no gradient
    raise_flag(a.status, kFlagRange);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int r = 0; r < NR; ++r) a.coeff_grad[((size_t)ax * NR + r) * Ps + p] = 0.0f;
    if (a.mass_grad) a.mass_grad[p] = 0.0f;
    return;
  }
  Rows R[3], dR[3];
  p2g_rows(t0, R[0], dR[0]);
  p2g_rows(t1, R[1], dR[1]);
  p2g_rows(t2, R[2], dR[2]);
  const float m = a.mass ? a.mass[p] : a.uniform_mass;
  const size_t N = (size_t)nx * ny * nz;
  const int nxny = nx * ny;
  const int gbase = (b2 * ny + b1) * nx + b0;

  float xg[3] = {0.0f, 0.0f, 0.0f};
  float mg = 0.0f;
  {
    float v[27];
#pragma unroll
    for (int jz = 0; jz < 3; ++jz)
#pragma unroll
      for (int jy = 0; jy < 3; ++jy)
#pragma unroll
        for (int jx = 0; jx < 3; ++jx)
          v[jx + 3 * jy + 9 * jz] = a.gmb[gbase + jz * nxny + jy * nx + jx];
    float o[27];
    contract_rows<1>(v, R[0], R[1], R[2], o);
    mg += o[0];
    contract_rows<1>(v, dR[0], R[1], R[2], o);
    xg[0] += m * o[0];
    contract_rows<1>(v, R[0], dR[1], R[2], o);
    xg[1] += m * o[0];
    contract_rows<1>(v, R[0], R[1], dR[2], o);
    xg[2] += m * o[0];
  }
  // Per momentum component: T_r = sum_i R_r(i) pb_i gives dL/dc_r = m T_r, and the
  // same contraction with the t-derivative row on axis b gives dT_r/dt_b, whose
  // sum over r weighted by c_r is the x gradient.  The four contractions share
  // their stages (x, then y, then z), one kx plane at a time, so no 27-wide
  // output array is held.
#pragma unroll 1
  for (int ax = 0; ax < 3; ++ax) {
    float v[27];
    const float* q = a.gpb + (size_t)ax * N + gbase;
#pragma unroll
    for (int jz = 0; jz < 3; ++jz)
#pragma unroll
      for (int jy = 0; jy < 3; ++jy)
#pragma unroll
        for (int jx = 0; jx < 3; ++jx) v[jx + 3 * jy + 9 * jz] = q[jz * nxny + jy * nx + jx];
    const float* cp = a.coeff + (size_t)ax * NR * Ps + p;
    float* cg = a.coeff_grad + (size_t)ax * NR * Ps + p;
    // all coefficients first: the compiler cannot move a load of coeff past a
    // store to coeff_grad (they might alias), so loads inside the mode loop
    // would each wait out their full latency.  Both streams are read or written
    // once, so they bypass the caches the grid gathers use (measured, 27 modes,
    // 4.19 M particles: 0.556 -> 0.510 ms)
    float c[27];
#pragma unroll
    for (int r = 0; r < 27; ++r)
      c[r] = (r < NR) ? __builtin_nontemporal_load(cp + (size_t)r * Ps) : 0.0f;
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
    for (int kx = 0; kx < 3; ++kx) {
      if (!any_kykz<NR>(kx)) continue;
      float A[3][3], Ad[3][3];  // [jy][jz]: x contracted with R, with dR
#pragma unroll
      for (int jy = 0; jy < 3; ++jy)
#pragma unroll
        for (int jz = 0; jz < 3; ++jz) {
          const float* vv = v + 3 * jy + 9 * jz;
          A[jy][jz] = fmaf(R[0].r[kx][2], vv[2], fmaf(R[0].r[kx][1], vv[1], R[0].r[kx][0] * vv[0]));
          Ad[jy][jz] =
              fmaf(dR[0].r[kx][2], vv[2], fmaf(dR[0].r[kx][1], vv[1], dR[0].r[kx][0] * vv[0]));
        }
#pragma unroll
      for (int ky = 0; ky < 3; ++ky) {
        if (!any_kz<NR>(kx, ky)) continue;
        float B[3], By[3], Bx[3];  // [jz]
#pragma unroll
        for (int jz = 0; jz < 3; ++jz) {
          B[jz] = fmaf(R[1].r[ky][2], A[2][jz], fmaf(R[1].r[ky][1], A[1][jz], R[1].r[ky][0] * A[0][jz]));
          By[jz] =
              fmaf(dR[1].r[ky][2], A[2][jz], fmaf(dR[1].r[ky][1], A[1][jz], dR[1].r[ky][0] * A[0][jz]));
          Bx[jz] =
              fmaf(R[1].r[ky][2], Ad[2][jz], fmaf(R[1].r[ky][1], Ad[1][jz], R[1].r[ky][0] * Ad[0][jz]));
        }
#pragma unroll
        for (int kz = 0; kz < 3; ++kz) {
          if (!has_mode<NR>(kx, ky, kz)) continue;
          const int r = mode_index(kx, ky, kz);
          const float cr = c[r];
          const float T = fmaf(R[2].r[kz][2], B[2], fmaf(R[2].r[kz][1], B[1], R[2].r[kz][0] * B[0]));
          const float Tz =
              fmaf(dR[2].r[kz][2], B[2], fmaf(dR[2].r[kz][1], B[1], dR[2].r[kz][0] * B[0]));
          const float Ty =
              fmaf(R[2].r[kz][2], By[2], fmaf(R[2].r[kz][1], By[1], R[2].r[kz][0] * By[0]));
          const float Tx =
              fmaf(R[2].r[kz][2], Bx[2], fmaf(R[2].r[kz][1], Bx[1], R[2].r[kz][0] * Bx[0]));
          __builtin_nontemporal_store(m * T, cg + (size_t)r * Ps);
          mg = fmaf(cr, T, mg);
          sx = fmaf(cr, Tx, sx);
          sy = fmaf(cr, Ty, sy);
          sz = fmaf(cr, Tz, sz);
        }
      }
    }
    xg[0] = fmaf(m, sx, xg[0]);
    xg[1] = fmaf(m, sy, xg[1]);
    xg[2] = fmaf(m, sz, xg[2]);
  }
  const float inv_dx = a.g.inv_dx;
  a.x_grad[p] += inv_dx * xg[0];
  a.x_grad[Ps + p] += inv_dx * xg[1];
  a.x_grad[2 * Ps + p] += inv_dx * xg[2];
  if (a.mass_grad) a.mass_grad[p] = mg;
}

// ---------------------------------------------------------------- G2P adjoint
// Scatter of v_bar into FP64 LDS bricks (the brick P2G scheme: lane groups of
// consecutive slots, which usually share a cell, add their node values across
// lanes first; the groups of a wavefront are spread over the workgroup's chunk
// so that their atomics fall in different cells) plus a gather of the grid
// velocity for x_bar.
constexpr int kBackKMAX = 3;

template <int NR, int BS>
__global__ __launch_bounds__(BS) void g2p_backward_kernel(G2PBackArgs a) {
  constexpr int NW = BS / kWave;
  constexpr int LG = NR >= 8 ? 2 : 1;  // log2 of the lane-group size
  __shared__ double brick[kBackKMAX * 3 * kBrickV];  // [brick][component][node]
  __shared__ uint32_t tile_of[BS];
  __shared__ int seg_of[BS];
  __shared__ uint32_t seg_tile[kBackKMAX];
  __shared__ int wave_heads[NW];

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  const int slot = (((lane >> LG) * NW + wv) << LG) | (lane & ((1 << LG) - 1));
  const int64_t i0 = (int64_t)blockIdx.x * BS;
  const int64_t i = i0 + slot;
  const int row_n = (int)min((int64_t)BS, a.P - i0);  // slots of this workgroup
  const int slot_off = slot * (int)sizeof(float);
  const size_t Ps = (size_t)a.P;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const size_t N = (size_t)nx * ny * nz;
  static_assert(kBrickNodes <= BS, "one brick node per thread");
  const BrickNode bn = brick_node(tid);

  bool valid = i < a.P;
  int p = 0;
  if (valid) p = a.perm ? min(max(a.perm[i], 0), (int)(a.P - 1)) : (int)i;
  int b0 = 0, b1 = 0, b2 = 0;
  float t0 = 0.f, t1 = 0.f, t2 = 0.f;
  float xp[3] = {0.f, 0.f, 0.f};
  if (valid) {
    xp[0] = a.x_in[p];
    xp[1] = a.x_in[Ps + p];
    xp[2] = a.x_in[2 * Ps + p];
    bool ok = stencil_axis(xp[0], a.g.ox, a.g.inv_dx, nx, b0, t0);
    ok &= stencil_axis(xp[1], a.g.oy, a.g.inv_dx, ny, b1, t1);
    ok &= stencil_axis(xp[2], a.g.oz, a.g.inv_dx, nz, b2, t2);
    if (!ok) {
      raise_flag(a.status, kFlagRange);
      valid = false;
      b0 = b1 = b2 = 0;  // (stencil_axis leaves 0 on its own failing axis only)
      t0 = t1 = t2 = 0.f;
    }
  }
  tile_of[slot] = valid ? ((uint32_t)(b0 >> 2) | ((uint32_t)(b1 >> 2) << 10) |
                           ((uint32_t)(b2 >> 2) << 20))
                        : 0xFFFFFFFFu;
  if (tid < kBrickNodes) {
#pragma unroll
    for (int k = 0; k < kBackKMAX * 3; ++k) brick[k * kBrickV + bn.lds] = 0.0;
  }
  __syncthreads();
  {
    const uint32_t tt = tile_of[tid];
    const bool head = tt != 0xFFFFFFFFu && (tid == 0 || tile_of[tid - 1] != tt);
    const unsigned long long hb = __ballot(head);
    if (lane == 0) wave_heads[wv] = __popcll(hb);
    __syncthreads();
    int pre = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) pre += (w < wv) ? wave_heads[w] : 0;
    const int sg = pre + lanes_below(hb) + (head ? 1 : 0) - 1;
    seg_of[tid] = sg;
    if (head && sg < kBackKMAX) seg_tile[sg] = tt;
  }
  __syncthreads();
  int nseg = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) nseg += wave_heads[w];
  const int seg = seg_of[slot];

  // Lanes that share this lane's segment and base node: the pair (lane ^ 1)
  // and, with groups of 4, the quad.  Every lane runs the node loop below (an
  // invalid one with base node 0 and zero gradients), since the DPP folds read
  // their partners.
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
    Rows Pr[3], dP[3];
    g2p_rows(t0, Pr[0], dP[0]);
    g2p_rows(t1, Pr[1], dP[1]);
    g2p_rows(t2, Pr[2], dP[2]);
    const bool lds = seg < kBackKMAX;
    const int lbase = (b0 & 3) + kBrickSY * (b1 & 3) + kBrickSZ * (b2 & 3);
    const int nxny = nx * ny;
    const int gbase = (b2 * ny + b1) * nx + b0;
    double* const lb = brick + (lds ? max(seg, 0) : 0) * 3 * kBrickV + lbase;
    float xg[3] = {0.f, 0.f, 0.f};
#pragma unroll 1
    for (int ax = 0; ax < 3; ++ax) {
      float v[27];
      const float* vg = a.gv + (size_t)ax * N + gbase;
#pragma unroll
      for (int jz = 0; jz < 3; ++jz)
#pragma unroll
        for (int jy = 0; jy < 3; ++jy)
#pragma unroll
          for (int jx = 0; jx < 3; ++jx) v[jx + 3 * jy + 9 * jz] = vg[jz * nxny + jy * nx + jx];
      float cb[27];
#pragma unroll
      for (int r = 0; r < 27; ++r) cb[r] = 0.0f;
      if (valid) {
        // this workgroup's slice of each row, read at the thread's slot
        const float* cbp = a.coeff_out_grad + (size_t)ax * NR * Ps + i0;
#pragma unroll
        for (int r = 0; r < NR; ++r) cb[r] = row_load(cbp + (size_t)r * Ps, row_n, slot_off);
        if (a.x_out_grad) {
          // advection x' = clamp(x + dt c'_0): recompute c'_0 for the clamp test
          float o[27];
          contract_rows<1>(v, Pr[0], Pr[1], Pr[2], o);
          const float xn = fmaf(a.dt, o[0], xp[ax]);
          if (xn >= a.lo[ax] && xn <= a.hi[ax]) {
            const float xb = row_load(a.x_out_grad + (size_t)ax * Ps + i0, row_n, slot_off);
            xg[ax] += xb;
            cb[0] = fmaf(a.dt, xb, cb[0]);
          }
        }
      }
      // One pass over the nodes gives, per node j, f = sum_r P_r(j) cb_r (the
      // transpose of the projection: v_bar, scattered to the brick), and the
      // sums of v times its t-derivatives, which are the x gradient.
      float sx = 0.0f, sy = 0.0f, sz = 0.0f;
      double* const lbc = lb + ax * kBrickV;
      float* const dst = a.gvb + (size_t)ax * N + gbase;
      stream_g2p_adjoint<NR>(cb, Pr[0], Pr[1], Pr[2], dP[0], dP[1], dP[2], v, sx, sy, sz,
                             [&](int jz, float (&f)[9]) {
                               float w[9];
#pragma unroll
                               for (int k = 0; k < 9; ++k) {
                                 w[k] = pair_fold(f[k], pair_f);
                                 if constexpr (LG == 2) w[k] = quad_fold(w[k], quad_f);
                               }
                               if (!emit) return;
                               if (lds) {
#pragma unroll
                                 for (int jy = 0; jy < 3; ++jy)
#pragma unroll
                                   for (int jx = 0; jx < 3; ++jx)
                                     atomicAdd(lbc + jx + kBrickSY * jy + kBrickSZ * jz,
                                               (double)w[jx + 3 * jy]);
                               } else {
#pragma unroll
                                 for (int jy = 0; jy < 3; ++jy)
#pragma unroll
                                   for (int jx = 0; jx < 3; ++jx)
                                     atomicAdd(dst + jz * nxny + jy * nx + jx, w[jx + 3 * jy]);
                               }
                             });
      xg[0] = fmaf(a.g.inv_dx, sx, xg[0]);
      xg[1] = fmaf(a.g.inv_dx, sy, xg[1]);
      xg[2] = fmaf(a.g.inv_dx, sz, xg[2]);
    }
    if (valid) {
      a.x_in_grad[p] += xg[0];
      a.x_in_grad[Ps + p] += xg[1];
      a.x_in_grad[2 * Ps + p] += xg[2];
    }
  }
  __syncthreads();

  // flush: one global float atomic per component per non-zero brick node, by
  // the node's owner thread
  const int nb = nseg < kBackKMAX ? nseg : kBackKMAX;
  if (tid < kBrickNodes) {
    for (int sb = 0; sb < nb; ++sb) {
      const uint32_t tl = seg_tile[sb];
      const int gx = (int)(tl & 1023u) * kBrickT + bn.lx;
      const int gy = (int)((tl >> 10) & 1023u) * kBrickT + bn.ly;
      const int gz = (int)(tl >> 20) * kBrickT + bn.lz;
      if (gx >= nx || gy >= ny || gz >= nz) continue;
      const size_t node = (size_t)(gz * ny + gy) * nx + gx;
      const double* const src = brick + sb * 3 * kBrickV + bn.lds;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const float v = (float)src[ax * kBrickV];
        if (v != 0.0f) atomicAdd(a.gvb + (size_t)ax * N + node, v);
      }
    }
  }
}

template <int NR>
hipError_t launch_p2g_back_nr(const P2GBackArgs& a, hipStream_t s) {
  p2g_backward_kernel<NR><<<(unsigned)((a.P + 255) / 256), 256, 0, s>>>(a);
  return hipGetLastError();
}

template <int NR>
hipError_t launch_g2p_back_nr(const G2PBackArgs& a, hipStream_t s) {
  constexpr int BS = 256;
  g2p_backward_kernel<NR, BS><<<(unsigned)((a.P + BS - 1) / BS), BS, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_grid_update_backward(const GridUpdateBackArgs& a, hipStream_t stream) {
  grid_update_backward_kernel<<<node_blocks(a.nx, a.ny, a.nz), 256, 0, stream>>>(a);
  return hipGetLastError();
}

hipError_t launch_p2g_backward(const P2GBackArgs& a, int n_modes, hipStream_t stream) {
  if (a.P == 0) return hipSuccess;
  switch (n_modes) {
    case 1: return launch_p2g_back_nr<1>(a, stream);
    case 4: return launch_p2g_back_nr<4>(a, stream);
    case 8: return launch_p2g_back_nr<8>(a, stream);
    case 27: return launch_p2g_back_nr<27>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_g2p_backward(const G2PBackArgs& a, int n_modes, hipStream_t stream) {
  if (a.P == 0) return hipSuccess;
  switch (n_modes) {
    case 1: return launch_g2p_back_nr<1>(a, stream);
    case 4: return launch_g2p_back_nr<4>(a, stream);
    case 8: return launch_g2p_back_nr<8>(a, stream);
    case 27: return launch_g2p_back_nr<27>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace polypic
