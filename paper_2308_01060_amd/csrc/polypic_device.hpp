// Device-side building blocks shared by the PolyPIC kernels (gfx950, wave64).
//
// Stencil, quadratic B-spline weights, the 1-D mode factors of Eq. 11 with the
// orthogonalised quadratic of Eq. 14, the G2P projection rows, the mode
// order, and the Morton key.  Everything is float32; the closed forms are the
// factored ones, which keep full relative accuracy as |t| -> 1/2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace polypic {

constexpr int kWave = 64;

// Device flags (mirrors POLYPIC_FLAG_* of the public header).
constexpr int kFlagRange = 1;
constexpr int kFlagOrder = 2;  // a re-sort was given previous keys out of order
constexpr int kFlagStall = 4;  // a sort's chained tile prefixes did not complete
constexpr int kFlagPhase = 8;  // a mixture particle with a phase other than 0 (fluid) or 1 (solid)
constexpr int kFlagMap = 16;   // a singular I + dt C in the affine back-map

struct GridDev {
  int nx, ny, nz;
  float inv_dx;
  float ox, oy, oz;
};

// ---------------------------------------------------------------- mode order
// r -> (kx, ky, kz), graded so that the prefixes 1, 4, 8, 27 are PIC, APIC,
// multilinear and the full quadratic basis.
__host__ __device__ constexpr int mode_code(int r) {
  // code = kx * 9 + ky * 3 + kz
  return r == 0    ? 0
         : r == 1  ? 9
         : r == 2  ? 3
         : r == 3  ? 1
         : r == 4  ? 12
         : r == 5  ? 10
         : r == 6  ? 4
         : r == 7  ? 13
         : r == 8  ? 18
         : r == 9  ? 6
         : r == 10 ? 2
         : r == 11 ? 21
         : r == 12 ? 19
         : r == 13 ? 15
         : r == 14 ? 7
         : r == 15 ? 11
         : r == 16 ? 5
         : r == 17 ? 22
         : r == 18 ? 16
         : r == 19 ? 14
         : r == 20 ? 24
         : r == 21 ? 20
         : r == 22 ? 8
         : r == 23 ? 25
         : r == 24 ? 23
         : r == 25 ? 17
                   : 26;
}

// (kx, ky, kz) -> r
__host__ __device__ constexpr int mode_index(int kx, int ky, int kz) {
  int code = kx * 9 + ky * 3 + kz;
  int r = 0;
  for (int i = 0; i < 27; ++i)
    if (mode_code(i) == code) r = i;
  return r;
}

// Is mode (kx, ky, kz) among the first NR modes?
template <int NR>
__host__ __device__ constexpr bool has_mode(int kx, int ky, int kz) {
  return mode_index(kx, ky, kz) < NR;
}

// ---------------------------------------------------------------- stencil
// u = (x - o) * inv_dx, b = floor(u - 1/2), t = u - b - 1, each a single
// round-to-nearest float32 operation (t is exact).  Returns false when b is
// outside [0, n - 3] (or the position is not finite).
__device__ __forceinline__ bool stencil_axis(float x, float o, float inv_dx, int n, int& b,
                                             float& t) {
  const float u = __fmul_rn(__fsub_rn(x, o), inv_dx);
  const float f = floorf(__fsub_rn(u, 0.5f));
  const bool ok = (f >= 0.0f) && (f <= (float)(n - 3));
  b = ok ? (int)f : 0;
  t = ok ? __fsub_rn(u, f + 1.0f) : 0.0f;
  return ok;
}

// 1-D factors for P2G at the three stencil nodes j = 0, 1, 2:
// w_j (quadratic B-spline), z_j = j - 1 - t, g_j = ghat(z_j) of Eq. 14.
struct Basis1D {
  float w[3];
  float z[3];
  float g[3];
};

__device__ __forceinline__ Basis1D basis_p2g(float t) {
  Basis1D B;
  const float h0 = 0.5f - t;  // exact
  const float h2 = 0.5f + t;  // exact
  const float q = h0 * h2;    // (1 - 4 t^2) / 4
  const float s3 = 2.0f + 4.0f * q;  // 3 - 4 t^2
  B.w[0] = 0.5f * h0 * h0;
  B.w[1] = 0.5f + q;
  B.w[2] = 0.5f * h2 * h2;
  B.z[0] = -1.0f - t;
  B.z[1] = -t;
  B.z[2] = 1.0f - t;
  // ghat_j = zhat_j^2 - t (1 - 4 t^2) zhat_j - 1/4 in factored form
  B.g[0] = h2 * h2 * s3;
  B.g[1] = -4.0f * q * q;
  B.g[2] = h0 * h0 * s3;
  return B;
}

// 1-D G2P projection rows pr[k][j]: coefficient k of a 1-D field f_j is
// sum_j pr[k][j] f_j, with pr[0] = w, pr[1] = 4 w z (since sum w z^2 = 1/4),
// pr[2] = (1/2, -1, 1/2) (since w_j ghat_j = K (1, -2, 1) and
// sum_j (1, -2, 1)_j ghat_j = 2).
struct Proj1D {
  float pr[3][3];
};

__device__ __forceinline__ Proj1D proj_g2p(float t) {
  Proj1D P;
  const float h0 = 0.5f - t;
  const float h2 = 0.5f + t;
  const float w0 = 0.5f * h0 * h0;
  const float w1 = 0.5f + h0 * h2;
  const float w2 = 0.5f * h2 * h2;
  P.pr[0][0] = w0;
  P.pr[0][1] = w1;
  P.pr[0][2] = w2;
  P.pr[1][0] = -2.0f * h0 * h0 * (1.0f + t);
  P.pr[1][1] = -4.0f * t * w1;
  P.pr[1][2] = 2.0f * h2 * h2 * (1.0f - t);
  P.pr[2][0] = 0.5f;
  P.pr[2][1] = -1.0f;
  P.pr[2][2] = 0.5f;
  return P;
}

// ---------------------------------------------------------------- G2P projection
template <int NR>
__device__ constexpr bool need_kx(int kx) {
  return has_mode<NR>(kx, 0, 0) || has_mode<NR>(kx, 0, 1) || has_mode<NR>(kx, 0, 2) ||
         has_mode<NR>(kx, 1, 0) || has_mode<NR>(kx, 1, 1) || has_mode<NR>(kx, 1, 2) ||
         has_mode<NR>(kx, 2, 0) || has_mode<NR>(kx, 2, 1) || has_mode<NR>(kx, 2, 2);
}

template <int NR>
__device__ constexpr bool need_kxky(int kx, int ky) {
  return has_mode<NR>(kx, ky, 0) || has_mode<NR>(kx, ky, 1) || has_mode<NR>(kx, ky, 2);
}

// c[r] = sum_j Px[kx][jx] Py[ky][jy] Pz[kz][jz] v[jx + 3 jy + 9 jz] for r < NR
template <int NR>
__device__ __forceinline__ void project_modes(const float (&v)[27], const Proj1D& px,
                                              const Proj1D& py, const Proj1D& pz,
                                              float (&c)[27]) {
  float A[3][3][3];  // [kx][jy][jz]
#pragma unroll
  for (int kx = 0; kx < 3; ++kx) {
    if (!need_kx<NR>(kx)) continue;
#pragma unroll
    for (int jy = 0; jy < 3; ++jy)
#pragma unroll
      for (int jz = 0; jz < 3; ++jz) {
        const float* vv = v + 3 * jy + 9 * jz;
        if (kx == 2)  // (1/2, -1, 1/2): additions only
          A[kx][jy][jz] = 0.5f * (vv[0] + vv[2]) - vv[1];
        else
          A[kx][jy][jz] = fmaf(px.pr[kx][2], vv[2], fmaf(px.pr[kx][1], vv[1], px.pr[kx][0] * vv[0]));
      }
  }
  float B[3][3][3];  // [kx][ky][jz]
#pragma unroll
  for (int kx = 0; kx < 3; ++kx)
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
      if (!need_kxky<NR>(kx, ky)) continue;
#pragma unroll
      for (int jz = 0; jz < 3; ++jz) {
        if (ky == 2)
          B[kx][ky][jz] = 0.5f * (A[kx][0][jz] + A[kx][2][jz]) - A[kx][1][jz];
        else
          B[kx][ky][jz] = fmaf(py.pr[ky][2], A[kx][2][jz],
                               fmaf(py.pr[ky][1], A[kx][1][jz], py.pr[ky][0] * A[kx][0][jz]));
      }
    }
#pragma unroll
  for (int kx = 0; kx < 3; ++kx)
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int kz = 0; kz < 3; ++kz) {
        if (!has_mode<NR>(kx, ky, kz)) continue;
        float s;
        if (kz == 2)
          s = 0.5f * (B[kx][ky][0] + B[kx][ky][2]) - B[kx][ky][1];
        else
          s = fmaf(pz.pr[kz][2], B[kx][ky][2],
                   fmaf(pz.pr[kz][1], B[kx][ky][1], pz.pr[kz][0] * B[kx][ky][0]));
        c[mode_index(kx, ky, kz)] = s;
      }
}


// ---------------------------------------------------------------- P2G mode evaluation
template <int NR>
__device__ constexpr bool any_kz(int kx, int ky) {
  return has_mode<NR>(kx, ky, 0) || has_mode<NR>(kx, ky, 1) || has_mode<NR>(kx, ky, 2);
}

template <int NR>
__device__ constexpr bool any_kykz(int kx) {
  return any_kz<NR>(kx, 0) || any_kz<NR>(kx, 1) || any_kz<NR>(kx, 2);
}

__device__ __forceinline__ float phi_1d(const Basis1D& B, int k, int j) {
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
          s = first ? (kz == 0 ? term : term * phi_1d(bz, kz, jz))
                    : (kz == 0 ? s + term : fmaf(term, phi_1d(bz, kz, jz), s));
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
          s = first ? (ky == 0 ? term : term * phi_1d(by, ky, jy))
                    : (ky == 0 ? s + term : fmaf(term, phi_1d(by, ky, jy), s));
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
          s = first ? (kx == 0 ? term : term * phi_1d(bx, kx, jx))
                    : (kx == 0 ? s + term : fmaf(term, phi_1d(bx, kx, jx), s));
          first = false;
        }
        V[jx + 3 * jy + 9 * jz] = s;
      }
}

// ---------------------------------------------------------------- adjoint building blocks
// General 1-D row matrix r[k][j]: factor k (0, 1, 2) at stencil node j (0, 1, 2).
struct Rows {
  float r[3][3];
};

// P2G rows R[k][j] = w_j phi_k(j) (weight times mode factor) and dR = dR/dt.
__device__ __forceinline__ void p2g_rows(float t, Rows& R, Rows& dR) {
  const Basis1D B = basis_p2g(t);
  const float h0 = 0.5f - t, h2 = 0.5f + t;
  const float s3 = 2.0f + 4.0f * h0 * h2;  // 3 - 4 t^2
  const float dw[3] = {-h0, -2.0f * t, h2};
  const float dg[3] = {2.0f * h2 * s3 - 8.0f * t * h2 * h2, 16.0f * t * h0 * h2,
                       -2.0f * h0 * s3 - 8.0f * t * h0 * h0};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    R.r[0][j] = B.w[j];
    R.r[1][j] = B.w[j] * B.z[j];
    R.r[2][j] = B.w[j] * B.g[j];
    dR.r[0][j] = dw[j];
    dR.r[1][j] = dw[j] * B.z[j] - B.w[j];  // d zhat / dt = -1
    dR.r[2][j] = dw[j] * B.g[j] + B.w[j] * dg[j];
  }
}

// G2P projection rows (as proj_g2p) and their t-derivatives; the quadratic row
// (1/2, -1, 1/2) does not depend on t.
__device__ __forceinline__ void g2p_rows(float t, Rows& Pr, Rows& dP) {
  const Proj1D P = proj_g2p(t);
  const float h0 = 0.5f - t, h2 = 0.5f + t;
  const float w[3] = {0.5f * h0 * h0, 0.5f + h0 * h2, 0.5f * h2 * h2};
  const float z[3] = {-1.0f - t, -t, 1.0f - t};
  const float dw[3] = {-h0, -2.0f * t, h2};
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 3; ++j) Pr.r[k][j] = P.pr[k][j];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    dP.r[0][j] = dw[j];
    dP.r[1][j] = 4.0f * (dw[j] * z[j] - w[j]);
    dP.r[2][j] = 0.0f;
  }
}

// P2G rows with the weight folded in, scaled by s: R[k][j] = s w_j phi_k(j).
__device__ __forceinline__ Rows p2g_rows_scaled(const Basis1D& B, float s) {
  Rows R;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const float w = s * B.w[j];
    R.r[0][j] = w;
    R.r[1][j] = w * B.z[j];
    R.r[2][j] = w * B.g[j];
  }
  return R;
}

// Nodal values of one channel, node by node: for every stencil node j (z
// outermost, then y, then x) emit(jx, jy, jz, sum_r c_r Rx[kx][jx] Ry[ky][jy]
// Rz[kz][jz]) over the first NR modes.  The three separable stages are
// interleaved with the walk over the nodes, so only 9 + 3 partial sums are live
// besides the coefficients and the rows (the same 3 x 81 multiply-adds as
// contracting the whole array stage by stage).
template <int NR, class Emit>
__device__ __forceinline__ void stream_modes(const float (&c)[27], const Rows& Rx, const Rows& Ry,
                                             const Rows& Rz, Emit&& emit) {
#pragma unroll
  for (int jz = 0; jz < 3; ++jz) {
    float C1[3][3];  // [kx][ky]: z contracted at this jz
#pragma unroll
    for (int kx = 0; kx < 3; ++kx)
#pragma unroll
      for (int ky = 0; ky < 3; ++ky) {
        if (!any_kz<NR>(kx, ky)) continue;
        float acc = 0.0f;
#pragma unroll
        for (int kz = 0; kz < 3; ++kz)
          if (has_mode<NR>(kx, ky, kz)) acc = fmaf(c[mode_index(kx, ky, kz)], Rz.r[kz][jz], acc);
        C1[kx][ky] = acc;
      }
#pragma unroll
    for (int jy = 0; jy < 3; ++jy) {
      float C2[3];  // [kx]
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        if (!any_kykz<NR>(kx)) continue;
        float acc = 0.0f;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
          if (any_kz<NR>(kx, ky)) acc = fmaf(C1[kx][ky], Ry.r[ky][jy], acc);
        C2[kx] = acc;
      }
#pragma unroll
      for (int jx = 0; jx < 3; ++jx) {
        float val = 0.0f;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx)
          if (any_kykz<NR>(kx)) val = fmaf(C2[kx], Rx.r[kx][jx], val);
        emit(jx, jy, jz, val);
      }
    }
  }
}

// As stream_modes, handing over one z plane of nodes at a time:
// emit_plane(jz, v) with v[jx + 3 jy] the 9 nodal values of plane jz.  A caller
// that predicates its atomics per lane then sets the lane mask once per plane
// instead of once per node.
template <int NR, class EmitPlane>
__device__ __forceinline__ void stream_modes_planes(const float (&c)[27], const Rows& Rx,
                                                    const Rows& Ry, const Rows& Rz,
                                                    EmitPlane&& emit_plane) {
#pragma unroll
  for (int jz = 0; jz < 3; ++jz) {
    float C1[3][3];  // [kx][ky]: z contracted at this jz
#pragma unroll
    for (int kx = 0; kx < 3; ++kx)
#pragma unroll
      for (int ky = 0; ky < 3; ++ky) {
        if (!any_kz<NR>(kx, ky)) continue;
        float acc = 0.0f;
#pragma unroll
        for (int kz = 0; kz < 3; ++kz)
          if (has_mode<NR>(kx, ky, kz)) acc = fmaf(c[mode_index(kx, ky, kz)], Rz.r[kz][jz], acc);
        C1[kx][ky] = acc;
      }
    float v[9];
#pragma unroll
    for (int jy = 0; jy < 3; ++jy) {
      float C2[3];  // [kx]
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        if (!any_kykz<NR>(kx)) continue;
        float acc = 0.0f;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
          if (any_kz<NR>(kx, ky)) acc = fmaf(C1[kx][ky], Ry.r[ky][jy], acc);
        C2[kx] = acc;
      }
#pragma unroll
      for (int jx = 0; jx < 3; ++jx) {
        float val = 0.0f;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx)
          if (any_kykz<NR>(kx)) val = fmaf(C2[kx], Rx.r[kx][jx], val);
        v[jx + 3 * jy] = val;
      }
    }
    emit_plane(jz, v);
  }
}

// Transpose of the G2P projection with the x gradient, for projection rows P
// (g2p_rows: row 2 is the constant (1/2, -1, 1/2), so dP row 2 is zero).  For
// every z plane of nodes emits (jz, f) with f[jx + 3 jy] = sum_r c_r Px Py Pz
// (v_bar), and accumulates s_b = sum_j v_j f^(b)_j, f^(b) being f with dP on axis b.  The x
// sums never form f^(b) per node: within one (jy, jz) row of nodes,
//   sum_jx v_j f^(x)_j = sum_kx C2[kx] (dPx v)[kx],
//   sum_jx v_j f^(y)_j = sum_kx C2y[kx] (Px v)[kx]   (and z alike),
// where C2, C2y, C2z are the row's coefficients contracted over z and y.
template <int NR, class Emit>
__device__ __forceinline__ void stream_g2p_adjoint(const float (&c)[27], const Rows& Px,
                                                   const Rows& Py, const Rows& Pz, const Rows& dPx,
                                                   const Rows& dPy, const Rows& dPz,
                                                   const float (&v)[27], float& sx, float& sy,
                                                   float& sz, Emit&& emit) {
#pragma unroll
  for (int jz = 0; jz < 3; ++jz) {
    float fp[9];                // f of the plane's nodes, [jx + 3 jy]
    float C1[3][3], C1z[3][3];  // [kx][ky]
#pragma unroll
    for (int kx = 0; kx < 3; ++kx)
#pragma unroll
      for (int ky = 0; ky < 3; ++ky) {
        if (!any_kz<NR>(kx, ky)) continue;
        float acc = 0.0f, accz = 0.0f;
#pragma unroll
        for (int kz = 0; kz < 3; ++kz)
          if (has_mode<NR>(kx, ky, kz)) {
            const float cr = c[mode_index(kx, ky, kz)];
            acc = fmaf(cr, Pz.r[kz][jz], acc);
            if (kz < 2) accz = fmaf(cr, dPz.r[kz][jz], accz);
          }
        C1[kx][ky] = acc;
        C1z[kx][ky] = accz;
      }
#pragma unroll
    for (int jy = 0; jy < 3; ++jy) {
      float C2[3], C2y[3], C2z[3];  // [kx]
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        if (!any_kykz<NR>(kx)) continue;
        float acc = 0.0f, accy = 0.0f, accz = 0.0f;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
          if (any_kz<NR>(kx, ky)) {
            acc = fmaf(C1[kx][ky], Py.r[ky][jy], acc);
            if (ky < 2) accy = fmaf(C1[kx][ky], dPy.r[ky][jy], accy);
            accz = fmaf(C1z[kx][ky], Py.r[ky][jy], accz);
          }
        C2[kx] = acc;
        C2y[kx] = accy;
        C2z[kx] = accz;
      }
      const float* vr = v + 3 * jy + 9 * jz;
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        if (!any_kykz<NR>(kx)) continue;
        const float pv = kx == 2 ? 0.5f * (vr[0] + vr[2]) - vr[1]
                                 : fmaf(Px.r[kx][2], vr[2], fmaf(Px.r[kx][1], vr[1], Px.r[kx][0] * vr[0]));
        if (kx < 2) {
          const float dv = fmaf(dPx.r[kx][2], vr[2], fmaf(dPx.r[kx][1], vr[1], dPx.r[kx][0] * vr[0]));
          sx = fmaf(C2[kx], dv, sx);
        }
        sy = fmaf(C2y[kx], pv, sy);
        sz = fmaf(C2z[kx], pv, sz);
      }
#pragma unroll
      for (int jx = 0; jx < 3; ++jx) {
        float f = 0.0f;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx)
          if (any_kykz<NR>(kx)) f = fmaf(C2[kx], Px.r[kx][jx], f);
        fp[jx + 3 * jy] = f;
      }
    }
    emit(jz, fp);
  }
}

template <int NR>
__device__ constexpr bool need_kx_any(int kx) {
  return any_kykz<NR>(kx);
}

// out[r] = sum_j Rx[kx][jx] Ry[ky][jy] Rz[kz][jz] v[jx + 3 jy + 9 jz] for r < NR
// (separable: contract x, then y, then z).
template <int NR>
__device__ __forceinline__ void contract_rows(const float (&v)[27], const Rows& Rx, const Rows& Ry,
                                              const Rows& Rz, float (&out)[27]) {
  float A[3][3][3];  // [kx][jy][jz]
#pragma unroll
  for (int kx = 0; kx < 3; ++kx) {
    if (!any_kykz<NR>(kx)) continue;
#pragma unroll
    for (int jy = 0; jy < 3; ++jy)
#pragma unroll
      for (int jz = 0; jz < 3; ++jz) {
        const float* vv = v + 3 * jy + 9 * jz;
        A[kx][jy][jz] = fmaf(Rx.r[kx][2], vv[2], fmaf(Rx.r[kx][1], vv[1], Rx.r[kx][0] * vv[0]));
      }
  }
  float B[3][3][3];  // [kx][ky][jz]
#pragma unroll
  for (int kx = 0; kx < 3; ++kx)
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
      if (!any_kz<NR>(kx, ky)) continue;
#pragma unroll
      for (int jz = 0; jz < 3; ++jz)
        B[kx][ky][jz] = fmaf(Ry.r[ky][2], A[kx][2][jz],
                             fmaf(Ry.r[ky][1], A[kx][1][jz], Ry.r[ky][0] * A[kx][0][jz]));
    }
#pragma unroll
  for (int kx = 0; kx < 3; ++kx)
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int kz = 0; kz < 3; ++kz) {
        if (!has_mode<NR>(kx, ky, kz)) continue;
        out[mode_index(kx, ky, kz)] =
            fmaf(Rz.r[kz][2], B[kx][ky][2], fmaf(Rz.r[kz][1], B[kx][ky][1], Rz.r[kz][0] * B[kx][ky][0]));
      }
}

// V[jx + 3 jy + 9 jz] = sum_{r < NR} c[r] Rx[kx][jx] Ry[ky][jy] Rz[kz][jz]
// (the transpose of contract_rows).
template <int NR>
__device__ __forceinline__ void expand_rows(const float (&c)[27], const Rows& Rx, const Rows& Ry,
                                            const Rows& Rz, float (&V)[27]) {
  float A[3][3][3];  // [kx][ky][jz]
#pragma unroll
  for (int kx = 0; kx < 3; ++kx)
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
      if (!any_kz<NR>(kx, ky)) continue;
#pragma unroll
      for (int jz = 0; jz < 3; ++jz) {
        float s = 0.0f;
#pragma unroll
        for (int kz = 0; kz < 3; ++kz)
          if (has_mode<NR>(kx, ky, kz)) s = fmaf(c[mode_index(kx, ky, kz)], Rz.r[kz][jz], s);
        A[kx][ky][jz] = s;
      }
    }
  float B[3][3][3];  // [kx][jy][jz]
#pragma unroll
  for (int kx = 0; kx < 3; ++kx) {
    if (!any_kykz<NR>(kx)) continue;
#pragma unroll
    for (int jy = 0; jy < 3; ++jy)
#pragma unroll
      for (int jz = 0; jz < 3; ++jz) {
        float s = 0.0f;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
          if (any_kz<NR>(kx, ky)) s = fmaf(A[kx][ky][jz], Ry.r[ky][jy], s);
        B[kx][jy][jz] = s;
      }
  }
#pragma unroll
  for (int jx = 0; jx < 3; ++jx)
#pragma unroll
    for (int jy = 0; jy < 3; ++jy)
#pragma unroll
      for (int jz = 0; jz < 3; ++jz) {
        float s = 0.0f;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx)
          if (any_kykz<NR>(kx)) s = fmaf(B[kx][jy][jz], Rx.r[kx][jx], s);
        V[jx + 3 * jy + 9 * jz] = s;
      }
}

// FP64 LDS brick of a 4^3-cell tile: 6^3 nodes stored with strides (1, 8, 68)
// doubles.  With the lanes of a wavefront spread over the 64 cells of a tile,
// the 32 cells handled by each half-wavefront fall on 32 distinct LDS bank
// pairs for every stencil node.
constexpr int kBrickKMAX = 3;  // bricks (tiles) per workgroup in LDS

// Tile id of a base node: 4^3-node tile coordinates, plus the scene relative
// to the chunk's first scene in the high word (zero for one scene).
__device__ __forceinline__ uint64_t brick_tile_id(int s_rel, int b0, int b1, int b2) {
  return ((uint64_t)(uint32_t)s_rel << 32) | (uint64_t)((uint32_t)(b0 >> 2) |
                                                       ((uint32_t)(b1 >> 2) << 10) |
                                                       ((uint32_t)(b2 >> 2) << 20));
}
constexpr uint64_t kNoTile = ~0ull;

constexpr int kBrickT = 4;  // tile edge in cells
constexpr int kBrickSY = 8;
constexpr int kBrickSZ = 68;
constexpr int kBrickV = 5 + 5 * kBrickSY + 5 * kBrickSZ + 1;  // 386 doubles per channel
constexpr int kBrickN = kBrickT + 2;                           // nodes per brick edge
constexpr int kBrickNodes = kBrickN * kBrickN * kBrickN;       // 216

// Brick node owned by thread t < kBrickNodes (x fastest): the thread clears it in
// every brick and channel and flushes it, so the padding is never touched.
struct BrickNode {
  int lx, ly, lz;
  int lds;  // offset in a channel, in doubles
};
__device__ __forceinline__ BrickNode brick_node(int t) {
  BrickNode n;
  n.lz = t / (kBrickN * kBrickN);
  n.ly = (t / kBrickN) % kBrickN;
  n.lx = t % kBrickN;
  n.lds = n.lx + kBrickSY * n.ly + kBrickSZ * n.lz;
  return n;
}

// ---------------------------------------------------------------- active regions
// Nodes grouped in boxes of 16 x 4 x 4 (x fastest; the last box of an axis may be
// partial), numbered x fastest, one uint32 flag each.  The scatter of a stepped
// simulation sets the flags of the boxes it touches (plain stores: nothing waits on
// them) and the next grid pass visits only flagged boxes, resetting their flags.  A
// row of a box is 64 bytes of one channel.
constexpr int kRegX = 16, kRegY = 4, kRegZ = 4;

__host__ __device__ inline int regions_along(int n, int e) { return (n + e - 1) / e; }

// region of node (gx, gy, gz) of an nx x ny grid
__device__ __forceinline__ int64_t region_of(int nx, int ny, int gx, int gy, int gz) {
  const int rx = regions_along(nx, kRegX), ry = regions_along(ny, kRegY);
  return ((int64_t)(gz / kRegZ) * ry + gy / kRegY) * rx + gx / kRegX;
}

// Flags every region that holds a node of the box [lo, lo + ext) per axis (ext <= 16
// on y and z, <= 32 on x: at most two regions per axis, found from the box's corners),
// clipped to the grid; corner in [0, 8) selects one corner: call it for each.  A flag
// holds 1 + the scene of the region (0 for one grid), so the pass that visits it needs
// no lookup.
__device__ __forceinline__ void flag_box_corner(uint32_t* flags, int64_t region_off,
                                                uint32_t scene, int nx, int ny, int nz, int lo0,
                                                int lo1, int lo2, int ext, int corner) {
  const int gx = min(lo0 + ((corner & 1) ? ext - 1 : 0), nx - 1);
  const int gy = min(lo1 + ((corner & 2) ? ext - 1 : 0), ny - 1);
  const int gz = min(lo2 + ((corner & 4) ? ext - 1 : 0), nz - 1);
  flags[region_off + region_of(nx, ny, gx, gy, gz)] = scene + 1u;
}

// ---------------------------------------------------------------- Morton key
__device__ __forceinline__ uint32_t spread_bits3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ __forceinline__ uint32_t compact_bits3(uint32_t v) {
  v &= 0x09249249u;
  v = (v | (v >> 2)) & 0x030C30C3u;
  v = (v | (v >> 4)) & 0x0300F00Fu;
  v = (v | (v >> 8)) & 0x030000FFu;
  v = (v | (v >> 16)) & 0x000003FFu;
  return v;
}

__device__ __forceinline__ uint32_t morton3(int bx, int by, int bz) {
  return spread_bits3((uint32_t)bx) | (spread_bits3((uint32_t)by) << 1) |
         (spread_bits3((uint32_t)bz) << 2);
}

// DPP exchanges within a quad of lanes: with lane ^ 1, and with lane ^ 2
__device__ __forceinline__ int pair_swap_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad_perm [1, 0, 3, 2]
}
__device__ __forceinline__ int quad_swap_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // quad_perm [2, 3, 0, 1]
}

// v + f * (v of lane ^ 1), and v + f * (v of lane ^ 2), each one v_fmac_f32 with a
// DPP source (the compiler emits a DPP move and a separate multiply-add instead).
// With f 1 or 0 per lane, a lane adds its partner's value only where both belong
// together; a non-finite partner value still reaches a lane with f = 0, as NaN.
// Every lane of the quad must execute the call.  The s_nop gives the two wait
// states a DPP read needs after a VALU write of its source.
__device__ __forceinline__ float pair_fold(float v, float f) {
  asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %0, %1 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf"
               : "+v"(v)
               : "v"(f));
  return v;
}
__device__ __forceinline__ float quad_fold(float v, float f) {
  asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %0, %1 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf"
               : "+v"(v)
               : "v"(f));
  return v;
}

// ---------------------------------------------------------------- workgroup rows
// Access to this thread's float of a workgroup's slice of a particle row, through
// a buffer descriptor over the slice (its base and its n valid floats), which is
// wave-uniform: the address is then a scalar base plus a 32-bit lane offset, with
// no per-access vector arithmetic (a global access to p + t costs a 64-bit vector
// add, and two registers while in flight).  Lanes at or past n are dropped (a
// store) or read 0 (a load) by the descriptor's range check.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const float* row, int n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(row), 0, n * (int)sizeof(float),
                                           0x00020000);
}
__device__ __forceinline__ void row_store_nt(float v, float* row, int n, int lane_byte_off) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), row_rsrc(row, n), lane_byte_off, 0,
                                        2 /* nt */);
}
__device__ __forceinline__ float row_load(const float* row, int n, int lane_byte_off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(row_rsrc(row, n), lane_byte_off, 0, 0));
}

// popcount of the bits of `mask` below this lane
__device__ __forceinline__ int lanes_below(unsigned long long mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ void raise_flag(int32_t* status, int flag) {
  if (status) atomicOr(status, flag);
}

// Node of this thread in a flat launch over an nx x ny x nz grid (x fastest, one
// node per thread): its flat index and coordinates; false past the last node.
// Flat, every wavefront covers 64 consecutive nodes whatever the row length.
__device__ __forceinline__ bool flat_node(int nx, int ny, int nz, uint32_t& n, int& ix, int& iy,
                                          int& iz) {
  n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= (uint32_t)nx * (uint32_t)ny * (uint32_t)nz) return false;
  const uint32_t r = n / (uint32_t)nx;
  ix = (int)(n - r * (uint32_t)nx);
  iz = (int)(r / (uint32_t)ny);
  iy = (int)(r - (uint32_t)iz * (uint32_t)ny);
  return true;
}

}  // namespace polypic
