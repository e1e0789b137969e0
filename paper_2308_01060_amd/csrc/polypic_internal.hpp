// Internal launch interface between the C ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "polypic_device.hpp"
#include "polypic_scene.hpp"

namespace polypic {

inline size_t align_up(size_t n, size_t a = 256) { return (n + a - 1) / a * a; }

constexpr int kComputeUnits = 256;  // MI355X

// workgroups of 256 threads for a flat one-node-per-thread launch over a grid
// (grids are at most 1026^3 nodes: the count fits 32 bits)
inline unsigned node_blocks(int nx, int ny, int nz) {
  return (unsigned)(((int64_t)nx * ny * nz + 255) / 256);
}

// active regions of an nx x ny x nz grid
inline int64_t region_count(int nx, int ny, int nz) {
  return (int64_t)regions_along(nx, kRegX) * regions_along(ny, kRegY) * regions_along(nz, kRegZ);
}

// ---- sort
size_t sort_workspace_bytes(int64_t P);
int sort_key_bits(const GridDev& g);
hipError_t launch_sort(const GridDev& g, int64_t P, const float* x, uint32_t* keys_out,
                       int32_t* perm_out, void* ws, int32_t* status, hipStream_t stream);
// re-sort after a step (keys_prev: the previous sort's keys, in the current slot order)
size_t sort_update_workspace_bytes(int64_t P);
hipError_t launch_sort_update(const GridDev& g, int64_t P, const float* x,
                              const uint32_t* keys_prev, uint32_t* keys_out, int32_t* perm_out,
                              void* ws, int32_t* status, hipStream_t stream);
hipError_t launch_sort_update_batch(const SceneDev* table, int n_scenes, int mbits, int key_bits,
                                    int64_t P, const float* x, const uint32_t* keys_prev,
                                    uint32_t* keys_out, int32_t* perm_out, void* ws,
                                    int32_t* status, hipStream_t stream);
// batch of scenes: key = scene << mbits | Morton(base node), key_bits in total
hipError_t launch_sort_batch(const SceneDev* table, int n_scenes, int mbits, int key_bits,
                             int64_t P, const float* x, uint32_t* keys_out, int32_t* perm_out,
                             void* ws, int32_t* status, hipStream_t stream);

// ---- P2G
struct P2GArgs {
  GridDev g;
  int64_t P;
  const float* x;      // [3][P]
  const float* mass;   // [P] or nullptr
  float uniform_mass;
  const float* coeff;  // [3][NR][P]
  const int32_t* perm; // [P] or nullptr
  float* gm;           // grid mass [N]
  float* gp0;          // grid momentum, one pointer per component
  float* gp1;
  float* gp2;
  int32_t* status;
  const uint32_t* keys;        // sorted cell keys (cell-gather path) or nullptr
  const uint32_t* tile_list;   // set by the launcher
  const uint32_t* tile_count;
  int sched;                   // chunk schedule (set by the launcher)
};

// Launch configuration chosen by the host (autotuned or default).
struct P2GConfig {
  int tile_log2;       // brick edge = 1 << tile_log2 cells
  int block;           // threads per block = particles per block
  int sched;           // kSchedLinear, kSchedXcd or kSchedPersistent
  int persist_per_cu;  // persistent workgroups per compute unit (kSchedPersistent)
};

P2GConfig p2g_default_config();
bool p2g_config_supported(const P2GConfig& c);
// zeroes grid mass/momentum and, if given, the cell-gather tile counter
hipError_t launch_grid_clear(float* gm, float* gp, int64_t n_nodes, uint32_t* counter,
                             hipStream_t stream);
hipError_t launch_p2g(const P2GArgs& a, int n_modes, const P2GConfig& cfg, hipStream_t stream);
// brick path over a batch of scenes (flattened particles, a.g unused)
hipError_t launch_p2g_batch(const P2GArgs& a, const SceneDev* table, int n_scenes, int n_modes,
                            const P2GConfig& cfg, hipStream_t stream);
int64_t p2g_max_tiles(const GridDev& g, int64_t P);
size_t p2g_workspace_bytes(const GridDev& g, int64_t P);
// sorted-input path; ws holds the tile counter and list (p2g_workspace_bytes)
hipError_t launch_p2g_sorted(const P2GArgs& a, int n_modes, void* ws, bool counter_zeroed,
                             hipStream_t stream);

// ---- grid update
struct GridUpdateArgs {
  int nx, ny, nz;
  float dt;
  float g0, g1, g2;
  int bc_layers;
  const float* gm;
  const float* gp;  // [3][N]
  float* gv;        // [3][N]
  float* clear_gm;  // gm and gp again when the update zeroes them after reading (or nullptr)
  float* clear_gp;
  uint32_t* regions;  // region flags (the active update only)
  int64_t n_regions;
};
hipError_t launch_grid_update(const GridUpdateArgs& a, hipStream_t stream);
// the flagged regions only (a.regions, a.n_regions, a.clear_gm and a.clear_gp set): each
// visited node is updated and cleared, each visited flag reset
hipError_t launch_grid_update_active(const GridUpdateArgs& a, hipStream_t stream);
hipError_t launch_grid_update_active_batch(const GridUpdateArgs& a, const SceneDev* table,
                                           int n_scenes, int64_t stride, hipStream_t stream);
// batch of scenes: a.nx/ny/nz unused; gm, gp, gv span `stride` nodes per channel
hipError_t launch_grid_update_batch(const GridUpdateArgs& a, const SceneDev* table, int n_scenes,
                                    int max_nodes, int64_t stride, hipStream_t stream);
// zero-fills p[0 .. n) with a kernel (no hipMemsetAsync: safe under graph capture)
hipError_t launch_zero(float* p, int64_t n, hipStream_t stream);

// ---- G2P
struct G2PArgs {
  GridDev g;
  int64_t P;
  float dt;
  float dx;
  float lo[3], hi[3];   // clamp bounds for advection
  const float* gv;      // [3][N]
  const float* x_in;    // [3][P]
  const int32_t* perm;  // [P] or nullptr
  float* x_out;         // [3][P] or nullptr
  float* coeff_out;     // [3][NR][P]
  const float* F_in;    // [9][P] or nullptr
  float* F_out;
  const float* mass_in; // [P] or nullptr
  float* mass_out;
  int32_t* status;
  int64_t gstride;      // channel stride of gv (set by the launcher for one scene)
  int sched;            // kSchedLinear or kSchedXcd
};
hipError_t launch_g2p(const G2PArgs& a, int n_modes, hipStream_t stream);
// over a batch of scenes (a.g, a.lo, a.hi, a.dx unused; a.gstride = total nodes)
hipError_t launch_g2p_batch(const G2PArgs& a, const SceneDev* table, int n_scenes, int n_modes,
                            hipStream_t stream);

// ---- G2P fused with the next step's P2G
struct G2P2GArgs {
  GridDev g;
  int64_t P;
  float dt;
  float dx;
  float lo[3], hi[3];    // clamp bounds for advection
  const float* gv;       // [3][N] grid velocity of this step
  const float* x_in;     // [3][P]
  const int32_t* perm;   // [P] or nullptr
  float* x_out;          // [3][P]
  float* coeff_out;      // [3][NR][P]
  const float* F_in;     // [9][P] or nullptr
  float* F_out;
  const float* mass_in;  // [P] or nullptr (then uniform_mass)
  float* mass_out;       // [P] or nullptr
  float uniform_mass;
  float* gm;             // next grid mass [N] (cleared by the launcher)
  float* gp0;            // next grid momentum, [3][N] contiguous from gp0
  float* gp1;
  float* gp2;
  int32_t* status;
  int64_t gstride;       // channel stride of gv
  int lane_group;        // particles folded per brick atomic: 2 (default) or 4
  int accumulate;        // 1: add to the grid as it is (the caller cleared it)
  int sched;             // chunk order: kSchedLinear or kSchedXcd
  uint32_t* regions;     // region flags to set where the scatter lands (or nullptr)
  int64_t n_regions;
};
hipError_t launch_g2p2g(const G2P2GArgs& a, int n_modes, hipStream_t stream);
// over a batch of scenes (a.g, a.lo, a.hi, a.dx unused; a.gstride = total nodes)
hipError_t launch_g2p2g_batch(const G2P2GArgs& a, const SceneDev* table, int n_scenes,
                              int n_modes, hipStream_t stream);

// ---- adjoint
struct GridUpdateBackArgs {
  int nx, ny, nz;
  float dt;
  float g0, g1, g2;
  int bc_layers;
  const float* gm;   // [N]
  const float* gp;   // [3][N]
  const float* gvb;  // [3][N] dL/d grid_vel
  float* gmb;        // [N]   dL/d grid_mass (written)
  float* gpb;        // [3][N] dL/d grid_mom (written)
};
hipError_t launch_grid_update_backward(const GridUpdateBackArgs& a, hipStream_t stream);

struct P2GBackArgs {
  GridDev g;
  int64_t P;
  const float* x;
  const float* mass;
  float uniform_mass;
  const float* coeff;   // [3][NR][P]
  const int32_t* perm;  // processing order or nullptr
  const float* gmb;     // [N]
  const float* gpb;     // [3][N]
  float* coeff_grad;    // [3][NR][P] (written)
  float* x_grad;        // [3][P] (accumulated)
  float* mass_grad;     // [P] (written) or nullptr
  int32_t* status;
};
hipError_t launch_p2g_backward(const P2GBackArgs& a, int n_modes, hipStream_t stream);

struct G2PBackArgs {
  GridDev g;
  int64_t P;
  float dt;
  float lo[3], hi[3];
  const float* gv;              // [3][N]
  const float* x_in;            // [3][P]
  const int32_t* perm;          // [P] or nullptr
  const float* coeff_out_grad;  // [3][NR][P], slot order
  const float* x_out_grad;      // [3][P], slot order, or nullptr
  float* gvb;                   // [3][N] (accumulated)
  float* x_in_grad;             // [3][P] (accumulated at perm[i])
  int32_t* status;
};
hipError_t launch_g2p_backward(const G2PBackArgs& a, int n_modes, hipStream_t stream);

// dst[r][i] = src[r][idx[i]], dst[r][idx[i]] = src[r][i] for rows of P 4-byte
// elements; inv[perm[i]] = i
hipError_t launch_gather_rows(const void* src, void* dst, const int32_t* idx, int64_t rows,
                              int64_t P, hipStream_t stream);
hipError_t launch_scatter_rows(const void* src, void* dst, const int32_t* idx, int64_t rows,
                               int64_t P, hipStream_t stream);
hipError_t launch_invert_permutation(const int32_t* perm, int32_t* inv, int64_t P,
                                     hipStream_t stream);

// ---- staggered (MAC) grid: component a on the faces at origin + (i + (1 - e_a)/2) dx
struct MacP2GArgs {
  GridDev g;
  int64_t P;
  const float* x;       // [3][P]
  const float* mass;    // [P] or nullptr
  float uniform_mass;
  const float* coeff;   // [3][NR][P]
  const int32_t* perm;  // [P] or nullptr
  float* fm;            // face masses [3][N]
  float* fp;            // face momenta [3][N]
  int32_t* status;
};
hipError_t launch_mac_p2g(const MacP2GArgs& a, int n_modes, bool accumulate, hipStream_t s);

struct MacUpdateArgs {
  int nx, ny, nz;
  float dt;
  float g0, g1, g2;
  int bc_layers;
  const float* fm;  // [3][N]
  const float* fp;  // [3][N]
  float* fv;        // [3][N]
};
hipError_t launch_mac_grid_update(const MacUpdateArgs& a, hipStream_t s);

struct MacG2PArgs {
  GridDev g;
  int64_t P;
  float dt;
  float dx;
  float lo[3], hi[3];
  const float* fv;      // face velocities [3][N]
  const float* x_in;
  const int32_t* perm;
  float* x_out;
  float* coeff_out;
  const float* F_in;
  float* F_out;
  const float* mass_in;
  float* mass_out;
  int32_t* status;
};
hipError_t launch_mac_g2p(const MacG2PArgs& a, int n_modes, hipStream_t s);

// ---- P2G with the affine back-map of Eq. 12
struct AffineP2GArgs {
  GridDev g;
  int64_t P;
  float dt;
  const float* x;       // [3][P] present positions
  const float* x_fit;   // [3][P] positions of the fit (nullptr: the present ones)
  const float* mass;    // [P] or nullptr
  float uniform_mass;
  const float* coeff;   // [3][NR][P]
  const int32_t* perm;  // [P] or nullptr
  float* gm;            // [N]
  float* gp;            // [3][N]
  int32_t* status;
};
hipError_t launch_p2g_affine(const AffineP2GArgs& a, int n_modes, bool accumulate, hipStream_t s);

// ---- liquid and fabric particles on one grid (two channel sets per node)
struct MixtureP2GArgs {
  GridDev g;
  int64_t P;
  const float* x;       // [3][P]
  const int32_t* phase; // [P]: 0 fluid, 1 solid
  const float* mass_f;  // [P] fluid mass (absorbed fluid of a solid particle)
  const float* mass_s;  // [P] solid mass or nullptr (0)
  const float* coeff;   // [3][NR][P]
  const int32_t* perm;  // [P] or nullptr
  float* gm;            // [2][N]
  float* gp;            // [2][3][N]
  int32_t* status;
};
hipError_t launch_mixture_p2g(const MixtureP2GArgs& a, int n_modes, bool accumulate,
                              hipStream_t s);

struct MixtureG2PArgs {
  GridDev g;
  int64_t P;
  float dt;
  float dx;
  float lo[3], hi[3];
  const float* gv;        // [2][3][N]
  const float* x_in;
  const int32_t* phase_in;
  const int32_t* perm;
  float* x_out;
  float* coeff_out;
  const float* F_in;
  float* F_out;
  int32_t* phase_out;
  const float* mass_f_in;
  float* mass_f_out;
  const float* mass_s_in;
  float* mass_s_out;
  int32_t* status;
};
hipError_t launch_mixture_g2p(const MixtureG2PArgs& a, int n_modes, hipStream_t s);

}  // namespace polypic
