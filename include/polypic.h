/*
 * polypic.h -- C ABI of the PolyPIC transfer library for AMD Instinct MI355X (gfx950).
 *
 * The library implements the particle/grid transfers of the Polynomial
 * Particle-in-Cell method as used for liquid and fabric in Dennison & Maddock,
 * "Using The Polynomial Particle-in-Cell Method for Liquid-Fabric Interaction"
 * (section 3): P2G (Eq. 1, 4, 13; Eq. 15-16 and 18-19 for the fluid and the
 * solid-plus-absorbed-fluid sets), the grid velocity of Eq. 5 with a light
 * explicit update, and G2P (Eq. 6-8 generalised to the weighted least-squares
 * fit of the polynomial modes, section 3.3).  APIC (section 3.2) is the
 * 4-mode case, PIC (section 3.1) the 1-mode case.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory      Every array argument is a DEVICE pointer owned by the caller.  The
 *             library allocates no device memory; scratch comes from a caller
 *             workspace whose size is queried first.  The polypic_grid struct
 *             and the gravity vector are HOST pointers, read during the call.
 * Streams     `stream` is a hipStream_t (NULL = the default stream).  Every
 *             call only enqueues work on it and never synchronises; buffers must
 *             stay alive until that work has completed.
 * Status      Calls return POLYPIC_OK or a host-detected error code below; on an
 *             error nothing is enqueued.  Conditions found on the device (a
 *             particle whose stencil leaves the grid) are OR-ed as POLYPIC_FLAG_*
 *             bits into the optional caller-owned `int32_t* status_dev` (device
 *             memory, may be NULL); the offending particle is skipped, never
 *             written out of bounds.  The library never aborts the process.
 * Layouts     SoA float32.  Positions x[3][P] (all x, then all y, then all z).
 *             Coefficients coeff[3][n_modes][P]: component a, mode r, particle p
 *             at ((a * n_modes) + r) * P + p.  Grid arrays grid_mass[N] and
 *             grid_mom[3][N] / grid_vel[3][N] with N = nx * ny * nz and node
 *             (ix, iy, iz) at (iz * ny + iy) * nx + ix (x fastest).
 *             Deformation gradients F[9][P], entry (a, b) of particle p at
 *             (3a + b) * P + p.
 * Grid        Collocated: node (ix, iy, iz) sits at origin + (ix, iy, iz) * dx.
 *             The paper's runs use MAC grids (section 3); this library uses the
 *             collocated form, where the per-face quantities of Table 1 become
 *             per-node quantities.
 * Stencil     Quadratic B-spline weights (section 3.1 leaves N(x) unnamed) over
 *             the 3x3x3 nodes b, b+1, b+2 per axis, where, in float32 with
 *             round-to-nearest and no contraction,
 *                 u = (x - origin) * inv_dx,   b = floor(u - 1/2),   t = u - b - 1
 *             (t in [-1/2, 1/2) is the offset from the nearest node b + 1).  A
 *             particle is in range when 0 <= b <= n_axis - 3 on every axis.
 * Modes       s_r = phi_kx(zx) phi_ky(zy) phi_kz(zz) evaluated at
 *             z = (x_i - x_p) / dx (the particle's current position; the affine
 *             map of Eq. 12 is not applied) with phi_0 = 1, phi_1 = z and
 *             phi_2 = ghat(z) = z^2 - t (1 - 4 t^2) z - 1/4, the orthogonalised
 *             quadratic of Eq. 14 in units of dx.  Mode order (r -> kx ky kz):
 *               0:000  1:100  2:010  3:001  4:110  5:101  6:011  7:111
 *               8:200  9:020 10:002 11:210 12:201 13:120 14:021 15:102 16:012
 *              17:211 18:121 19:112 20:220 21:202 22:022 23:221 24:212 25:122
 *              26:222
 *             so n_modes = 1, 4, 8, 27 is PIC, APIC, multilinear (the paper's
 *             8 modes, section 4) and the full quadratic basis.  Coefficients are
 *             in these normalised units: mode 0 is the particle velocity, and
 *             the APIC matrix of section 3.2 is C_ab = coeff[a][1 + b] / dx.
 * Sizes       P <= 2^31 - 1 particles; 3 <= n_axis <= 1026 nodes per axis.
 * Threads     All entry points are reentrant; calls on different streams may
 *             run concurrently on disjoint outputs.
 */
#ifndef POLYPIC_H
#define POLYPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes (return values) ---- */
#define POLYPIC_OK 0
#define POLYPIC_EINVAL 1   /* null pointer, bad size, n_modes not in {1, 4, 8, 27}, ... */
#define POLYPIC_ERANGE 2   /* host-detected range problem (e.g. grid too large for the keys) */
#define POLYPIC_EDEVICE 3  /* a HIP call failed (launch error, no device) */
#define POLYPIC_ENOSPACE 4 /* the workspace is smaller than the queried size */
#define POLYPIC_ENOTSUP 5  /* valid request this build does not support */

/* ---- device status flags, OR-ed into *status_dev ---- */
#define POLYPIC_FLAG_RANGE 1 /* a particle's stencil left the grid; it was skipped */
#define POLYPIC_FLAG_ORDER 2 /* polypic_sort_update was given keys_prev out of order */
#define POLYPIC_FLAG_STALL 4 /* a re-sort pass gave up waiting on an earlier tile (a tile that
                              * waits far longer than any run takes); outputs unspecified */
#define POLYPIC_FLAG_PHASE 8 /* a mixture particle's phase was neither 0 (fluid) nor 1 (solid);
                              * it was skipped */
#define POLYPIC_FLAG_MAP 16  /* a singular I + dt C in the affine back-map; particle skipped */

/* Collocated grid description (host struct, passed by pointer). */
typedef struct polypic_grid {
  int32_t nx, ny, nz; /* node counts per axis, each in [3, 1026] */
  float dx;           /* node spacing (> 0) */
  float inv_dx;       /* the float32 factor used in u = (x - origin) * inv_dx */
  float origin[3];    /* world position of node (0, 0, 0) */
} polypic_grid;

/* Human-readable name of a status code (static string, never NULL). */
const char* polypic_strerror(int32_t code);

/* Library ABI version: major * 10000 + minor * 100 + patch. */
int32_t polypic_version(void);

/* Name of the HIP error behind the last POLYPIC_EDEVICE returned on the calling
 * thread ("no error" if none).  Static string owned by the library. */
const char* polypic_last_device_error(void);

/* ------------------------------------------------------------------------
 * Cell-key sort (not part of the paper: it orders particles so that P2G can
 * accumulate neighbouring particles in on-chip grid bricks).
 *
 * key(p) = Morton code of the stencil base node b(p): bit k of b_x, b_y, b_z
 * goes to key bits 3k, 3k+1, 3k+2.  The sort is a stable LSD radix sort:
 * keys_out[i] = key(perm_out[i]), ascending, ties in input order.  Particles
 * out of range get the key of their clamped base node and raise
 * POLYPIC_FLAG_RANGE.
 *
 * x[3][P] in; keys_out[P], perm_out[P] out (device).  ws: device workspace of
 * at least polypic_sort_workspace_bytes() bytes, contents scratch.
 * ------------------------------------------------------------------------ */
int32_t polypic_sort_workspace_bytes(const polypic_grid* grid, int64_t P, size_t* bytes);
int32_t polypic_sort(const polypic_grid* grid, int64_t P, const float* x, uint32_t* keys_out,
                     int32_t* perm_out, void* ws, size_t ws_bytes, int32_t* status_dev,
                     void* stream);

/* ------------------------------------------------------------------------
 * Allocation-free variant of polypic_sort, for callers that cannot allocate
 * device memory or pass a workspace: code under HIP graph capture, tight
 * stepping loops, harnesses that forbid hipMalloc.
 *
 * Same keys_out / perm_out as polypic_sort, bit for bit.  The workspace is a
 * static device array inside the library (18 MiB, held on every GPU the
 * library runs on until the process ends), so the call allocates nothing and
 * takes no ws argument.  P is limited to POLYPIC_SORT_NOALLOC_MAX_P particles;
 * a larger P returns POLYPIC_ENOSPACE with nothing enqueued.
 *
 * All calls on one GPU share that GPU's array: two calls whose work overlaps
 * on the device (on different streams, or from different threads without
 * ordering) race and give unspecified keys and permutations.  Calls ordered
 * on one stream are safe; every word the sort reads from the array it has
 * written earlier in the same call.
 * ------------------------------------------------------------------------ */
#define POLYPIC_SORT_NOALLOC_MAX_P 2097152
int32_t polypic_sort_noalloc(const polypic_grid* grid, int64_t P, const float* x,
                             uint32_t* keys_out, int32_t* perm_out, int32_t* status_dev,
                             void* stream);

/* ------------------------------------------------------------------------
 * Re-sort after a step: the same result as polypic_sort, bit for bit, faster
 * when few particles changed cell.
 *
 * keys_prev[P] (device, read only): the keys_out of the previous sort, the
 * particle arrays having been permuted by its perm_out since (as polypic_g2p
 * does with perm), so that keys_prev[i] is the key slot i was sorted under
 * and keys_prev is ascending.  Particles whose key is unchanged already form
 * an ordered subsequence; only the changed ones are sorted (radix), and the
 * two are merged by (key, index).  keys_prev must not alias keys_out.  If
 * keys_prev is not ascending, POLYPIC_FLAG_ORDER is raised and the outputs
 * are unspecified (every written index stays in [0, P)).  The sort of the
 * changed particles chains its tiles' digit prefixes through device memory;
 * a tile that waits on its predecessor far longer than any run takes (which
 * does not happen when the launches run in order on one stream) stops
 * waiting and raises POLYPIC_FLAG_STALL, the outputs then unspecified.
 * ws: at least polypic_sort_update_workspace_bytes() bytes (about 19 B per
 * particle plus 128 KB), contents scratch.
 * ------------------------------------------------------------------------ */
int32_t polypic_sort_update_workspace_bytes(const polypic_grid* grid, int64_t P, size_t* bytes);
int32_t polypic_sort_update(const polypic_grid* grid, int64_t P, const float* x,
                            const uint32_t* keys_prev, uint32_t* keys_out, int32_t* perm_out,
                            void* ws, size_t ws_bytes, int32_t* status_dev, void* stream);

/* ------------------------------------------------------------------------
 * P2G scatter.  Section 3.1 Eq. 1 and 4 (mass), Eq. 13 (momentum), summed over
 * particles as in Eq. 3; for a fluid set Eq. 15-16, for a fabric set Eq. 18-19
 * with the per-point mass m_s + m_f folded into `mass`:
 *     grid_mass[i]    (+)= sum_p m_p W_ip
 *     grid_mom[a][i]  (+)= sum_p m_p W_ip sum_{r < n_modes} coeff[a][r][p] s_r(z_ip)
 * with W_ip = w_x w_y w_z the product of quadratic B-spline weights.
 *
 * P             particle count (0 is allowed: only the clear happens).
 * n_modes       1, 4, 8 or 27.
 * x[3][P]       positions.  mass[P] per-particle mass, or NULL for uniform_mass.
 * coeff         [3][n_modes][P] coefficients.
 * perm          NULL, or the processing order (a permutation of 0..P-1): slot i
 *               handles particle perm[i].
 * keys_sorted   NULL, or the sorted cell keys of that order (keys_sorted and
 *               perm as returned together by polypic_sort for this x and grid).
 *               They enable the cell-run path (per-cell sums, one workgroup
 *               per 4^3-cell tile), used when the configuration table selects
 *               it.  The default brick path needs only perm: in sorted order,
 *               lane groups of particles sharing a cell add their nodal values
 *               across lanes, bricks of 4^3 tiles accumulate in LDS and reach
 *               HBM with one atomic per node and channel.  Any order is
 *               correct; unsorted input is slower.
 * ws, ws_bytes  device workspace, at least polypic_p2g_workspace_bytes(); used
 *               only with keys_sorted (may be NULL otherwise).
 * grid_mass[N], grid_mom[3][N]   outputs (device).
 * accumulate    0: outputs are zeroed first; 1: sums are added to their contents.
 * Summation order is not fixed (float atomics), so results are deterministic
 * only up to rounding.  A particle whose stencil leaves the grid (or, on the
 * fast path, whose key does not match its position) is skipped and raises
 * POLYPIC_FLAG_RANGE.
 * ------------------------------------------------------------------------ */
int32_t polypic_p2g_workspace_bytes(const polypic_grid* grid, int64_t P, size_t* bytes);
int32_t polypic_p2g(const polypic_grid* grid, int64_t P, int32_t n_modes, const float* x,
                    const float* mass, float uniform_mass, const float* coeff, const int32_t* perm,
                    const uint32_t* keys_sorted, void* ws, size_t ws_bytes, float* grid_mass,
                    float* grid_mom, int32_t accumulate, int32_t* status_dev, void* stream);

/* ------------------------------------------------------------------------
 * P2G launch configuration and autotuner (a runtime choice, no effect on
 * results beyond float summation order).
 *
 * path   POLYPIC_P2G_BRICKS: per-particle scatter into FP64 LDS bricks (needs
 *        only perm); POLYPIC_P2G_CELLS: per-cell run sums of 4^3-cell tiles
 *        (needs keys_sorted).  block: workgroup size of the brick path (256 or
 *        512).
 * brick  edge of the brick path's tiles in cells: 2, 4 (the default) or 8.  A
 *        brick holds the (edge + 2)^3 nodes of a tile's stencils; a workgroup
 *        has 12, 3 or 1 of them in LDS (29 to 37 KB).  Runs of one tile in the
 *        chunk share a brick; runs beyond the bricks add to HBM.
 * schedule  how the brick path's workgroups take chunks of `block` slots:
 *        POLYPIC_SCHED_LINEAR      one chunk per workgroup, in index order;
 *        POLYPIC_SCHED_XCD         one chunk per workgroup, renumbered so that
 *                                  the workgroups the dispatcher places on one
 *                                  of the 8 XCDs take a contiguous eighth of
 *                                  the chunks (sorted neighbours share an L2);
 *        POLYPIC_SCHED_PERSISTENT  per_cu workgroups per compute unit (1..64),
 *                                  each looping over a contiguous chunk range.
 *        per_cu is ignored by the other schedules (pass 0).
 * The choice is kept per n_modes in a process-wide, mutex-guarded table.
 * Without an entry polypic_p2g uses the brick path (block 256, linear, 4^3
 * bricks); the cell path runs only when chosen and keys_sorted is given.
 *
 * polypic_autotune_p2g runs P2G once per candidate configuration on the given
 * inputs (same arguments as polypic_p2g, keys_sorted may be NULL), times each
 * with HIP events on `stream`, stores the fastest and returns it through the
 * *_out host pointers (each may be NULL).  Unlike the other entry points it
 * SYNCHRONISES the stream.  On return grid_mass / grid_mom hold a P2G result
 * (accumulate = 0).
 *
 * polypic_set_g2p_schedule: process-wide chunk schedule of G2P (LINEAR or XCD;
 * default LINEAR).
 * ------------------------------------------------------------------------ */
#define POLYPIC_P2G_DEFAULT (-1)
#define POLYPIC_P2G_BRICKS 0
#define POLYPIC_P2G_CELLS 1
#define POLYPIC_SCHED_LINEAR 0
#define POLYPIC_SCHED_XCD 1
#define POLYPIC_SCHED_PERSISTENT 2
int32_t polypic_set_p2g_config(int32_t n_modes, int32_t path, int32_t block, int32_t schedule,
                               int32_t per_cu, int32_t brick);
int32_t polypic_get_p2g_config(int32_t n_modes, int32_t* path, int32_t* block, int32_t* schedule,
                               int32_t* per_cu, int32_t* brick);
int32_t polypic_autotune_p2g(const polypic_grid* grid, int64_t P, int32_t n_modes, const float* x,
                             const float* mass, float uniform_mass, const float* coeff,
                             const int32_t* perm, const uint32_t* keys_sorted, void* ws,
                             size_t ws_bytes, float* grid_mass, float* grid_mom,
                             int32_t* path_out, int32_t* block_out, int32_t* schedule_out,
                             int32_t* per_cu_out, int32_t* brick_out, void* stream);
int32_t polypic_set_g2p_schedule(int32_t schedule);
int32_t polypic_get_g2p_schedule(int32_t* schedule);

/* ------------------------------------------------------------------------
 * Grid update.  Eq. 5 (v = (mv) / m) followed by an explicit update that the
 * paper delegates to its host model: gravity and separating slip walls.
 *     v_i = grid_mom[i] / grid_mass[i] + dt * gravity   where grid_mass[i] > 0
 *     v_i = 0                                           where grid_mass[i] == 0
 * then, if bc_layers > 0, per axis a with storage index i_a along it:
 *     v_a = max(v_a, 0)  where i_a <= 1 + bc_layers
 *     v_a = min(v_a, 0)  where i_a >= n_a - 1 - bc_layers
 * gravity: HOST float[3].  grid_vel[3][N] out; may not alias the inputs.
 * ------------------------------------------------------------------------ */
int32_t polypic_grid_update(const polypic_grid* grid, float dt, const float* gravity,
                            int32_t bc_layers, const float* grid_mass, const float* grid_mom,
                            float* grid_vel, void* stream);

/* ------------------------------------------------------------------------
 * polypic_grid_update that also clears its inputs: each node's mass and
 * momentum are set to zero once read, so that the next fused call
 * (polypic_g2p2g with accumulate = 1) scatters into a cleared grid without a
 * pass of its own.  Not in the paper: a merge of two passes over the grid.
 * grid_mass and grid_mom are read, then overwritten with zeros; grid_vel as
 * polypic_grid_update.
 * ------------------------------------------------------------------------ */
int32_t polypic_grid_update_clear(const polypic_grid* grid, float dt, const float* gravity,
                                  int32_t bc_layers, float* grid_mass, float* grid_mom,
                                  float* grid_vel, void* stream);

/* ------------------------------------------------------------------------
 * Active regions: the grid passes of a stepped simulation restricted to where
 * the particles are.  Not in the paper (the grid is dense there); bookkeeping
 * that spares the passes the empty part of a large grid.
 *
 * The nodes are grouped in regions of 16 x 4 x 4 (x fastest; the last region of
 * an axis may be partial), numbered x fastest: region (qx, qy, qz) has index
 * (qz * ry + qy) * rx + qx with rx = ceil(nx / 16), ry = ceil(ny / 4);
 * polypic_region_count gives their number R.  The caller owns the region state:
 * R uint32 flags (word q for region q), zero at first.
 *
 * polypic_g2p2g with region_state non-NULL sets the flag of every region its
 * scatter adds to (and possibly of a few next to them).
 * polypic_grid_update_active then does what polypic_grid_update_clear does, on
 * the flagged regions only, and resets their flags.  It requires grid_mass and
 * grid_mom to be zero outside the flagged regions; it leaves them zero
 * everywhere, and grid_vel unchanged outside the flagged regions (velocities a
 * later G2P does not read: a G2P reads the nodes of its particles' stencils, all
 * in regions the scatter of the same positions flagged).  A stepped run keeps
 * the requirement: after a dense update with clearing, every later step is
 * polypic_grid_update_active, then polypic_g2p2g with accumulate = 1 and the
 * region state.
 * ------------------------------------------------------------------------ */
int32_t polypic_region_count(const polypic_grid* grid, int64_t* count);
int32_t polypic_grid_update_active(const polypic_grid* grid, float dt, const float* gravity,
                                   int32_t bc_layers, float* grid_mass, float* grid_mom,
                                   float* grid_vel, uint32_t* region_state, void* stream);

/* ------------------------------------------------------------------------
 * G2P gather + projection.  Eq. 6-8 generalised as in section 3.3: the
 * coefficients minimise sum_i W_ip (v_i - sum_r c_r s_r(z_ip))^2.  The modes
 * are W-orthogonal (Eq. 14), so mode by mode
 *     coeff_out[a][r][i] = <v_a, s_r>_W / <s_r, s_r>_W
 * On an axis where the mode is quadratic the common factor of numerator and
 * denominator, K(t) = (1 - 4t^2)^2 (3 - 4t^2) / 32, is cancelled; this also
 * defines the coefficient at t = -1/2, where K vanishes, as the limit from
 * t > -1/2.
 *
 * Output slot i belongs to particle perm[i] (identity when perm is NULL), so
 * with a sort permutation every output comes out in sorted order.
 * x_out[3][P]   optional (NULL: no advection): clamp(x + dt * coeff_out[.][0]),
 *               each axis kept in [origin + 2 dx, origin + (n_a - 2) dx) -- the
 *               lower bound, or the largest float32 below the upper bound.
 * F_in, F_out   optional [9][P] (both or neither): F' = (I + dt C) F with
 *               C_ab = coeff_out[a][1 + b] / dx (C = 0 when n_modes == 1).
 * mass_in, mass_out  optional [P] (both or neither): mass_out[i] = mass_in[perm[i]]
 *               so a per-particle mass follows the new order.
 * Outputs may not alias inputs.  coeff_out may be the coefficient array of the
 * preceding polypic_p2g (G2P reads no coefficients): an in-place update.
 * ------------------------------------------------------------------------ */
int32_t polypic_g2p(const polypic_grid* grid, int64_t P, int32_t n_modes, float dt,
                    const float* grid_vel, const float* x_in, const int32_t* perm, float* x_out,
                    float* coeff_out, const float* F_in, float* F_out, const float* mass_in,
                    float* mass_out, int32_t* status_dev, void* stream);

/* ------------------------------------------------------------------------
 * G2P of a step fused with the P2G of the next.  Equal, up to the order of the
 * floating-point sums, to
 *     polypic_g2p(grid, P, n_modes, dt, grid_vel, x_in, perm, x_out, coeff_out,
 *                 F_in, F_out, mass_in, mass_out, ...)
 *     polypic_p2g(grid, P, n_modes, x_out, mass_out (or uniform_mass), uniform_mass,
 *                 coeff_out, perm = NULL, ..., grid_mass, grid_mom, accumulate = 0, ...)
 * i.e. the new state's mass and momentum (Eq. 1, 4, 13) are scattered from the
 * coefficients while they are still in registers: the coefficient array is
 * written but not read back (28 + 12 n_modes instead of 40 + 24 n_modes bytes
 * per particle).  Not in the paper: a reordering of its transfers.
 *
 * x_out[3][P] is required (the scatter is at the advected positions);
 * F_in/F_out and mass_in/mass_out are optional pairs as in polypic_g2p; without
 * mass_in every particle has mass uniform_mass.  grid_mass[N] and grid_mom[3][N]
 * are overwritten (cleared first), or with accumulate = 1 added to (the caller
 * cleared them, e.g. with polypic_grid_update_clear).  region_state (optional)
 * is flagged as described under "Active regions".  They, x_out, F_out and
 * mass_out may not overlap grid_vel, x_in, perm, F_in or mass_in; coeff_out may be the
 * coefficient array of the preceding P2G (nothing reads coefficients here).
 * ------------------------------------------------------------------------ */
int32_t polypic_g2p2g(const polypic_grid* grid, int64_t P, int32_t n_modes, float dt,
                      const float* grid_vel, const float* x_in, const int32_t* perm,
                      float* x_out, float* coeff_out, const float* F_in, float* F_out,
                      const float* mass_in, float* mass_out, float uniform_mass,
                      float* grid_mass, float* grid_mom, int32_t accumulate,
                      uint32_t* region_state, int32_t* status_dev, void* stream);

/* ------------------------------------------------------------------------
 * P2G with the affine back-map of Eq. 12 (section 3.3).  The coefficients of a
 * particle were fitted by G2P at an earlier position x_fit, in the basis
 * orthogonalised there; the particle has since moved to x.  Eq. 12 maps the
 * present configuration back to that one, so the modes of Eq. 13 are evaluated at
 *     z'_i = (I + dt C)^-1 (x_i - x_p) / dx,   C_ab = coeff[a][1 + b] / dx
 * (C = 0 below 4 modes), with the quadratic factor of Eq. 14 of the fitting
 * position, ghat(z) = z^2 - a z - 1/4, a = t_fit (1 - 4 t_fit^2), t_fit the
 * offset of x_fit from its nearest node per axis.  The weights W_ip are those of
 * the present position x.  grid_mass is the plain P2G mass (the map does not
 * enter it); grid_mom[a] = sum_p m_p W_ip sum_r c_{p a r} s_r(z'_i).
 *
 * x_fit[3][P] may be NULL (the present offsets are used).  dt is the step that
 * carried x_fit to x.  With dt = 0 and x_fit NULL the result is polypic_p2g's.
 * Other arguments as polypic_p2g (no sorted-cell path; pass the perm of
 * polypic_sort for speed).  A particle with a singular I + dt C raises
 * POLYPIC_FLAG_MAP, one with x or x_fit out of range POLYPIC_FLAG_RANGE; either
 * is skipped.
 * ------------------------------------------------------------------------ */
int32_t polypic_p2g_affine(const polypic_grid* grid, int64_t P, int32_t n_modes, float dt,
                           const float* x, const float* x_fit, const float* mass,
                           float uniform_mass, const float* coeff, const int32_t* perm,
                           float* grid_mass, float* grid_mom, int32_t accumulate,
                           int32_t* status_dev, void* stream);

/* ------------------------------------------------------------------------
 * Liquid and fabric particles on one grid (section 3.4, Eq. 15-20).  One
 * particle array holds both phases, phase[p] = 0 for a fluid particle and 1 for
 * a solid (fabric) point; every node carries a fluid and a solid set of channels:
 *   grid_mass[2][N]   fluid mass m_f,i (Eq. 16's sum of Eq. 1 over fluid
 *                     particles), then the solid mixture mass (m_s + m_f)_i
 *                     (Eq. 18-19 summed over solid points: the point and its
 *                     absorbed fluid);
 *   grid_mom[2][3][N] the momenta of the two sets (Eq. 15-16, 18-19 with the
 *                     polynomial modes of Eq. 13);
 *   grid_vel[2][3][N] the velocities of the two sets.
 * Set k's arrays start at k * N (mass) and k * 3 * N (momentum, velocity).
 *
 * polypic_mixture_p2g: a fluid particle scatters with mass mass_f[p]; a solid
 *   one with mass_s[p] + mass_f[p] (mass_s NULL: 0).  phase and mass_f are
 *   required for P > 0.  A phase other than 0 or 1 raises POLYPIC_FLAG_PHASE and
 *   the particle is skipped.  Other arguments as polypic_p2g (no sorted-cell
 *   path; pass the perm of polypic_sort for speed).
 * polypic_mixture_grid_update: v = p / m + dt g where m > 0, else 0, and the walls
 *   of polypic_grid_update, for each set with its own mass (Eq. 17 and 20, the
 *   latter's mixture mass read as the grid sum).
 * polypic_mixture_g2p: each particle is fitted (as polypic_g2p) from the
 *   velocity of its own phase; phase_out, mass_f_out and mass_s_out (optional,
 *   each paired with its input) receive the per-particle arrays in slot order.
 * ------------------------------------------------------------------------ */
int32_t polypic_mixture_p2g(const polypic_grid* grid, int64_t P, int32_t n_modes,
                            const float* x, const int32_t* phase, const float* mass_f,
                            const float* mass_s, const float* coeff, const int32_t* perm,
                            float* grid_mass, float* grid_mom, int32_t accumulate,
                            int32_t* status_dev, void* stream);
int32_t polypic_mixture_grid_update(const polypic_grid* grid, float dt, const float* gravity,
                                    int32_t bc_layers, const float* grid_mass,
                                    const float* grid_mom, float* grid_vel, void* stream);
int32_t polypic_mixture_g2p(const polypic_grid* grid, int64_t P, int32_t n_modes, float dt,
                            const float* grid_vel, const float* x_in, const int32_t* phase_in,
                            const int32_t* perm, float* x_out, float* coeff_out,
                            const float* F_in, float* F_out, int32_t* phase_out,
                            const float* mass_f_in, float* mass_f_out, const float* mass_s_in,
                            float* mass_s_out, int32_t* status_dev, void* stream);

/* ------------------------------------------------------------------------
 * Staggered (marker-and-cell) grid.  The paper applies its transfers on MAC
 * grids (section 3; Table 1's per-face mass m_{i a}, momentum (mv)_{i a} and
 * velocity v_{i a}): velocity component a lives on the faces of component a,
 * face (ix, iy, iz) of component a at
 *     origin + ((ix, iy, iz) + (1 - e_a) / 2) * dx,
 * i.e. on the node lattice along axis a and half a spacing up along the two
 * other axes.  Each face carries its own mass.  Every component is a scalar
 * transfer on its own lattice with its own quadratic B-spline stencil: along an
 * axis where component a is staggered, u' = u - 1/2 (exact in float32),
 * b = floor(u' - 1/2), t = u' - b - 1.  A particle is in range when the
 * stencils of all three components fit: 0 <= b <= n_axis - 3 for both the
 * node form and the shifted form on every axis (1 <= u < n_axis - 3/2).
 * Modes, coefficient units and the projection are those of the collocated
 * calls, per component over its own stencil.
 *
 * Arrays: face_mass[3][N], face_mom[3][N], face_vel[3][N], component a's faces
 * at a * N + (iz * ny + iy) * nx + ix, N = nx * ny * nz (the grid struct's node
 * counts are the face counts of every component).
 *
 * polypic_mac_p2g: face_mass[a] = sum_p m_p W_{ip a};
 *   face_mom[a] = sum_p m_p W_{ip a} sum_r c_{p r a} s_r (Eq. 1, 4, 13 per face).
 *   Other arguments as polypic_p2g (no sorted-cell path: the workspace-free
 *   brick kernel accumulates runs of equal 4^3 tiles of the particles' node
 *   bases, so pass the perm of polypic_sort for speed; any order is correct).
 * polypic_mac_grid_update: per component, v = p / m + dt g_a where m > 0, else
 *   0 (Eq. 5 per face); walls as polypic_grid_update, on the face index along
 *   the component's own axis.
 * polypic_mac_g2p: c'_{p r a} = <v_a, s_r>_{W_a} / <s_r, s_r>_{W_a} over
 *   component a's face stencil (Eq. 6-8 per face, section 3.3); advection,
 *   clamp, F update and the optional mass copy as polypic_g2p.
 * Out-of-range particles raise POLYPIC_FLAG_RANGE and are skipped (P2G) or get
 *   zero coefficients (G2P).
 * ------------------------------------------------------------------------ */
int32_t polypic_mac_p2g(const polypic_grid* grid, int64_t P, int32_t n_modes, const float* x,
                        const float* mass, float uniform_mass, const float* coeff,
                        const int32_t* perm, float* face_mass, float* face_mom,
                        int32_t accumulate, int32_t* status_dev, void* stream);
int32_t polypic_mac_grid_update(const polypic_grid* grid, float dt, const float* gravity,
                                int32_t bc_layers, const float* face_mass, const float* face_mom,
                                float* face_vel, void* stream);
int32_t polypic_mac_g2p(const polypic_grid* grid, int64_t P, int32_t n_modes, float dt,
                        const float* face_vel, const float* x_in, const int32_t* perm,
                        float* x_out, float* coeff_out, const float* F_in, float* F_out,
                        const float* mass_in, float* mass_out, int32_t* status_dev,
                        void* stream);

/* Launch choice of polypic_g2p2g per mode count:
 *   lane_group: the number of particles of consecutive sorted slots whose node
 *     values are added across lanes before one brick atomic (2, the default, or
 *     4).  The lanes' groups are spread over the workgroup's chunk 8 or 16 slots
 *     apart, so 4 suits about 16 particles per cell.
 *   schedule: the order in which workgroups take the chunks of slots,
 *     POLYPIC_SCHED_LINEAR (the default: in launch order) or POLYPIC_SCHED_XCD
 *     (each XCD takes a contiguous eighth, so that neighbouring chunks, which
 *     gather and scatter the same nodes, share one L2).
 * -1 restores a default.  polypic_autotune_g2p2g runs the call (same arguments
 * and outputs as polypic_g2p2g) once per candidate pair, timed with HIP events on
 * `stream` (one untimed and three timed runs each; it synchronises the stream),
 * keeps the fastest for later calls at this mode count and writes it to
 * *lane_group_out and *schedule_out (either may be NULL); the outputs are those of
 * a final run with the choice.  The choice changes only the order of the grid
 * sums.  (polypic_batch_g2p2g always uses pairs in the XCD order.) */
int32_t polypic_set_g2p2g_config(int32_t n_modes, int32_t lane_group, int32_t schedule);
int32_t polypic_get_g2p2g_config(int32_t n_modes, int32_t* lane_group, int32_t* schedule);
int32_t polypic_autotune_g2p2g(const polypic_grid* grid, int64_t P, int32_t n_modes, float dt,
                               const float* grid_vel, const float* x_in, const int32_t* perm,
                               float* x_out, float* coeff_out, const float* F_in, float* F_out,
                               const float* mass_in, float* mass_out, float uniform_mass,
                               float* grid_mass, float* grid_mom, int32_t* lane_group_out,
                               int32_t* schedule_out, void* stream);

/* ------------------------------------------------------------------------
 * Adjoint (reverse mode) of one step.  For a scalar loss L of the step's
 * outputs, these propagate dL/d(output) to dL/d(input) through the same
 * operations as above, in reverse order:
 *
 *   polypic_g2p_backward(dL/dcoeff_out, dL/dx_out) -> dL/dgrid_vel, += dL/dx_in
 *   polypic_grid_update_backward(dL/dgrid_vel)       -> dL/dgrid_mass, dL/dgrid_mom
 *   polypic_p2g_backward(dL/dgrid_mass, dL/dgrid_mom) -> dL/dcoeff, += dL/dx, dL/dmass
 *
 * Their inputs are the forward inputs of the step (recomputed or kept by the
 * caller -- no weights are stored) and, for the grid update and G2P, the
 * forward grid quantities.  Gradient arrays use the layouts of the forward
 * arrays they belong to.  Derivatives are taken almost everywhere: the stencil
 * base node b is treated as constant (it is piecewise constant in x), a wall
 * clamp or the advection clamp passes zero gradient to the clamped component,
 * empty grid nodes (mass 0) pass none, and the F update is not differentiated.
 * The sort permutation only reorders; pass the perm used in the forward step.
 * Out-of-range particles raise POLYPIC_FLAG_RANGE and get zero gradient.
 *
 * polypic_g2p_backward: coeff_out_grad [3][n_modes][P] and x_out_grad [3][P]
 *   (NULL: no dependence on x_out) are in output-slot order (slot i belongs to
 *   particle perm[i]); grid_vel_grad [3][N] receives dL/dv (zeroed first unless
 *   accumulate); x_in_grad [3][P] is ADDED to at perm[i] (caller zeroes it).
 * polypic_grid_update_backward: writes grid_mass_grad [N], grid_mom_grad [3][N]
 *   from grid_vel_grad and the forward grid_mass / grid_mom.
 * polypic_p2g_backward: writes coeff_grad [3][n_modes][P] and, when not NULL,
 *   mass_grad [P]; ADDS to x_grad [3][P].  perm (NULL allowed) only sets the
 *   processing order.
 * ------------------------------------------------------------------------ */
int32_t polypic_g2p_backward(const polypic_grid* grid, int64_t P, int32_t n_modes, float dt,
                             const float* grid_vel, const float* x_in, const int32_t* perm,
                             const float* coeff_out_grad, const float* x_out_grad,
                             float* grid_vel_grad, int32_t accumulate, float* x_in_grad,
                             int32_t* status_dev, void* stream);
int32_t polypic_grid_update_backward(const polypic_grid* grid, float dt, const float* gravity,
                                     int32_t bc_layers, const float* grid_mass,
                                     const float* grid_mom, const float* grid_vel_grad,
                                     float* grid_mass_grad, float* grid_mom_grad, void* stream);
int32_t polypic_p2g_backward(const polypic_grid* grid, int64_t P, int32_t n_modes, const float* x,
                             const float* mass, float uniform_mass, const float* coeff,
                             const int32_t* perm, const float* grid_mass_grad,
                             const float* grid_mom_grad, float* coeff_grad, float* x_grad,
                             float* mass_grad, int32_t* status_dev, void* stream);

/* ------------------------------------------------------------------------
 * Particle order.  The per-step cell sort (not part of the paper) leaves every particle array
 * in slot order; these move whole arrays between orders on the device.
 *
 * polypic_gather_rows: dst[r][i] = src[r][idx[i]] for r < rows, i < P, with
 *   rows of P 4-byte elements (float32 or int32; the bits are copied).  src and
 *   dst are device arrays of rows * P elements and must not overlap; idx is a
 *   device array of P indices, each clamped into [0, P) (a bad index gives a
 *   wrong element, never an out-of-bounds read).
 *   Returns POLYPIC_EINVAL for a null pointer with rows * P > 0, rows < 0, P
 *   outside [0, 2^31), or overlapping src and dst.
 * polypic_scatter_rows: dst[r][idx[i]] = src[r][i], arguments and errors as
 *   polypic_gather_rows.  With idx a permutation every element of dst is
 *   written once; otherwise repeated indices race (one of the values is kept)
 *   and elements no index names keep their previous values.
 * polypic_invert_permutation: inv[perm[i]] = i for i < P (device arrays of P
 *   int32, not overlapping).  perm must be a permutation of [0, P): entries
 *   outside that range are clamped into it, and an entry of inv that no perm
 *   entry names keeps its previous value.
 * All three run asynchronously on `stream`. */
int32_t polypic_gather_rows(const void* src, void* dst, const int32_t* idx, int64_t rows,
                            int64_t P, void* stream);
int32_t polypic_scatter_rows(const void* src, void* dst, const int32_t* idx, int64_t rows,
                             int64_t P, void* stream);
int32_t polypic_invert_permutation(const int32_t* perm, int32_t* inv, int64_t P, void* stream);

/* ------------------------------------------------------------------------
 * Batches of independent scenes (not in the paper: many small simulations
 * stepped together).  Every scene has its own grid and particles; the
 * particle arrays of all scenes are laid end to end (flattened index), and so
 * are the grid arrays.  One call runs one step phase for every scene with a
 * single launch (or a fixed sequence of launches for the sort), so a whole
 * step can be captured once in a HIP graph and replayed.
 *
 * polypic_scene (host): scene s owns particles [p_offset, p_offset +
 *   n_particles) of every particle array and nodes [node_offset, node_offset
 *   + nx*ny*nz) of every grid channel.  Particle ranges must be contiguous
 *   and in scene order starting at 0 (empty scenes allowed); node ranges in
 *   scene order, not overlapping, inside [0, n_nodes_total).
 * Layouts: x[3][P], coeff[3][n_modes][P], mass[P], F[9][P] with P the total
 *   particle count; grid_mass[N], grid_mom[3][N], grid_vel[3][N] with
 *   N = n_nodes_total.
 *
 * polypic_batch_plan validates the scenes, writes the device scene table
 *   into table_dev (caller-owned device memory of polypic_batch_table_bytes()
 *   bytes, which must outlive every call that uses the batch) and fills the
 *   host descriptor *batch.  It copies synchronously (the scenes array may
 *   be freed on return) and must not be called during graph capture.  The
 *   descriptor is sealed: a batch call whose descriptor was modified after
 *   planning returns POLYPIC_EINVAL.
 * polypic_batch_sort: keys = scene << morton_bits | Morton(base node), sorted
 *   stably over all P (so every particle stays inside its scene's range, in
 *   cell order).  Workspace: polypic_batch_sort_workspace_bytes().
 *   Returns POLYPIC_ENOTSUP if the scene index and the largest grid's Morton
 *   code do not fit in 32 key bits.
 * polypic_batch_p2g / _grid_update / _g2p: as polypic_p2g (brick path) /
 *   polypic_grid_update / polypic_g2p, per scene, with the batch layouts.
 *   perm (optional) must keep every particle inside its scene's range, as
 *   the batched sort's does; slot i is processed with the grid of the scene
 *   whose range holds i.
 * polypic_batch_set_config / _get_config / _autotune: block, schedule, per_cu
 *   and brick edge of the batched P2G (same meaning as for polypic_p2g; default
 *   block 256, POLYPIC_SCHED_XCD, 4^3 bricks), per n_modes, process-wide.  The
 *   autotuner times every candidate on the given inputs and SYNCHRONISES the
 *   stream.
 * ------------------------------------------------------------------------ */
typedef struct polypic_scene {
  polypic_grid grid;
  int64_t p_offset;
  int64_t n_particles;
  int64_t node_offset;
} polypic_scene;

typedef struct polypic_batch {
  int32_t n_scenes;
  int32_t key_bits;    /* bits of the batched sort keys */
  int32_t morton_bits; /* Morton bits below the scene index */
  int32_t max_nodes;   /* largest scene node count */
  int64_t P;           /* total particles */
  int64_t N;           /* total nodes per grid channel */
  int64_t n_regions;   /* active regions of all scenes */
  const void* table;   /* device scene table (in the caller's buffer) */
  uint64_t seal;       /* written by polypic_batch_plan */
} polypic_batch;

int32_t polypic_batch_table_bytes(int32_t n_scenes, size_t* bytes);
int32_t polypic_batch_plan(const polypic_scene* scenes, int32_t n_scenes, int64_t n_nodes_total,
                           void* table_dev, size_t table_bytes, polypic_batch* batch,
                           void* stream);
int32_t polypic_batch_sort_workspace_bytes(const polypic_batch* batch, size_t* bytes);
int32_t polypic_batch_sort(const polypic_batch* batch, const float* x, uint32_t* keys_out,
                           int32_t* perm_out, void* ws, size_t ws_bytes, int32_t* status_dev,
                           void* stream);
/* polypic_batch_sort_update: polypic_sort_update over the batch -- the same keys and
 * permutation as polypic_batch_sort, bit for bit, from the previous batched sort's
 * keys (keys_prev[i]: the key slot i was sorted under; ascending).  Flags, aliasing
 * and workspace rules as polypic_sort_update. */
int32_t polypic_batch_sort_update_workspace_bytes(const polypic_batch* batch, size_t* bytes);
int32_t polypic_batch_sort_update(const polypic_batch* batch, const float* x,
                                  const uint32_t* keys_prev, uint32_t* keys_out,
                                  int32_t* perm_out, void* ws, size_t ws_bytes,
                                  int32_t* status_dev, void* stream);
int32_t polypic_batch_p2g(const polypic_batch* batch, int32_t n_modes, const float* x,
                          const float* mass, float uniform_mass, const float* coeff,
                          const int32_t* perm, float* grid_mass, float* grid_mom,
                          int32_t accumulate, int32_t* status_dev, void* stream);
int32_t polypic_batch_grid_update(const polypic_batch* batch, float dt, const float* gravity,
                                  int32_t bc_layers, const float* grid_mass,
                                  const float* grid_mom, float* grid_vel, void* stream);
int32_t polypic_batch_g2p(const polypic_batch* batch, int32_t n_modes, float dt,
                          const float* grid_vel, const float* x_in, const int32_t* perm,
                          float* x_out, float* coeff_out, const float* F_in, float* F_out,
                          const float* mass_in, float* mass_out, int32_t* status_dev,
                          void* stream);
/* polypic_batch_g2p2g: polypic_g2p2g over every scene of the batch (each scene's
 * G2P, advection and next P2G on its own grid; grid_mass / grid_mom span batch->N
 * nodes and are cleared first unless accumulate = 1).  Arguments as
 * polypic_batch_g2p plus uniform_mass, grid_mass, grid_mom, accumulate and
 * region_state (batch->n_regions flags: the regions of the scenes in order,
 * each scene's numbered as for its grid alone), with the rules of
 * polypic_g2p2g. */
int32_t polypic_batch_g2p2g(const polypic_batch* batch, int32_t n_modes, float dt,
                            const float* grid_vel, const float* x_in, const int32_t* perm,
                            float* x_out, float* coeff_out, const float* F_in, float* F_out,
                            const float* mass_in, float* mass_out, float uniform_mass,
                            float* grid_mass, float* grid_mom, int32_t accumulate,
                            uint32_t* region_state, int32_t* status_dev, void* stream);
/* polypic_batch_grid_update_active: polypic_grid_update_active over every scene of
 * the batch, with the batch layouts. */
int32_t polypic_batch_grid_update_active(const polypic_batch* batch, float dt,
                                         const float* gravity, int32_t bc_layers,
                                         float* grid_mass, float* grid_mom, float* grid_vel,
                                         uint32_t* region_state, void* stream);
int32_t polypic_batch_set_config(int32_t n_modes, int32_t block, int32_t schedule,
                                 int32_t per_cu, int32_t brick);
int32_t polypic_batch_get_config(int32_t n_modes, int32_t* block, int32_t* schedule,
                                 int32_t* per_cu, int32_t* brick);
int32_t polypic_batch_autotune(const polypic_batch* batch, int32_t n_modes, const float* x,
                               const float* mass, float uniform_mass, const float* coeff,
                               const int32_t* perm, float* grid_mass, float* grid_mom,
                               int32_t* block_out, int32_t* schedule_out, int32_t* per_cu_out,
                               int32_t* brick_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* POLYPIC_H */
