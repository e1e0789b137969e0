// C ABI layer: argument validation, launch configuration and dispatch.
// Every entry point only enqueues work on the caller's stream.
#include <math.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "polypic.h"
#include "polypic_internal.hpp"

using namespace polypic;

namespace {

constexpr int32_t kVersion = 100;  // 0.1.0

bool valid_modes(int32_t n) { return n == 1 || n == 4 || n == 8 || n == 27; }

// [a, a + na) and [b, b + nb) floats overlap (either may be null)
bool overlaps(const void* a, int64_t na, const void* b, int64_t nb) {
  if (!a || !b) return false;
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb * 4 && pb < pa + na * 4;
}

int32_t check_grid(const polypic_grid* g) {
  if (!g) return POLYPIC_EINVAL;
  const int32_t d[3] = {g->nx, g->ny, g->nz};
  for (int a = 0; a < 3; ++a) {
    if (d[a] < 3) return POLYPIC_EINVAL;
    if (d[a] > 1026) return POLYPIC_ENOTSUP;  // 10-bit base node per axis in the keys
  }
  if (!(g->dx > 0.0f) || !isfinite(g->dx) || !(g->inv_dx > 0.0f) || !isfinite(g->inv_dx))
    return POLYPIC_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (!isfinite(g->origin[a])) return POLYPIC_EINVAL;
  return POLYPIC_OK;
}

GridDev to_dev(const polypic_grid* g) {
  GridDev d;
  d.nx = g->nx;
  d.ny = g->ny;
  d.nz = g->nz;
  d.inv_dx = g->inv_dx;
  d.ox = g->origin[0];
  d.oy = g->origin[1];
  d.oz = g->origin[2];
  return d;
}

int32_t check_P(int64_t P) {
  if (P < 0 || P > (int64_t)INT32_MAX) return POLYPIC_EINVAL;
  return POLYPIC_OK;
}

// Name of the last HIP error an entry point of this thread reported as EDEVICE.
thread_local const char* g_last_device_error = "no error";

int32_t from_hip(hipError_t e) {
  if (e == hipSuccess) return POLYPIC_OK;
  g_last_device_error = hipGetErrorName(e);
  return POLYPIC_EDEVICE;
}

// HIP keeps a per-thread "last error" that any runtime call may set (including
// calls made by other libraries in the process).  Entry points discard it before
// launching so that the status they return describes their own launches only.
void discard_stale_error() { (void)hipGetLastError(); }

int64_t n_nodes(const polypic_grid* g) { return (int64_t)g->nx * g->ny * g->nz; }

// Advection clamp bounds [origin + 2 dx, origin + (n - 2) dx): the lower bound and
// the largest float below the upper one, both rounded from double.
void clamp_bounds(const polypic_grid* grid, float lo[3], float hi[3]) {
  const int32_t d[3] = {grid->nx, grid->ny, grid->nz};
  for (int ax = 0; ax < 3; ++ax) {
    lo[ax] = (float)((double)grid->origin[ax] + 2.0 * (double)grid->dx);
    const float top = (float)((double)grid->origin[ax] + (double)(d[ax] - 2) * (double)grid->dx);
    hi[ax] = nextafterf(top, -INFINITY);
  }
}

// ---- P2G launch-configuration table (per n_modes), shared by the process
struct P2GChoice {
  int path = POLYPIC_P2G_DEFAULT;
  int block = 256;
  int sched = POLYPIC_SCHED_LINEAR;
  int per_cu = 0;
  int brick = 4;  // brick edge in cells: 2, 4 or 8
};

bool valid_brick(int32_t brick) { return brick == 2 || brick == 4 || brick == 8; }
int brick_log2(int brick) { return brick == 2 ? 1 : brick == 8 ? 3 : 2; }

bool valid_schedule(int32_t schedule, int32_t per_cu) {
  if (schedule == POLYPIC_SCHED_LINEAR || schedule == POLYPIC_SCHED_XCD) return true;
  return schedule == POLYPIC_SCHED_PERSISTENT && per_cu >= 1 && per_cu <= 64;
}

P2GConfig to_config(const P2GChoice& c) {
  P2GConfig cfg = p2g_default_config();
  cfg.block = c.block;
  cfg.sched = c.sched == POLYPIC_SCHED_XCD          ? kSchedXcd
              : c.sched == POLYPIC_SCHED_PERSISTENT ? kSchedPersistent
                                                    : kSchedLinear;
  cfg.persist_per_cu = c.sched == POLYPIC_SCHED_PERSISTENT ? c.per_cu : 0;
  cfg.tile_log2 = brick_log2(c.brick);
  return cfg;
}

std::atomic<int> g_g2p_sched{POLYPIC_SCHED_LINEAR};
// lane-group size of the fused G2P2G kernel per mode count (0: the default, pairs)
std::atomic<int> g_fused_lane[28];
std::atomic<int> g_fused_sched[28];  // POLYPIC_SCHED_LINEAR (the default) or _XCD

int fused_lane_group(int n_modes) {
  const int v = g_fused_lane[n_modes].load();
  return v == 4 ? 4 : 2;
}
int fused_sched(int n_modes) {
  return g_fused_sched[n_modes].load() == POLYPIC_SCHED_XCD ? kSchedXcd : kSchedLinear;
}
std::mutex g_tune_mutex;
P2GChoice g_tune[28];

P2GChoice get_choice(int n_modes) {
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  return g_tune[n_modes];
}

void set_choice(int n_modes, P2GChoice c) {
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  g_tune[n_modes] = c;
}

// Enqueue one P2G with an explicit configuration (arguments already validated).
int32_t run_p2g(const polypic_grid* grid, int64_t P, int32_t n_modes, const float* x,
                const float* mass, float uniform_mass, const float* coeff, const int32_t* perm,
                const uint32_t* keys_sorted, void* ws, float* grid_mass, float* grid_mom,
                int32_t accumulate, int32_t* status_dev, hipStream_t s, P2GChoice c) {
  int32_t st;
  const int64_t N = n_nodes(grid);
  const bool cells = keys_sorted != nullptr && c.path == POLYPIC_P2G_CELLS;
  uint32_t* counter = cells ? (uint32_t*)ws : nullptr;
  if (!accumulate) {
    if ((st = from_hip(launch_grid_clear(grid_mass, grid_mom, N, counter, s)))) return st;
  }
  P2GArgs a;
  a.g = to_dev(grid);
  a.P = P;
  a.x = x;
  a.mass = mass;
  a.uniform_mass = uniform_mass;
  a.coeff = coeff;
  a.perm = perm;
  a.gm = grid_mass;
  a.gp0 = grid_mom;
  a.gp1 = grid_mom + N;
  a.gp2 = grid_mom + 2 * N;
  a.status = status_dev;
  a.keys = keys_sorted;
  a.tile_list = nullptr;
  a.tile_count = nullptr;
  a.sched = kSchedLinear;
  if (cells) return from_hip(launch_p2g_sorted(a, n_modes, ws, !accumulate, s));
  return from_hip(launch_p2g(a, n_modes, to_config(c), s));
}


// Times `run(k)` for every candidate k < n on stream s: one untimed run, then
// the median of three timed ones (HIP events).  Synchronises s.  Writes the
// fastest candidate to *best.
template <class Run>
int32_t time_candidates(int n, hipStream_t s, Run run, int* best) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return POLYPIC_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return POLYPIC_EDEVICE;
  }
  int32_t st = POLYPIC_OK;
  float best_ms = -1.0f;
  constexpr int kReps = 3;
  for (int k = 0; k < n && st == POLYPIC_OK; ++k) {
    float t[kReps];
    for (int rep = -1; rep < kReps && st == POLYPIC_OK; ++rep) {
      if (rep >= 0 && hipEventRecord(e0, s) != hipSuccess) st = POLYPIC_EDEVICE;
      if (!st) st = run(k);
      if (!st && rep >= 0) {
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t[rep], e0, e1) != hipSuccess)
          st = POLYPIC_EDEVICE;
      }
    }
    if (st) break;
    std::sort(t, t + kReps);
    if (best_ms < 0.0f || t[kReps / 2] < best_ms) {
      best_ms = t[kReps / 2];
      *best = k;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st) return st;
  if (hipStreamSynchronize(s) != hipSuccess) return POLYPIC_EDEVICE;
  return POLYPIC_OK;
}

// ---- batches of scenes
constexpr int32_t kMaxScenes = 65536;

uint64_t batch_seal(const polypic_batch* b) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the descriptor's fields
  auto mix = [&h](uint64_t v) {
    for (int k = 0; k < 8; ++k) {
      h ^= (v >> (8 * k)) & 0xffu;
      h *= 1099511628211ull;
    }
  };
  mix((uint32_t)b->n_scenes);
  mix((uint32_t)b->key_bits);
  mix((uint32_t)b->morton_bits);
  mix((uint32_t)b->max_nodes);
  mix((uint64_t)b->P);
  mix((uint64_t)b->N);
  mix((uint64_t)b->n_regions);
  mix((uint64_t)(uintptr_t)b->table);
  return h;
}

int32_t check_batch(const polypic_batch* b) {
  if (!b || !b->table || b->n_scenes < 1 || b->n_scenes > kMaxScenes) return POLYPIC_EINVAL;
  if (b->seal != batch_seal(b)) return POLYPIC_EINVAL;
  return POLYPIC_OK;
}

const SceneDev* batch_table(const polypic_batch* b) { return (const SceneDev*)b->table; }

struct BatchChoice {
  int block = 256;
  int sched = POLYPIC_SCHED_XCD;
  int per_cu = 0;
  int brick = 4;
};
BatchChoice g_btune[28];

BatchChoice get_bchoice(int n_modes) {
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  return g_btune[n_modes];
}

void set_bchoice(int n_modes, BatchChoice c) {
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  g_btune[n_modes] = c;
}

int32_t run_batch_p2g(const polypic_batch* b, int32_t n_modes, const float* x, const float* mass,
                      float uniform_mass, const float* coeff, const int32_t* perm,
                      float* grid_mass, float* grid_mom, int32_t accumulate, int32_t* status_dev,
                      hipStream_t s, const BatchChoice& c) {
  int32_t st;
  if (!accumulate) {
    if ((st = from_hip(launch_grid_clear(grid_mass, grid_mom, b->N, nullptr, s)))) return st;
  }
  P2GArgs a;
  a.g = GridDev{3, 3, 3, 1.0f, 0.0f, 0.0f, 0.0f};  // unused: every slot reads its scene's grid
  a.P = b->P;
  a.x = x;
  a.mass = mass;
  a.uniform_mass = uniform_mass;
  a.coeff = coeff;
  a.perm = perm;
  a.gm = grid_mass;
  a.gp0 = grid_mom;
  a.gp1 = grid_mom + b->N;
  a.gp2 = grid_mom + 2 * b->N;
  a.status = status_dev;
  a.keys = nullptr;
  a.tile_list = nullptr;
  a.tile_count = nullptr;
  a.sched = kSchedLinear;
  P2GChoice pc;
  pc.block = c.block;
  pc.sched = c.sched;
  pc.per_cu = c.per_cu;
  pc.brick = c.brick;
  return from_hip(
      launch_p2g_batch(a, batch_table(b), b->n_scenes, n_modes, to_config(pc), s));
}

// ---- allocation-free sort: the workspace lives in a file-scope device array
//
// Each GPU the library runs on holds its own copy of `scratch` from module load
// to the end of the process.  In host code the array's name is not a device
// address: its address on the current device is looked up once per device with
// hipGetSymbolAddress and only that pointer is handed to kernels.
constexpr int64_t kNoAllocMaxP = 2097152;               // particles per call
constexpr size_t kScratchBytes = (size_t)18 << 20;      // 18 MiB >= sort workspace of kNoAllocMaxP
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's scratch (looked up on the first call on the device).
hipError_t scratch_on_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

const char* polypic_strerror(int32_t code) {
  switch (code) {
    case POLYPIC_OK: return "ok";
    case POLYPIC_EINVAL: return "invalid argument";
    case POLYPIC_ERANGE: return "value out of range";
    case POLYPIC_EDEVICE: return "HIP device error";
    case POLYPIC_ENOSPACE: return "workspace too small";
    case POLYPIC_ENOTSUP: return "not supported";
    default: return "unknown status code";
  }
}

int32_t polypic_version(void) { return kVersion; }

const char* polypic_last_device_error(void) { return g_last_device_error; }

int32_t polypic_sort_workspace_bytes(const polypic_grid* grid, int64_t P, size_t* bytes) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (!bytes) return POLYPIC_EINVAL;
  *bytes = sort_workspace_bytes(P);
  return POLYPIC_OK;
}

int32_t polypic_sort(const polypic_grid* grid, int64_t P, const float* x, uint32_t* keys_out,
                     int32_t* perm_out, void* ws, size_t ws_bytes, int32_t* status_dev,
                     void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (P == 0) return POLYPIC_OK;
  if (!x || !keys_out || !perm_out || !ws) return POLYPIC_EINVAL;
  if (ws_bytes < sort_workspace_bytes(P)) return POLYPIC_ENOSPACE;
  discard_stale_error();
  return from_hip(launch_sort(to_dev(grid), P, x, keys_out, perm_out, ws, status_dev,
                              (hipStream_t)stream));
}

int32_t polypic_sort_noalloc(const polypic_grid* grid, int64_t P, const float* x,
                             uint32_t* keys_out, int32_t* perm_out, int32_t* status_dev,
                             void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (P > kNoAllocMaxP || sort_workspace_bytes(P) > kScratchBytes) return POLYPIC_ENOSPACE;
  if (P == 0) return POLYPIC_OK;
  if (!x || !keys_out || !perm_out) return POLYPIC_EINVAL;
  discard_stale_error();
  void* ws = nullptr;
  hipError_t e = scratch_on_current_device(&ws);
  if (e != hipSuccess) return from_hip(e);
  // every word of the workspace that the sort reads it has written first in the same
  // call (keys, indices, tile counts, digit totals): nothing needs clearing
  return from_hip(launch_sort(to_dev(grid), P, x, keys_out, perm_out, ws, status_dev,
                              (hipStream_t)stream));
}

int32_t polypic_sort_update_workspace_bytes(const polypic_grid* grid, int64_t P, size_t* bytes) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (!bytes) return POLYPIC_EINVAL;
  *bytes = sort_update_workspace_bytes(P);
  return POLYPIC_OK;
}

int32_t polypic_sort_update(const polypic_grid* grid, int64_t P, const float* x,
                            const uint32_t* keys_prev, uint32_t* keys_out, int32_t* perm_out,
                            void* ws, size_t ws_bytes, int32_t* status_dev, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (P == 0) return POLYPIC_OK;
  if (!x || !keys_prev || !keys_out || !perm_out || !ws) return POLYPIC_EINVAL;
  if ((const void*)keys_prev == (const void*)keys_out) return POLYPIC_EINVAL;
  if (ws_bytes < sort_update_workspace_bytes(P)) return POLYPIC_ENOSPACE;
  discard_stale_error();
  return from_hip(launch_sort_update(to_dev(grid), P, x, keys_prev, keys_out, perm_out, ws,
                                     status_dev, (hipStream_t)stream));
}

int32_t polypic_p2g_workspace_bytes(const polypic_grid* grid, int64_t P, size_t* bytes) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (!bytes) return POLYPIC_EINVAL;
  *bytes = p2g_workspace_bytes(to_dev(grid), P);
  return POLYPIC_OK;
}

int32_t polypic_p2g(const polypic_grid* grid, int64_t P, int32_t n_modes, const float* x,
                    const float* mass, float uniform_mass, const float* coeff, const int32_t* perm,
                    const uint32_t* keys_sorted, void* ws, size_t ws_bytes, float* grid_mass,
                    float* grid_mom, int32_t accumulate, int32_t* status_dev, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (!valid_modes(n_modes)) return POLYPIC_EINVAL;
  if (!grid_mass || !grid_mom) return POLYPIC_EINVAL;
  if (P > 0 && (!x || !coeff)) return POLYPIC_EINVAL;
  if (!mass && !isfinite(uniform_mass)) return POLYPIC_EINVAL;
  const bool sorted = keys_sorted != nullptr;
  if (sorted) {
    if (!perm || !ws) return POLYPIC_EINVAL;
    if (ws_bytes < p2g_workspace_bytes(to_dev(grid), P)) return POLYPIC_ENOSPACE;
  }
  discard_stale_error();
  return run_p2g(grid, P, n_modes, x, mass, uniform_mass, coeff, perm, keys_sorted, ws, grid_mass,
                 grid_mom, accumulate, status_dev, (hipStream_t)stream, get_choice(n_modes));
}

int32_t polypic_set_p2g_config(int32_t n_modes, int32_t path, int32_t block, int32_t schedule,
                               int32_t per_cu, int32_t brick) {
  if (!valid_modes(n_modes)) return POLYPIC_EINVAL;
  if (path != POLYPIC_P2G_DEFAULT && path != POLYPIC_P2G_BRICKS && path != POLYPIC_P2G_CELLS)
    return POLYPIC_EINVAL;
  if (block != 256 && block != 512) return POLYPIC_EINVAL;
  if (!valid_schedule(schedule, per_cu)) return POLYPIC_EINVAL;
  if (!valid_brick(brick)) return POLYPIC_EINVAL;
  P2GChoice c;
  c.path = path;
  c.block = block;
  c.sched = schedule;
  c.per_cu = schedule == POLYPIC_SCHED_PERSISTENT ? per_cu : 0;
  c.brick = brick;
  set_choice(n_modes, c);
  return POLYPIC_OK;
}

int32_t polypic_get_p2g_config(int32_t n_modes, int32_t* path, int32_t* block, int32_t* schedule,
                               int32_t* per_cu, int32_t* brick) {
  if (!valid_modes(n_modes)) return POLYPIC_EINVAL;
  const P2GChoice c = get_choice(n_modes);
  if (path) *path = c.path;
  if (block) *block = c.block;
  if (schedule) *schedule = c.sched;
  if (per_cu) *per_cu = c.per_cu;
  if (brick) *brick = c.brick;
  return POLYPIC_OK;
}

int32_t polypic_set_g2p_schedule(int32_t schedule) {
  if (schedule != POLYPIC_SCHED_LINEAR && schedule != POLYPIC_SCHED_XCD) return POLYPIC_EINVAL;
  g_g2p_sched.store(schedule);
  return POLYPIC_OK;
}

int32_t polypic_get_g2p_schedule(int32_t* schedule) {
  if (!schedule) return POLYPIC_EINVAL;
  *schedule = g_g2p_sched.load();
  return POLYPIC_OK;
}

int32_t polypic_autotune_p2g(const polypic_grid* grid, int64_t P, int32_t n_modes, const float* x,
                             const float* mass, float uniform_mass, const float* coeff,
                             const int32_t* perm, const uint32_t* keys_sorted, void* ws,
                             size_t ws_bytes, float* grid_mass, float* grid_mom,
                             int32_t* path_out, int32_t* block_out, int32_t* schedule_out,
                             int32_t* per_cu_out, int32_t* brick_out, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (!valid_modes(n_modes)) return POLYPIC_EINVAL;
  if (!grid_mass || !grid_mom) return POLYPIC_EINVAL;
  if (P > 0 && (!x || !coeff)) return POLYPIC_EINVAL;
  if (!mass && !isfinite(uniform_mass)) return POLYPIC_EINVAL;
  if (keys_sorted) {
    if (!perm || !ws) return POLYPIC_EINVAL;
    if (ws_bytes < p2g_workspace_bytes(to_dev(grid), P)) return POLYPIC_ENOSPACE;
  }
  const hipStream_t s = (hipStream_t)stream;
  std::vector<P2GChoice> cand;
  for (int brick : {4, 2, 8})
    for (int block : {256, 512})
      for (int sched : {POLYPIC_SCHED_LINEAR, POLYPIC_SCHED_XCD}) {
        P2GChoice c;
        c.path = POLYPIC_P2G_BRICKS;
        c.block = block;
        c.sched = sched;
        c.brick = brick;
        cand.push_back(c);
      }
  if (keys_sorted) {
    P2GChoice c;
    c.path = POLYPIC_P2G_CELLS;
    cand.push_back(c);
  }
  discard_stale_error();
  int bi = 0;
  st = time_candidates(
      (int)cand.size(), s,
      [&](int k) {
        return run_p2g(grid, P, n_modes, x, mass, uniform_mass, coeff, perm, keys_sorted, ws,
                       grid_mass, grid_mom, 0, nullptr, s, cand[k]);
      },
      &bi);
  if (st) return st;
  const P2GChoice best = cand[bi];
  set_choice(n_modes, best);
  if (path_out) *path_out = best.path;
  if (block_out) *block_out = best.block;
  if (schedule_out) *schedule_out = best.sched;
  if (per_cu_out) *per_cu_out = best.per_cu;
  if (brick_out) *brick_out = best.brick;
  return POLYPIC_OK;
}

int32_t polypic_grid_update(const polypic_grid* grid, float dt, const float* gravity,
                            int32_t bc_layers, const float* grid_mass, const float* grid_mom,
                            float* grid_vel, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if (!gravity || !grid_mass || !grid_mom || !grid_vel) return POLYPIC_EINVAL;
  if (!isfinite(dt) || bc_layers < 0) return POLYPIC_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (!isfinite(gravity[a])) return POLYPIC_EINVAL;
  GridUpdateArgs a;
  a.nx = grid->nx;
  a.ny = grid->ny;
  a.nz = grid->nz;
  a.dt = dt;
  a.g0 = gravity[0];
  a.g1 = gravity[1];
  a.g2 = gravity[2];
  a.bc_layers = bc_layers;
  a.gm = grid_mass;
  a.gp = grid_mom;
  a.gv = grid_vel;
  a.clear_gm = nullptr;
  a.clear_gp = nullptr;
  a.regions = nullptr;
  a.n_regions = 0;
  discard_stale_error();
  return from_hip(launch_grid_update(a, (hipStream_t)stream));
}

int32_t polypic_grid_update_clear(const polypic_grid* grid, float dt, const float* gravity,
                                  int32_t bc_layers, float* grid_mass, float* grid_mom,
                                  float* grid_vel, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if (!gravity || !grid_mass || !grid_mom || !grid_vel) return POLYPIC_EINVAL;
  if (!isfinite(dt) || bc_layers < 0) return POLYPIC_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (!isfinite(gravity[k])) return POLYPIC_EINVAL;
  const int64_t N = n_nodes(grid);
  if (overlaps(grid_vel, 3 * N, grid_mass, N) || overlaps(grid_vel, 3 * N, grid_mom, 3 * N))
    return POLYPIC_EINVAL;
  GridUpdateArgs a;
  a.nx = grid->nx;
  a.ny = grid->ny;
  a.nz = grid->nz;
  a.dt = dt;
  a.g0 = gravity[0];
  a.g1 = gravity[1];
  a.g2 = gravity[2];
  a.bc_layers = bc_layers;
  a.gm = grid_mass;
  a.gp = grid_mom;
  a.gv = grid_vel;
  a.clear_gm = grid_mass;
  a.clear_gp = grid_mom;
  a.regions = nullptr;
  a.n_regions = 0;
  discard_stale_error();
  return from_hip(launch_grid_update(a, (hipStream_t)stream));
}

int32_t polypic_region_count(const polypic_grid* grid, int64_t* count) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if (!count) return POLYPIC_EINVAL;
  *count = region_count(grid->nx, grid->ny, grid->nz);
  return POLYPIC_OK;
}

int32_t polypic_grid_update_active(const polypic_grid* grid, float dt, const float* gravity,
                                   int32_t bc_layers, float* grid_mass, float* grid_mom,
                                   float* grid_vel, uint32_t* region_state, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if (!gravity || !grid_mass || !grid_mom || !grid_vel || !region_state) return POLYPIC_EINVAL;
  if (!isfinite(dt) || bc_layers < 0) return POLYPIC_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (!isfinite(gravity[k])) return POLYPIC_EINVAL;
  const int64_t N = n_nodes(grid);
  if (overlaps(grid_vel, 3 * N, grid_mass, N) || overlaps(grid_vel, 3 * N, grid_mom, 3 * N))
    return POLYPIC_EINVAL;
  GridUpdateArgs a;
  a.nx = grid->nx;
  a.ny = grid->ny;
  a.nz = grid->nz;
  a.dt = dt;
  a.g0 = gravity[0];
  a.g1 = gravity[1];
  a.g2 = gravity[2];
  a.bc_layers = bc_layers;
  a.gm = grid_mass;
  a.gp = grid_mom;
  a.gv = grid_vel;
  a.clear_gm = grid_mass;
  a.clear_gp = grid_mom;
  a.regions = region_state;
  a.n_regions = region_count(grid->nx, grid->ny, grid->nz);
  discard_stale_error();
  return from_hip(launch_grid_update_active(a, (hipStream_t)stream));
}

int32_t polypic_g2p(const polypic_grid* grid, int64_t P, int32_t n_modes, float dt,
                    const float* grid_vel, const float* x_in, const int32_t* perm, float* x_out,
                    float* coeff_out, const float* F_in, float* F_out, const float* mass_in,
                    float* mass_out, int32_t* status_dev, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (!valid_modes(n_modes) || !isfinite(dt)) return POLYPIC_EINVAL;
  if (P == 0) return POLYPIC_OK;
  if (!grid_vel || !x_in || !coeff_out) return POLYPIC_EINVAL;
  if ((F_in == nullptr) != (F_out == nullptr)) return POLYPIC_EINVAL;
  if ((mass_in == nullptr) != (mass_out == nullptr)) return POLYPIC_EINVAL;
  G2PArgs a;
  a.g = to_dev(grid);
  a.P = P;
  a.dt = dt;
  a.dx = grid->dx;
  clamp_bounds(grid, a.lo, a.hi);
  a.gv = grid_vel;
  a.x_in = x_in;
  a.perm = perm;
  a.x_out = x_out;
  a.coeff_out = coeff_out;
  a.F_in = F_in;
  a.F_out = F_out;
  a.mass_in = mass_in;
  a.mass_out = mass_out;
  a.status = status_dev;
  a.gstride = n_nodes(grid);
  a.sched = g_g2p_sched.load() == POLYPIC_SCHED_XCD ? kSchedXcd : kSchedLinear;
  discard_stale_error();
  return from_hip(launch_g2p(a, n_modes, (hipStream_t)stream));
}

// ---- P2G with the affine back-map of Eq. 12
int32_t polypic_p2g_affine(const polypic_grid* grid, int64_t P, int32_t n_modes, float dt,
                           const float* x, const float* x_fit, const float* mass,
                           float uniform_mass, const float* coeff, const int32_t* perm,
                           float* grid_mass, float* grid_mom, int32_t accumulate,
                           int32_t* status_dev, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (!valid_modes(n_modes) || !isfinite(dt)) return POLYPIC_EINVAL;
  if (!grid_mass || !grid_mom) return POLYPIC_EINVAL;
  if (P > 0 && (!x || !coeff)) return POLYPIC_EINVAL;
  if (!mass && !isfinite(uniform_mass)) return POLYPIC_EINVAL;
  AffineP2GArgs a;
  a.g = to_dev(grid);
  a.P = P;
  a.dt = dt;
  a.x = x;
  a.x_fit = x_fit;
  a.mass = mass;
  a.uniform_mass = uniform_mass;
  a.coeff = coeff;
  a.perm = perm;
  a.gm = grid_mass;
  a.gp = grid_mom;
  a.status = status_dev;
  discard_stale_error();
  return from_hip(launch_p2g_affine(a, n_modes, accumulate != 0, (hipStream_t)stream));
}

// ---- liquid and fabric particles on one grid
int32_t polypic_mixture_p2g(const polypic_grid* grid, int64_t P, int32_t n_modes,
                            const float* x, const int32_t* phase, const float* mass_f,
                            const float* mass_s, const float* coeff, const int32_t* perm,
                            float* grid_mass, float* grid_mom, int32_t accumulate,
                            int32_t* status_dev, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (!valid_modes(n_modes)) return POLYPIC_EINVAL;
  if (!grid_mass || !grid_mom) return POLYPIC_EINVAL;
  if (P > 0 && (!x || !coeff || !phase || !mass_f)) return POLYPIC_EINVAL;
  MixtureP2GArgs a;
  a.g = to_dev(grid);
  a.P = P;
  a.x = x;
  a.phase = phase;
  a.mass_f = mass_f;
  a.mass_s = mass_s;
  a.coeff = coeff;
  a.perm = perm;
  a.gm = grid_mass;
  a.gp = grid_mom;
  a.status = status_dev;
  discard_stale_error();
  return from_hip(launch_mixture_p2g(a, n_modes, accumulate != 0, (hipStream_t)stream));
}

int32_t polypic_mixture_grid_update(const polypic_grid* grid, float dt, const float* gravity,
                                    int32_t bc_layers, const float* grid_mass,
                                    const float* grid_mom, float* grid_vel, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if (!gravity || !grid_mass || !grid_mom || !grid_vel) return POLYPIC_EINVAL;
  if (!isfinite(dt) || bc_layers < 0) return POLYPIC_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (!isfinite(gravity[k])) return POLYPIC_EINVAL;
  const size_t N = (size_t)n_nodes(grid);
  discard_stale_error();
  for (int ph = 0; ph < 2; ++ph) {
    GridUpdateArgs a;
    a.nx = grid->nx;
    a.ny = grid->ny;
    a.nz = grid->nz;
    a.dt = dt;
    a.g0 = gravity[0];
    a.g1 = gravity[1];
    a.g2 = gravity[2];
    a.bc_layers = bc_layers;
    a.gm = grid_mass + ph * N;
    a.gp = grid_mom + ph * 3 * N;
    a.gv = grid_vel + ph * 3 * N;
    a.clear_gm = nullptr;
    a.clear_gp = nullptr;
    a.regions = nullptr;
    a.n_regions = 0;
    if ((st = from_hip(launch_grid_update(a, (hipStream_t)stream)))) return st;
  }
  return POLYPIC_OK;
}

int32_t polypic_mixture_g2p(const polypic_grid* grid, int64_t P, int32_t n_modes, float dt,
                            const float* grid_vel, const float* x_in, const int32_t* phase_in,
                            const int32_t* perm, float* x_out, float* coeff_out,
                            const float* F_in, float* F_out, int32_t* phase_out,
                            const float* mass_f_in, float* mass_f_out, const float* mass_s_in,
                            float* mass_s_out, int32_t* status_dev, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (!valid_modes(n_modes) || !isfinite(dt)) return POLYPIC_EINVAL;
  if (P == 0) return POLYPIC_OK;
  if (!grid_vel || !x_in || !phase_in || !coeff_out) return POLYPIC_EINVAL;
  if ((F_in == nullptr) != (F_out == nullptr)) return POLYPIC_EINVAL;
  if ((mass_f_in == nullptr) != (mass_f_out == nullptr)) return POLYPIC_EINVAL;
  if ((mass_s_in == nullptr) != (mass_s_out == nullptr)) return POLYPIC_EINVAL;
  MixtureG2PArgs a;
  a.g = to_dev(grid);
  a.P = P;
  a.dt = dt;
  a.dx = grid->dx;
  clamp_bounds(grid, a.lo, a.hi);
  a.gv = grid_vel;
  a.x_in = x_in;
  a.phase_in = phase_in;
  a.perm = perm;
  a.x_out = x_out;
  a.coeff_out = coeff_out;
  a.F_in = F_in;
  a.F_out = F_out;
  a.phase_out = phase_out;
  a.mass_f_in = mass_f_in;
  a.mass_f_out = mass_f_out;
  a.mass_s_in = mass_s_in;
  a.mass_s_out = mass_s_out;
  a.status = status_dev;
  discard_stale_error();
  return from_hip(launch_mixture_g2p(a, n_modes, (hipStream_t)stream));
}

// ---- staggered (MAC) grid
int32_t polypic_mac_p2g(const polypic_grid* grid, int64_t P, int32_t n_modes, const float* x,
                        const float* mass, float uniform_mass, const float* coeff,
                        const int32_t* perm, float* face_mass, float* face_mom,
                        int32_t accumulate, int32_t* status_dev, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (!valid_modes(n_modes)) return POLYPIC_EINVAL;
  if (!face_mass || !face_mom) return POLYPIC_EINVAL;
  if (P > 0 && (!x || !coeff)) return POLYPIC_EINVAL;
  if (!mass && !isfinite(uniform_mass)) return POLYPIC_EINVAL;
  MacP2GArgs a;
  a.g = to_dev(grid);
  a.P = P;
  a.x = x;
  a.mass = mass;
  a.uniform_mass = uniform_mass;
  a.coeff = coeff;
  a.perm = perm;
  a.fm = face_mass;
  a.fp = face_mom;
  a.status = status_dev;
  discard_stale_error();
  return from_hip(launch_mac_p2g(a, n_modes, accumulate != 0, (hipStream_t)stream));
}

int32_t polypic_mac_grid_update(const polypic_grid* grid, float dt, const float* gravity,
                                int32_t bc_layers, const float* face_mass, const float* face_mom,
                                float* face_vel, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if (!gravity || !face_mass || !face_mom || !face_vel) return POLYPIC_EINVAL;
  if (!isfinite(dt) || bc_layers < 0) return POLYPIC_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (!isfinite(gravity[k])) return POLYPIC_EINVAL;
  MacUpdateArgs a;
  a.nx = grid->nx;
  a.ny = grid->ny;
  a.nz = grid->nz;
  a.dt = dt;
  a.g0 = gravity[0];
  a.g1 = gravity[1];
  a.g2 = gravity[2];
  a.bc_layers = bc_layers;
  a.fm = face_mass;
  a.fp = face_mom;
  a.fv = face_vel;
  discard_stale_error();
  return from_hip(launch_mac_grid_update(a, (hipStream_t)stream));
}

int32_t polypic_mac_g2p(const polypic_grid* grid, int64_t P, int32_t n_modes, float dt,
                        const float* face_vel, const float* x_in, const int32_t* perm,
                        float* x_out, float* coeff_out, const float* F_in, float* F_out,
                        const float* mass_in, float* mass_out, int32_t* status_dev,
                        void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (!valid_modes(n_modes) || !isfinite(dt)) return POLYPIC_EINVAL;
  if (P == 0) return POLYPIC_OK;
  if (!face_vel || !x_in || !coeff_out) return POLYPIC_EINVAL;
  if ((F_in == nullptr) != (F_out == nullptr)) return POLYPIC_EINVAL;
  if ((mass_in == nullptr) != (mass_out == nullptr)) return POLYPIC_EINVAL;
  MacG2PArgs a;
  a.g = to_dev(grid);
  a.P = P;
  a.dt = dt;
  a.dx = grid->dx;
  clamp_bounds(grid, a.lo, a.hi);
  a.fv = face_vel;
  a.x_in = x_in;
  a.perm = perm;
  a.x_out = x_out;
  a.coeff_out = coeff_out;
  a.F_in = F_in;
  a.F_out = F_out;
  a.mass_in = mass_in;
  a.mass_out = mass_out;
  a.status = status_dev;
  discard_stale_error();
  return from_hip(launch_mac_g2p(a, n_modes, (hipStream_t)stream));
}

namespace {
// an output of the fused call overlaps an input it reads, or the two grid outputs overlap
bool g2p2g_overlap(int64_t P, int64_t N, const float* grid_vel, const float* x_in,
                   const int32_t* perm, const float* F_in, const float* mass_in,
                   const float* grid_mass, const float* grid_mom, const float* x_out,
                   const float* F_out, const float* mass_out) {
  const void* ins[5] = {grid_vel, x_in, perm, F_in, mass_in};
  const int64_t nin[5] = {3 * N, 3 * P, P, 9 * P, P};
  const void* outs[5] = {grid_mass, grid_mom, x_out, F_out, mass_out};
  const int64_t nout[5] = {N, 3 * N, 3 * P, 9 * P, P};
  for (int o = 0; o < 5; ++o)
    for (int k = 0; k < 5; ++k)
      if (overlaps(outs[o], nout[o], ins[k], nin[k])) return true;
  return overlaps(grid_mass, N, grid_mom, 3 * N);
}
}  // namespace

namespace {
int32_t check_rows(const void* src, const void* dst, const int32_t* idx, int64_t rows,
                   int64_t P) {
  int32_t st;
  if ((st = check_P(P))) return st;
  if (rows < 0) return POLYPIC_EINVAL;
  if (rows == 0 || P == 0) return POLYPIC_OK;
  if (!src || !dst || !idx) return POLYPIC_EINVAL;
  if (rows > INT64_MAX / 4 / P) return POLYPIC_EINVAL;
  if (overlaps(src, rows * P, dst, rows * P)) return POLYPIC_EINVAL;
  return POLYPIC_OK;
}
}  // namespace

int32_t polypic_gather_rows(const void* src, void* dst, const int32_t* idx, int64_t rows,
                            int64_t P, void* stream) {
  int32_t st;
  if ((st = check_rows(src, dst, idx, rows, P))) return st;
  if (rows == 0 || P == 0) return POLYPIC_OK;
  discard_stale_error();
  return from_hip(launch_gather_rows(src, dst, idx, rows, P, (hipStream_t)stream));
}

int32_t polypic_scatter_rows(const void* src, void* dst, const int32_t* idx, int64_t rows,
                             int64_t P, void* stream) {
  int32_t st;
  if ((st = check_rows(src, dst, idx, rows, P))) return st;
  if (rows == 0 || P == 0) return POLYPIC_OK;
  discard_stale_error();
  return from_hip(launch_scatter_rows(src, dst, idx, rows, P, (hipStream_t)stream));
}

int32_t polypic_invert_permutation(const int32_t* perm, int32_t* inv, int64_t P, void* stream) {
  int32_t st;
  if ((st = check_P(P))) return st;
  if (P == 0) return POLYPIC_OK;
  if (!perm || !inv || overlaps(perm, P, inv, P)) return POLYPIC_EINVAL;
  discard_stale_error();
  return from_hip(launch_invert_permutation(perm, inv, P, (hipStream_t)stream));
}

int32_t polypic_g2p2g(const polypic_grid* grid, int64_t P, int32_t n_modes, float dt,
                      const float* grid_vel, const float* x_in, const int32_t* perm,
                      float* x_out, float* coeff_out, const float* F_in, float* F_out,
                      const float* mass_in, float* mass_out, float uniform_mass,
                      float* grid_mass, float* grid_mom, int32_t accumulate,
                      uint32_t* region_state, int32_t* status_dev, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (!valid_modes(n_modes) || !isfinite(dt)) return POLYPIC_EINVAL;
  if (!grid_mass || !grid_mom) return POLYPIC_EINVAL;
  if (!mass_in && !isfinite(uniform_mass)) return POLYPIC_EINVAL;
  if (P > 0 && (!grid_vel || !x_in || !x_out || !coeff_out)) return POLYPIC_EINVAL;
  if ((F_in == nullptr) != (F_out == nullptr)) return POLYPIC_EINVAL;
  if (mass_out && !mass_in) return POLYPIC_EINVAL;
  const int64_t N = n_nodes(grid);
  if (g2p2g_overlap(P, N, grid_vel, x_in, perm, F_in, mass_in, grid_mass, grid_mom, x_out, F_out,
                    mass_out))
    return POLYPIC_EINVAL;
  G2P2GArgs a;
  a.g = to_dev(grid);
  a.P = P;
  a.dt = dt;
  a.dx = grid->dx;
  clamp_bounds(grid, a.lo, a.hi);
  a.gv = grid_vel;
  a.x_in = x_in;
  a.perm = perm;
  a.x_out = x_out;
  a.coeff_out = coeff_out;
  a.F_in = F_in;
  a.F_out = F_out;
  a.mass_in = mass_in;
  a.mass_out = mass_out;
  a.uniform_mass = uniform_mass;
  a.gm = grid_mass;
  a.gp0 = grid_mom;
  a.gp1 = grid_mom + N;
  a.gp2 = grid_mom + 2 * N;
  a.status = status_dev;
  a.gstride = N;
  a.lane_group = fused_lane_group(n_modes);
  a.accumulate = accumulate != 0;
  a.sched = fused_sched(n_modes);
  a.regions = region_state;
  a.n_regions = region_count(grid->nx, grid->ny, grid->nz);
  discard_stale_error();
  return from_hip(launch_g2p2g(a, n_modes, (hipStream_t)stream));
}

int32_t polypic_set_g2p2g_config(int32_t n_modes, int32_t lane_group, int32_t schedule) {
  if (!valid_modes(n_modes)) return POLYPIC_EINVAL;
  if (lane_group != -1 && lane_group != 2 && lane_group != 4) return POLYPIC_EINVAL;
  if (schedule != -1 && schedule != POLYPIC_SCHED_LINEAR && schedule != POLYPIC_SCHED_XCD)
    return POLYPIC_EINVAL;
  g_fused_lane[n_modes].store(lane_group == -1 ? 0 : lane_group);
  g_fused_sched[n_modes].store(schedule == -1 ? POLYPIC_SCHED_LINEAR : schedule);
  return POLYPIC_OK;
}

int32_t polypic_get_g2p2g_config(int32_t n_modes, int32_t* lane_group, int32_t* schedule) {
  if (!valid_modes(n_modes) || !lane_group || !schedule) return POLYPIC_EINVAL;
  *lane_group = fused_lane_group(n_modes);
  *schedule = fused_sched(n_modes) == kSchedXcd ? POLYPIC_SCHED_XCD : POLYPIC_SCHED_LINEAR;
  return POLYPIC_OK;
}

int32_t polypic_autotune_g2p2g(const polypic_grid* grid, int64_t P, int32_t n_modes, float dt,
                               const float* grid_vel, const float* x_in, const int32_t* perm,
                               float* x_out, float* coeff_out, const float* F_in, float* F_out,
                               const float* mass_in, float* mass_out, float uniform_mass,
                               float* grid_mass, float* grid_mom, int32_t* lane_group_out,
                               int32_t* schedule_out, void* stream) {
  // the candidates run the call itself: validate once through it with the setting it has
  const int m = n_modes < 0 || n_modes > 27 ? 0 : n_modes;
  const int keep_lane = g_fused_lane[m].load(), keep_sched = g_fused_sched[m].load();
  int32_t st = polypic_g2p2g(grid, P, n_modes, dt, grid_vel, x_in, perm, x_out, coeff_out, F_in,
                             F_out, mass_in, mass_out, uniform_mass, grid_mass, grid_mom, 0,
                             nullptr, nullptr, stream);
  if (st) return st;
  const hipStream_t s = (hipStream_t)stream;
  // lane groups x chunk orders
  const int cand_lane[4] = {2, 4, 2, 4};
  const int cand_sched[4] = {POLYPIC_SCHED_LINEAR, POLYPIC_SCHED_LINEAR, POLYPIC_SCHED_XCD,
                             POLYPIC_SCHED_XCD};
  int bi = 0;
  st = time_candidates(
      4, s,
      [&](int k) {
        g_fused_lane[n_modes].store(cand_lane[k]);
        g_fused_sched[n_modes].store(cand_sched[k]);
        return polypic_g2p2g(grid, P, n_modes, dt, grid_vel, x_in, perm, x_out, coeff_out, F_in,
                             F_out, mass_in, mass_out, uniform_mass, grid_mass, grid_mom, 0,
                             nullptr, nullptr, stream);
      },
      &bi);
  if (st) {
    g_fused_lane[n_modes].store(keep_lane);
    g_fused_sched[n_modes].store(keep_sched);
    return st;
  }
  g_fused_lane[n_modes].store(cand_lane[bi]);
  g_fused_sched[n_modes].store(cand_sched[bi]);
  if (lane_group_out) *lane_group_out = cand_lane[bi];
  if (schedule_out) *schedule_out = cand_sched[bi];
  // the outputs hold the last candidate's results: rerun the chosen one so that they
  // are the call's (the two differ only in the order of the grid sums)
  return polypic_g2p2g(grid, P, n_modes, dt, grid_vel, x_in, perm, x_out, coeff_out, F_in,
                       F_out, mass_in, mass_out, uniform_mass, grid_mass, grid_mom, 0, nullptr,
                       nullptr, stream);
}

int32_t polypic_g2p_backward(const polypic_grid* grid, int64_t P, int32_t n_modes, float dt,
                             const float* grid_vel, const float* x_in, const int32_t* perm,
                             const float* coeff_out_grad, const float* x_out_grad,
                             float* grid_vel_grad, int32_t accumulate, float* x_in_grad,
                             int32_t* status_dev, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (!valid_modes(n_modes) || !isfinite(dt)) return POLYPIC_EINVAL;
  if (!grid_vel_grad) return POLYPIC_EINVAL;
  if (P > 0 && (!grid_vel || !x_in || !coeff_out_grad || !x_in_grad)) return POLYPIC_EINVAL;
  const hipStream_t s = (hipStream_t)stream;
  discard_stale_error();
  if (!accumulate) {
    if ((st = from_hip(launch_zero(grid_vel_grad, 3 * n_nodes(grid), s)))) return st;
  }
  if (P == 0) return POLYPIC_OK;
  G2PBackArgs a;
  a.g = to_dev(grid);
  a.P = P;
  a.dt = dt;
  clamp_bounds(grid, a.lo, a.hi);
  a.gv = grid_vel;
  a.x_in = x_in;
  a.perm = perm;
  a.coeff_out_grad = coeff_out_grad;
  a.x_out_grad = x_out_grad;
  a.gvb = grid_vel_grad;
  a.x_in_grad = x_in_grad;
  a.status = status_dev;
  return from_hip(launch_g2p_backward(a, n_modes, s));
}

int32_t polypic_grid_update_backward(const polypic_grid* grid, float dt, const float* gravity,
                                     int32_t bc_layers, const float* grid_mass,
                                     const float* grid_mom, const float* grid_vel_grad,
                                     float* grid_mass_grad, float* grid_mom_grad, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if (!gravity || !grid_mass || !grid_mom || !grid_vel_grad || !grid_mass_grad || !grid_mom_grad)
    return POLYPIC_EINVAL;
  if (!isfinite(dt) || bc_layers < 0) return POLYPIC_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (!isfinite(gravity[a])) return POLYPIC_EINVAL;
  GridUpdateBackArgs a;
  a.nx = grid->nx;
  a.ny = grid->ny;
  a.nz = grid->nz;
  a.dt = dt;
  a.g0 = gravity[0];
  a.g1 = gravity[1];
  a.g2 = gravity[2];
  a.bc_layers = bc_layers;
  a.gm = grid_mass;
  a.gp = grid_mom;
  a.gvb = grid_vel_grad;
  a.gmb = grid_mass_grad;
  a.gpb = grid_mom_grad;
  discard_stale_error();
  return from_hip(launch_grid_update_backward(a, (hipStream_t)stream));
}

int32_t polypic_p2g_backward(const polypic_grid* grid, int64_t P, int32_t n_modes, const float* x,
                             const float* mass, float uniform_mass, const float* coeff,
                             const int32_t* perm, const float* grid_mass_grad,
                             const float* grid_mom_grad, float* coeff_grad, float* x_grad,
                             float* mass_grad, int32_t* status_dev, void* stream) {
  int32_t st = check_grid(grid);
  if (st) return st;
  if ((st = check_P(P))) return st;
  if (!valid_modes(n_modes)) return POLYPIC_EINVAL;
  if (P == 0) return POLYPIC_OK;
  if (!x || !coeff || !grid_mass_grad || !grid_mom_grad || !coeff_grad || !x_grad)
    return POLYPIC_EINVAL;
  if (!mass && !isfinite(uniform_mass)) return POLYPIC_EINVAL;
  P2GBackArgs a;
  a.g = to_dev(grid);
  a.P = P;
  a.x = x;
  a.mass = mass;
  a.uniform_mass = uniform_mass;
  a.coeff = coeff;
  a.perm = perm;
  a.gmb = grid_mass_grad;
  a.gpb = grid_mom_grad;
  a.coeff_grad = coeff_grad;
  a.x_grad = x_grad;
  a.mass_grad = mass_grad;
  a.status = status_dev;
  discard_stale_error();
  return from_hip(launch_p2g_backward(a, n_modes, (hipStream_t)stream));
}


// ---------------------------------------------------------------- batches
int32_t polypic_batch_table_bytes(int32_t n_scenes, size_t* bytes) {
  if (!bytes || n_scenes < 1 || n_scenes > kMaxScenes) return POLYPIC_EINVAL;
  *bytes = align_up((size_t)n_scenes * sizeof(SceneDev));
  return POLYPIC_OK;
}

int32_t polypic_batch_plan(const polypic_scene* scenes, int32_t n_scenes, int64_t n_nodes_total,
                           void* table_dev, size_t table_bytes, polypic_batch* batch,
                           void* stream) {
  if (!scenes || !batch || !table_dev) return POLYPIC_EINVAL;
  if (n_scenes < 1 || n_scenes > kMaxScenes || n_nodes_total < 1) return POLYPIC_EINVAL;
  if (table_bytes < (size_t)n_scenes * sizeof(SceneDev)) return POLYPIC_ENOSPACE;
  std::vector<SceneDev> host((size_t)n_scenes);
  int64_t p_next = 0, node_end = 0, max_nodes = 0, chunks = 0, regions = 0;
  int mbits = 0;
  for (int32_t k = 0; k < n_scenes; ++k) {
    const polypic_scene& sc = scenes[k];
    int32_t st = check_grid(&sc.grid);
    if (st) return st;
    if (sc.n_particles < 0 || sc.p_offset != p_next) return POLYPIC_EINVAL;
    p_next += sc.n_particles;
    if (p_next > (int64_t)INT32_MAX) return POLYPIC_EINVAL;
    const int64_t nn = n_nodes(&sc.grid);
    if (sc.node_offset < node_end || sc.node_offset > n_nodes_total - nn) return POLYPIC_EINVAL;
    node_end = sc.node_offset + nn;
    max_nodes = std::max(max_nodes, nn);
    mbits = std::max(mbits, sort_key_bits(to_dev(&sc.grid)));
    SceneDev& d = host[(size_t)k];
    d.nx = sc.grid.nx;
    d.ny = sc.grid.ny;
    d.nz = sc.grid.nz;
    d.inv_dx = sc.grid.inv_dx;
    d.ox = sc.grid.origin[0];
    d.oy = sc.grid.origin[1];
    d.oz = sc.grid.origin[2];
    d.dx = sc.grid.dx;
    clamp_bounds(&sc.grid, d.lo, d.hi);
    d.p_begin = sc.p_offset;
    d.p_end = sc.p_offset + sc.n_particles;
    d.node_off = sc.node_offset;
    d.chunk_begin = chunks;
    chunks += (sc.n_particles + kSceneChunk - 1) / kSceneChunk;
    d.region_begin = regions;
    regions += region_count(sc.grid.nx, sc.grid.ny, sc.grid.nz);
  }
  int sbits = 0;
  while (((int64_t)1 << sbits) < (int64_t)n_scenes) ++sbits;
  if (mbits + sbits > 32) return POLYPIC_ENOTSUP;
  const hipStream_t s = (hipStream_t)stream;
  discard_stale_error();
  int32_t st = from_hip(hipMemcpyAsync(table_dev, host.data(), host.size() * sizeof(SceneDev),
                                       hipMemcpyHostToDevice, s));
  if (!st) st = from_hip(hipStreamSynchronize(s));
  if (st) return st;
  batch->n_scenes = n_scenes;
  batch->key_bits = mbits + sbits;
  batch->morton_bits = mbits;
  batch->max_nodes = (int32_t)max_nodes;
  batch->P = p_next;
  batch->N = n_nodes_total;
  batch->n_regions = regions;
  batch->table = table_dev;
  batch->seal = batch_seal(batch);
  return POLYPIC_OK;
}

int32_t polypic_batch_sort_workspace_bytes(const polypic_batch* batch, size_t* bytes) {
  int32_t st = check_batch(batch);
  if (st) return st;
  if (!bytes) return POLYPIC_EINVAL;
  *bytes = sort_workspace_bytes(batch->P);
  return POLYPIC_OK;
}

int32_t polypic_batch_sort(const polypic_batch* batch, const float* x, uint32_t* keys_out,
                           int32_t* perm_out, void* ws, size_t ws_bytes, int32_t* status_dev,
                           void* stream) {
  int32_t st = check_batch(batch);
  if (st) return st;
  if (batch->P == 0) return POLYPIC_OK;
  if (!x || !keys_out || !perm_out || !ws) return POLYPIC_EINVAL;
  if (ws_bytes < sort_workspace_bytes(batch->P)) return POLYPIC_ENOSPACE;
  discard_stale_error();
  return from_hip(launch_sort_batch(batch_table(batch), batch->n_scenes, batch->morton_bits,
                                    batch->key_bits, batch->P, x, keys_out, perm_out, ws,
                                    status_dev, (hipStream_t)stream));
}

int32_t polypic_batch_sort_update_workspace_bytes(const polypic_batch* batch, size_t* bytes) {
  int32_t st = check_batch(batch);
  if (st) return st;
  if (!bytes) return POLYPIC_EINVAL;
  *bytes = sort_update_workspace_bytes(batch->P);
  return POLYPIC_OK;
}

int32_t polypic_batch_sort_update(const polypic_batch* batch, const float* x,
                                  const uint32_t* keys_prev, uint32_t* keys_out,
                                  int32_t* perm_out, void* ws, size_t ws_bytes,
                                  int32_t* status_dev, void* stream) {
  int32_t st = check_batch(batch);
  if (st) return st;
  if (batch->P == 0) return POLYPIC_OK;
  if (!x || !keys_prev || !keys_out || !perm_out || !ws) return POLYPIC_EINVAL;
  if ((const void*)keys_prev == (const void*)keys_out) return POLYPIC_EINVAL;
  if (ws_bytes < sort_update_workspace_bytes(batch->P)) return POLYPIC_ENOSPACE;
  discard_stale_error();
  return from_hip(launch_sort_update_batch(batch_table(batch), batch->n_scenes,
                                           batch->morton_bits, batch->key_bits, batch->P, x,
                                           keys_prev, keys_out, perm_out, ws, status_dev,
                                           (hipStream_t)stream));
}

int32_t polypic_batch_p2g(const polypic_batch* batch, int32_t n_modes, const float* x,
                          const float* mass, float uniform_mass, const float* coeff,
                          const int32_t* perm, float* grid_mass, float* grid_mom,
                          int32_t accumulate, int32_t* status_dev, void* stream) {
  int32_t st = check_batch(batch);
  if (st) return st;
  if (!valid_modes(n_modes)) return POLYPIC_EINVAL;
  if (!grid_mass || !grid_mom) return POLYPIC_EINVAL;
  if (batch->P > 0 && (!x || !coeff)) return POLYPIC_EINVAL;
  if (!mass && !isfinite(uniform_mass)) return POLYPIC_EINVAL;
  discard_stale_error();
  return run_batch_p2g(batch, n_modes, x, mass, uniform_mass, coeff, perm, grid_mass, grid_mom,
                       accumulate, status_dev, (hipStream_t)stream, get_bchoice(n_modes));
}

int32_t polypic_batch_grid_update(const polypic_batch* batch, float dt, const float* gravity,
                                  int32_t bc_layers, const float* grid_mass,
                                  const float* grid_mom, float* grid_vel, void* stream) {
  int32_t st = check_batch(batch);
  if (st) return st;
  if (!gravity || !grid_mass || !grid_mom || !grid_vel) return POLYPIC_EINVAL;
  if (!isfinite(dt) || bc_layers < 0) return POLYPIC_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (!isfinite(gravity[a])) return POLYPIC_EINVAL;
  GridUpdateArgs a;
  a.nx = a.ny = a.nz = 0;  // per scene, from the table
  a.dt = dt;
  a.g0 = gravity[0];
  a.g1 = gravity[1];
  a.g2 = gravity[2];
  a.bc_layers = bc_layers;
  a.gm = grid_mass;
  a.gp = grid_mom;
  a.gv = grid_vel;
  a.clear_gm = nullptr;
  a.clear_gp = nullptr;
  a.regions = nullptr;
  a.n_regions = 0;
  discard_stale_error();
  return from_hip(launch_grid_update_batch(a, batch_table(batch), batch->n_scenes,
                                           batch->max_nodes, batch->N, (hipStream_t)stream));
}

int32_t polypic_batch_grid_update_active(const polypic_batch* batch, float dt,
                                         const float* gravity, int32_t bc_layers,
                                         float* grid_mass, float* grid_mom, float* grid_vel,
                                         uint32_t* region_state, void* stream) {
  int32_t st = check_batch(batch);
  if (st) return st;
  if (!gravity || !grid_mass || !grid_mom || !grid_vel || !region_state) return POLYPIC_EINVAL;
  if (!isfinite(dt) || bc_layers < 0) return POLYPIC_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (!isfinite(gravity[a])) return POLYPIC_EINVAL;
  const int64_t N = batch->N;
  if (overlaps(grid_vel, 3 * N, grid_mass, N) || overlaps(grid_vel, 3 * N, grid_mom, 3 * N))
    return POLYPIC_EINVAL;
  GridUpdateArgs a;
  a.nx = a.ny = a.nz = 0;  // per scene, from the table
  a.dt = dt;
  a.g0 = gravity[0];
  a.g1 = gravity[1];
  a.g2 = gravity[2];
  a.bc_layers = bc_layers;
  a.gm = grid_mass;
  a.gp = grid_mom;
  a.gv = grid_vel;
  a.clear_gm = grid_mass;
  a.clear_gp = grid_mom;
  a.regions = region_state;
  a.n_regions = batch->n_regions;
  discard_stale_error();
  return from_hip(launch_grid_update_active_batch(a, batch_table(batch), batch->n_scenes, N,
                                                  (hipStream_t)stream));
}

int32_t polypic_batch_g2p(const polypic_batch* batch, int32_t n_modes, float dt,
                          const float* grid_vel, const float* x_in, const int32_t* perm,
                          float* x_out, float* coeff_out, const float* F_in, float* F_out,
                          const float* mass_in, float* mass_out, int32_t* status_dev,
                          void* stream) {
  int32_t st = check_batch(batch);
  if (st) return st;
  if (!valid_modes(n_modes) || !isfinite(dt)) return POLYPIC_EINVAL;
  if (batch->P == 0) return POLYPIC_OK;
  if (!grid_vel || !x_in || !coeff_out) return POLYPIC_EINVAL;
  if ((F_in == nullptr) != (F_out == nullptr)) return POLYPIC_EINVAL;
  if ((mass_in == nullptr) != (mass_out == nullptr)) return POLYPIC_EINVAL;
  G2PArgs a;
  a.g = GridDev{3, 3, 3, 1.0f, 0.0f, 0.0f, 0.0f};  // unused: per scene, from the table
  a.P = batch->P;
  a.dt = dt;
  a.dx = 1.0f;
  for (int k = 0; k < 3; ++k) a.lo[k] = a.hi[k] = 0.0f;
  a.gv = grid_vel;
  a.x_in = x_in;
  a.perm = perm;
  a.x_out = x_out;
  a.coeff_out = coeff_out;
  a.F_in = F_in;
  a.F_out = F_out;
  a.mass_in = mass_in;
  a.mass_out = mass_out;
  a.status = status_dev;
  a.gstride = batch->N;
  a.sched = g_g2p_sched.load() == POLYPIC_SCHED_XCD ? kSchedXcd : kSchedLinear;
  discard_stale_error();
  return from_hip(
      launch_g2p_batch(a, batch_table(batch), batch->n_scenes, n_modes, (hipStream_t)stream));
}

int32_t polypic_batch_g2p2g(const polypic_batch* batch, int32_t n_modes, float dt,
                            const float* grid_vel, const float* x_in, const int32_t* perm,
                            float* x_out, float* coeff_out, const float* F_in, float* F_out,
                            const float* mass_in, float* mass_out, float uniform_mass,
                            float* grid_mass, float* grid_mom, int32_t accumulate,
                            uint32_t* region_state, int32_t* status_dev, void* stream) {
  int32_t st = check_batch(batch);
  if (st) return st;
  if (!valid_modes(n_modes) || !isfinite(dt)) return POLYPIC_EINVAL;
  if (!grid_mass || !grid_mom) return POLYPIC_EINVAL;
  if (!mass_in && !isfinite(uniform_mass)) return POLYPIC_EINVAL;
  const int64_t P = batch->P, N = batch->N;
  if (P > 0 && (!grid_vel || !x_in || !x_out || !coeff_out)) return POLYPIC_EINVAL;
  if ((F_in == nullptr) != (F_out == nullptr)) return POLYPIC_EINVAL;
  if (mass_out && !mass_in) return POLYPIC_EINVAL;
  if (g2p2g_overlap(P, N, grid_vel, x_in, perm, F_in, mass_in, grid_mass, grid_mom, x_out, F_out,
                    mass_out))
    return POLYPIC_EINVAL;
  G2P2GArgs a;
  a.g = GridDev{3, 3, 3, 1.0f, 0.0f, 0.0f, 0.0f};  // unused: per scene, from the table
  a.P = P;
  a.dt = dt;
  a.dx = 1.0f;
  for (int k = 0; k < 3; ++k) a.lo[k] = a.hi[k] = 0.0f;
  a.gv = grid_vel;
  a.x_in = x_in;
  a.perm = perm;
  a.x_out = x_out;
  a.coeff_out = coeff_out;
  a.F_in = F_in;
  a.F_out = F_out;
  a.mass_in = mass_in;
  a.mass_out = mass_out;
  a.uniform_mass = uniform_mass;
  a.gm = grid_mass;
  a.gp0 = grid_mom;
  a.gp1 = grid_mom + N;
  a.gp2 = grid_mom + 2 * N;
  a.status = status_dev;
  a.gstride = N;
  a.accumulate = accumulate != 0;
  a.regions = region_state;
  a.n_regions = batch->n_regions;
  // lane pairs; chunks XCD-contiguous: a batch's grids do not stay in the last-level
  // cache between the passes, so neighbouring chunks share one L2 (measured, 64
  // scenes, 25.7 M particles: 3.81 -> 3.57 ms per graph step)
  a.sched = kSchedXcd;
  a.lane_group = 2;
  discard_stale_error();
  return from_hip(launch_g2p2g_batch(a, batch_table(batch), batch->n_scenes, n_modes,
                                     (hipStream_t)stream));
}

int32_t polypic_batch_set_config(int32_t n_modes, int32_t block, int32_t schedule,
                                 int32_t per_cu, int32_t brick) {
  if (!valid_modes(n_modes)) return POLYPIC_EINVAL;
  if (block != 256 && block != 512) return POLYPIC_EINVAL;
  if (!valid_schedule(schedule, per_cu)) return POLYPIC_EINVAL;
  if (!valid_brick(brick)) return POLYPIC_EINVAL;
  BatchChoice c;
  c.block = block;
  c.sched = schedule;
  c.per_cu = schedule == POLYPIC_SCHED_PERSISTENT ? per_cu : 0;
  c.brick = brick;
  set_bchoice(n_modes, c);
  return POLYPIC_OK;
}

int32_t polypic_batch_get_config(int32_t n_modes, int32_t* block, int32_t* schedule,
                                 int32_t* per_cu, int32_t* brick) {
  if (!valid_modes(n_modes)) return POLYPIC_EINVAL;
  const BatchChoice c = get_bchoice(n_modes);
  if (block) *block = c.block;
  if (schedule) *schedule = c.sched;
  if (per_cu) *per_cu = c.per_cu;
  if (brick) *brick = c.brick;
  return POLYPIC_OK;
}

int32_t polypic_batch_autotune(const polypic_batch* batch, int32_t n_modes, const float* x,
                               const float* mass, float uniform_mass, const float* coeff,
                               const int32_t* perm, float* grid_mass, float* grid_mom,
                               int32_t* block_out, int32_t* schedule_out, int32_t* per_cu_out,
                               int32_t* brick_out, void* stream) {
  int32_t st = check_batch(batch);
  if (st) return st;
  if (!valid_modes(n_modes)) return POLYPIC_EINVAL;
  if (!grid_mass || !grid_mom) return POLYPIC_EINVAL;
  if (batch->P > 0 && (!x || !coeff)) return POLYPIC_EINVAL;
  if (!mass && !isfinite(uniform_mass)) return POLYPIC_EINVAL;
  std::vector<BatchChoice> cand;
  for (int block : {256, 512}) {
    for (int brick : {4, 2, 8})
      for (int sched : {POLYPIC_SCHED_LINEAR, POLYPIC_SCHED_XCD}) {
        BatchChoice c;
        c.block = block;
        c.sched = sched;
        c.brick = brick;
        cand.push_back(c);
      }
    for (int per_cu : {2, 4, 8}) {  // (4^3 bricks)
      BatchChoice c;
      c.block = block;
      c.sched = POLYPIC_SCHED_PERSISTENT;
      c.per_cu = per_cu;
      cand.push_back(c);
    }
  }
  const hipStream_t s = (hipStream_t)stream;
  discard_stale_error();
  int bi = 0;
  st = time_candidates(
      (int)cand.size(), s,
      [&](int k) {
        return run_batch_p2g(batch, n_modes, x, mass, uniform_mass, coeff, perm, grid_mass,
                             grid_mom, 0, nullptr, s, cand[k]);
      },
      &bi);
  if (st) return st;
  set_bchoice(n_modes, cand[bi]);
  if (block_out) *block_out = cand[bi].block;
  if (schedule_out) *schedule_out = cand[bi].sched;
  if (per_cu_out) *per_cu_out = cand[bi].per_cu;
  if (brick_out) *brick_out = cand[bi].brick;
  return POLYPIC_OK;
}

}  // extern "C"
