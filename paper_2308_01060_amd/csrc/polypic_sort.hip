// Cell keys, the stable LSD radix sort (8-bit digits) and the re-sort, for gfx950.
//
// Full sort, per pass: (1) per-tile digit histograms, (2) per-digit exclusive
// scan over tiles, (3) a stable scatter in which every tile ranks its keys in
// input order -- within a wavefront by ballot matching of equal digits, across
// the wavefronts of the block through small LDS histograms.  Ties keep input
// order, so the result equals a stable argsort of the keys.
//
// Re-sort: after a step whose particle arrays were permuted by the previous
// sort, only the particles whose cell changed are out of place.  They are
// compacted and sorted on their own (a radix sort whose length only the device
// knows), then merged with the unchanged ones by (key, index).
#include "polypic_internal.hpp"

namespace polypic {

namespace {

constexpr int kSortBS = 256;
constexpr int kSortIPT = 8;
constexpr int kSortTile = kSortBS * kSortIPT;
constexpr int kRadix = 256;
constexpr int kSortWaves = kSortBS / kWave;

// Cell key of every particle: Morton code of its base node, with the scene
// index above bit `mbits` when the launch covers a batch of scenes.
template <class Scenes>
__global__ __launch_bounds__(256) void sort_keys_kernel(Scenes sc, int mbits, int64_t P,
                                                        const float* __restrict__ x,
                                                        uint32_t* __restrict__ keys,
                                                        int32_t* __restrict__ vals,
                                                        int32_t* __restrict__ status) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x;
  const int64_t i = i0 + threadIdx.x;
  if (i >= P) return;
  const int s0 = sc.first(i0);  // uniform over the workgroup
  const int s = sc.of(i, s0);
  SceneGrid g = sc.grid(s0);
  if constexpr (Scenes::kMany) {
    if (__ballot(s != s0) != 0ull) g = sc.grid(s);
  }
  const size_t Ps = (size_t)P;
  int b0, b1, b2;
  float t0, t1, t2;
  bool ok = stencil_axis(x[i], g.ox, g.inv_dx, g.nx, b0, t0);
  ok &= stencil_axis(x[Ps + i], g.oy, g.inv_dx, g.ny, b1, t1);
  ok &= stencil_axis(x[2 * Ps + i], g.oz, g.inv_dx, g.nz, b2, t2);
  if (!ok) {
    raise_flag(status, kFlagRange);
    // stencil_axis returns b = 0 for an out-of-range axis: the key stays in the
    // configured bit range (and in its scene) and the order is deterministic.
  }
  keys[i] = ((uint32_t)s << mbits) | morton3(b0, b1, b2);
  vals[i] = (int32_t)i;
}

__global__ __launch_bounds__(kSortBS) void sort_hist_kernel(const uint32_t* __restrict__ keys,
                                                           int64_t P, int shift,
                                                           uint32_t* __restrict__ counts,
                                                           int n_tiles) {
  __shared__ uint32_t hist[kRadix];
  const int tid = threadIdx.x;
  hist[tid] = 0;  // kSortBS == kRadix
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
  for (int k = 0; k < kSortIPT; ++k) {
    const int64_t idx = base + (int64_t)k * kSortBS + tid;
    if (idx < P) atomicAdd(&hist[(keys[idx] >> shift) & (kRadix - 1)], 1u);
  }
  __syncthreads();
  counts[(size_t)tid * n_tiles + blockIdx.x] = hist[tid];
}

// One block per digit: exclusive scan of counts[d][0..n_tiles) in place.
__global__ __launch_bounds__(256) void sort_scan_kernel(uint32_t* __restrict__ counts, int n_tiles,
                                                        uint32_t* __restrict__ totals) {
  __shared__ uint32_t wsum[256 / kWave];
  const int d = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  uint32_t* row = counts + (size_t)d * n_tiles;
  uint32_t running = 0;
  for (int base = 0; base < n_tiles; base += 256) {
    const int idx = base + tid;
    const uint32_t v = idx < n_tiles ? row[idx] : 0u;
    // inclusive wave scan
    uint32_t s = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t o = __shfl_up(s, off, kWave);
      if (lane >= off) s += o;
    }
    if (lane == kWave - 1) wsum[wv] = s;
    __syncthreads();
    uint32_t pre = 0;
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < 256 / kWave; ++w) {
      const uint32_t ws = wsum[w];
      pre += (w < wv) ? ws : 0u;
      tot += ws;
    }
    if (idx < n_tiles) row[idx] = running + pre + s - v;
    running += tot;
    __syncthreads();
  }
  if (tid == 0) totals[d] = running;
}

__global__ __launch_bounds__(kSortBS) void sort_scatter_kernel(
    const uint32_t* __restrict__ keys_in, const int32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, int32_t* __restrict__ vals_out, int64_t P, int shift,
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ totals, int n_tiles) {
  __shared__ uint32_t offset[kRadix];               // next output slot per digit
  __shared__ uint32_t wave_hist[kSortWaves][kRadix];  // per-wave digit counts of one round
  __shared__ uint32_t wsum[kSortWaves];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;

  // digit base = exclusive scan of totals; plus this tile's prefix
  {
    const uint32_t v = totals[tid];
    uint32_t s = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t o = __shfl_up(s, off, kWave);
      if (lane >= off) s += o;
    }
    if (lane == kWave - 1) wsum[wv] = s;
    __syncthreads();
    uint32_t pre = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) pre += (w < wv) ? wsum[w] : 0u;
    offset[tid] = pre + s - v + counts[(size_t)tid * n_tiles + blockIdx.x];
  }

  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int k = 0; k < kSortIPT; ++k) {
    const int64_t idx = base + (int64_t)k * kSortBS + tid;
    const bool valid = idx < P;
    uint32_t key = 0;
    int32_t val = 0;
    if (valid) {
      key = keys_in[idx];
      val = vals_in[idx];
    }
    const uint32_t d = (key >> shift) & (kRadix - 1);
    // lanes of this wave holding the same digit
    unsigned long long same = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const unsigned long long bal = __ballot((d >> bit) & 1u);
      same &= ((d >> bit) & 1u) ? bal : ~bal;
    }
    const int rank = lanes_below(same);
    const int cnt = __popcll(same);

#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) wave_hist[w][tid] = 0u;
    __syncthreads();
    if (valid && rank == 0) wave_hist[wv][d] = (uint32_t)cnt;
    __syncthreads();
    if (valid) {
      uint32_t pos = offset[d] + (uint32_t)rank;
      for (int w = 0; w < wv; ++w) pos += wave_hist[w][d];
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) add += wave_hist[w][tid];
    offset[tid] += add;
    // the next round's clear of wave_hist is ordered after these reads by the
    // barrier that follows it
    __syncthreads();
  }
}

}  // namespace

size_t sort_workspace_bytes(int64_t P) {
  const int64_t n_tiles = (P + kSortTile - 1) / kSortTile;
  size_t bytes = 0;
  bytes += align_up((size_t)P * sizeof(uint32_t));             // alternate keys
  bytes += align_up((size_t)P * sizeof(int32_t));              // alternate values
  bytes += align_up((size_t)kRadix * (size_t)n_tiles * sizeof(uint32_t));  // counts
  bytes += align_up((size_t)kRadix * sizeof(uint32_t));        // totals
  return bytes;
}

int sort_key_bits(const GridDev& g) {
  int maxb = g.nx;
  if (g.ny > maxb) maxb = g.ny;
  if (g.nz > maxb) maxb = g.nz;
  maxb -= 3;  // largest base node index
  int bits = 0;
  while ((1 << bits) <= maxb) ++bits;
  if (bits == 0) bits = 1;
  return 3 * bits;
}

namespace {

// Stable LSD radix sort of the keys the key kernel wrote to (ksrc, vsrc); the
// last pass lands in (keys_out, perm_out).
template <class Scenes>
hipError_t sort_with(const Scenes& sc, int mbits, int key_bits, int64_t P, const float* x,
                     uint32_t* keys_out, int32_t* perm_out, void* ws, int32_t* status,
                     hipStream_t stream) {
  if (P == 0) return hipSuccess;
  const int n_tiles = (int)((P + kSortTile - 1) / kSortTile);
  char* w = (char*)ws;
  uint32_t* keys_alt = (uint32_t*)w;
  w += align_up((size_t)P * sizeof(uint32_t));
  int32_t* vals_alt = (int32_t*)w;
  w += align_up((size_t)P * sizeof(int32_t));
  uint32_t* counts = (uint32_t*)w;
  w += align_up((size_t)kRadix * (size_t)n_tiles * sizeof(uint32_t));
  uint32_t* totals = (uint32_t*)w;

  const int passes = (key_bits + 7) / 8;
  // Ping-pong so that the last pass writes keys_out / perm_out.
  uint32_t* ksrc = (passes % 2) ? keys_alt : keys_out;
  int32_t* vsrc = (passes % 2) ? vals_alt : perm_out;
  uint32_t* kdst = (passes % 2) ? keys_out : keys_alt;
  int32_t* vdst = (passes % 2) ? perm_out : vals_alt;

  const int kb = 256;
  sort_keys_kernel<Scenes><<<(unsigned)((P + kb - 1) / kb), kb, 0, stream>>>(sc, mbits, P, x,
                                                                            ksrc, vsrc, status);
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = 8 * pass;
    sort_hist_kernel<<<n_tiles, kSortBS, 0, stream>>>(ksrc, P, shift, counts, n_tiles);
    sort_scan_kernel<<<kRadix, 256, 0, stream>>>(counts, n_tiles, totals);
    sort_scatter_kernel<<<n_tiles, kSortBS, 0, stream>>>(ksrc, vsrc, kdst, vdst, P, shift, counts,
                                                         totals, n_tiles);
    uint32_t* kt = ksrc;
    ksrc = kdst;
    kdst = kt;
    int32_t* vt = vsrc;
    vsrc = vdst;
    vdst = vt;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sort(const GridDev& g, int64_t P, const float* x, uint32_t* keys_out,
                       int32_t* perm_out, void* ws, int32_t* status, hipStream_t stream) {
  OneScene one;
  one.sg.nx = g.nx;
  one.sg.ny = g.ny;
  one.sg.nz = g.nz;
  one.sg.inv_dx = g.inv_dx;
  one.sg.ox = g.ox;
  one.sg.oy = g.oy;
  one.sg.oz = g.oz;
  one.sg.dx = 0.0f;
  for (int k = 0; k < 3; ++k) one.sg.lo[k] = one.sg.hi[k] = 0.0f;
  one.sg.node_off = 0;
  const int bits = sort_key_bits(g);
  return sort_with(one, bits, bits, P, x, keys_out, perm_out, ws, status, stream);
}

hipError_t launch_sort_batch(const SceneDev* table, int n_scenes, int mbits, int key_bits,
                             int64_t P, const float* x, uint32_t* keys_out, int32_t* perm_out,
                             void* ws, int32_t* status, hipStream_t stream) {
  SceneTable st{table, n_scenes};
  return sort_with(st, mbits, key_bits, P, x, keys_out, perm_out, ws, status, stream);
}


// ------------------------------------------------ sort of a device-counted list
// Sorts the first *count (key, value) pairs of a buffer sized for `cap` pairs
// when the host does not know the count.  The kernel that writes the list also
// writes the count, the digit totals of every pass and cleared look-back words
// (the re-sort's compaction below); then comes one stable scatter launch per
// pass.  A scatter tile learns how many keys of each digit precede it from its
// predecessors' published counts (decoupled look-back): each tile publishes
// its own digit counts as soon as it has them, then reads its predecessors'
// words, nearest first and kLookWindow per round trip, until an inclusive
// prefix, and publishes its own inclusive prefix.  Tiles are numbered in the
// order workgroups claim them (an atomic counter), so a tile only waits on
// tiles whose workgroups already run and publish before they wait.  The polls
// must be coherent across the chip's L2 caches, so a chain over thousands of
// tiles is slow; the lists sorted here are short (the changed particles).
//
// Inside a tile, wave w ranks the contiguous keys [w * 512, (w + 1) * 512) in
// rounds of 64 by ballot matching of equal digits, keeping a wave-private
// running count per digit; the per-digit counts are then prefixed over the
// waves.  Order inside a tile is (wave, round, lane) = input order: stable.
namespace {

constexpr int kMaxPasses = 4;
constexpr int kWaveKeys = kSortTile / kSortWaves;
constexpr uint32_t kInclusive = 0x80000000u;
// look-back word: 0 = not yet published; 1 + n = the tile's own count n;
// kInclusive | n = keys with this digit in this tile and all tiles before it
constexpr int kSpinLimit = 1 << 20;  // polls without progress before giving up
constexpr int kLookWindow = 16;      // predecessors read per round trip
constexpr int kCountedGrid = 512;    // workgroups of the device-counted sort's launches
// The digit totals are accumulated in kTotalsRep copies, workgroup b adding into
// copy b % kTotalsRep: the changed particles crowd into few digits (they sit
// near one front), and one copy's atomics from thousands of workgroups
// serialise (measured: 6 -> 26 us for the compaction as the front grew).
constexpr int kTotalsRep = 32;
constexpr int kTotalsStride = kMaxPasses * kRadix;  // words per copy
static_assert(kSortBS == kRadix, "one thread per digit");
static_assert(kWaveKeys == kSortIPT * kWave, "a wave's keys are kSortIPT rounds of a wave");

__device__ __forceinline__ uint32_t load_agent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// lanes of the wave whose (valid) digit equals this lane's; every lane calls it
__device__ __forceinline__ unsigned long long match_digit(uint32_t d, bool valid) {
  unsigned long long same = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < 8; ++bit) {
    const unsigned long long bal = __ballot((d >> bit) & 1u);
    same &= ((d >> bit) & 1u) ? bal : ~bal;
  }
  return same;
}

// One stable scatter pass (digit at `shift`) over the first *count pairs;
// workgroups claim tiles until none is left.
__global__ __launch_bounds__(kSortBS) void counted_scatter_kernel(
    const uint32_t* __restrict__ keys_in, const int32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, int32_t* __restrict__ vals_out,
    const uint32_t* __restrict__ count, int shift, const uint32_t* __restrict__ totals,
    uint32_t* __restrict__ look, uint32_t* __restrict__ tile_ctr, int32_t* __restrict__ status) {
  __shared__ uint32_t whist[kSortWaves][kRadix];  // per wave: running digit counts
  __shared__ uint32_t offset[kRadix];
  __shared__ uint32_t wsum[kSortWaves];
  __shared__ uint32_t tile_sh;
  const int64_t M = (int64_t)*count;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  // Workgroups with no tile to start on leave without touching the counter
  // (a counter that every workgroup of a large grid bumps serialises them).
  if ((int64_t)blockIdx.x * kSortTile >= M) return;
  // With no more tiles than workgroups, the first claims of the workgroups that
  // start take every tile: each leaves after its first, without a second claim.
  const bool one_each = (M + kSortTile - 1) / kSortTile <= (int64_t)gridDim.x;
  while (true) {
#pragma unroll
  for (int w = 0; w < kSortWaves; ++w) whist[w][tid] = 0u;
  if (tid == 0) tile_sh = atomicAdd(tile_ctr, 1u);
  __syncthreads();
  const int64_t tile = (int64_t)tile_sh;
  if (tile * kSortTile >= M) return;  // uniform: every tile is taken

  const int64_t base = tile * kSortTile + (int64_t)wv * kWaveKeys;
  uint32_t key[kSortIPT];
  int32_t val[kSortIPT];
  uint32_t rank[kSortIPT];
#pragma unroll
  for (int j = 0; j < kSortIPT; ++j) {
    const int64_t i = base + (int64_t)j * kWave + lane;
    key[j] = i < M ? keys_in[i] : 0u;
    val[j] = i < M ? vals_in[i] : 0;
  }
#pragma unroll
  for (int j = 0; j < kSortIPT; ++j) {
    const bool valid = base + (int64_t)j * kWave + lane < M;
    const uint32_t d = (key[j] >> shift) & (kRadix - 1);
    const unsigned long long same = match_digit(d, valid);
    const int r = lanes_below(same);
    const uint32_t before = whist[wv][d];  // this wave's keys with digit d so far
    if (valid && r == 0) whist[wv][d] = before + (uint32_t)__popcll(same);
    rank[j] = before + (uint32_t)r;
  }
  __syncthreads();

  // digit tid: prefix over the waves, this tile's count, published at once
  uint32_t cnt = 0;
#pragma unroll
  for (int w = 0; w < kSortWaves; ++w) {
    const uint32_t c = whist[w][tid];
    whist[w][tid] = cnt;
    cnt += c;
  }
  uint32_t* mine = look + tile * kRadix + tid;
  store_agent(mine, tile == 0 ? (kInclusive | cnt) : cnt + 1u);

  // keys with a smaller digit, all tiles: exclusive scan of the totals
  uint32_t digit_base;
  {
    uint32_t v = 0;
#pragma unroll
    for (int r = 0; r < kTotalsRep; ++r) v += totals[r * kTotalsStride + tid];
    uint32_t sc = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t o = __shfl_up(sc, off, kWave);
      if (lane >= off) sc += o;
    }
    if (lane == kWave - 1) wsum[wv] = sc;
    __syncthreads();
    uint32_t pre = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) pre += (w < wv) ? wsum[w] : 0u;
    digit_base = pre + sc - v;
  }

  // keys with digit tid in earlier tiles
  uint32_t excl = 0;
  if (tile > 0) {
    int64_t j = tile - 1;  // nearest predecessor not yet accounted for
    int spins = 0;
    bool done = false;
    while (!done) {
      uint32_t w[kLookWindow];
#pragma unroll
      for (int k = 0; k < kLookWindow; ++k)
        w[k] = j - k >= 0 ? load_agent(look + (j - k) * kRadix + tid) : kInclusive;
      int advanced = 0;
#pragma unroll
      for (int k = 0; k < kLookWindow; ++k) {
        if (done || advanced < k) continue;  // stopped at a tile not yet published
        if (w[k] & kInclusive) {
          excl += w[k] & ~kInclusive;  // (tile 0 is inclusive: the walk ends there)
          done = true;
        } else if (w[k] != 0u) {
          excl += w[k] - 1u;
          advanced = k + 1;
        }
      }
      if (done) break;
      if (advanced > 0) {
        j -= advanced;
        spins = 0;
        continue;
      }
      if (++spins > kSpinLimit) {
        raise_flag(status, kFlagStall);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    store_agent(mine, kInclusive | (excl + cnt));
  }
  offset[tid] = digit_base + excl;
  __syncthreads();

#pragma unroll
  for (int j = 0; j < kSortIPT; ++j) {
    const int64_t i = base + (int64_t)j * kWave + lane;
    if (i < M) {
      const uint32_t d = (key[j] >> shift) & (kRadix - 1);
      int64_t pos = (int64_t)offset[d] + whist[wv][d] + rank[j];
      pos = pos < M ? pos : M - 1;  // only after a stall (flagged) can it be out of range
      keys_out[pos] = key[j];
      vals_out[pos] = val[j];
    }
  }
  if (one_each) return;  // uniform
  __syncthreads();  // LDS is reused by the next tile
  }
}

// ---------------------------------------------------------------- re-sort
// Slots are taken in groups of 64 (one wavefront's round); a workgroup covers
// kUpdTile slots = 32 groups.  Per group: a 64-bit mask of the changed slots
// and the number of changed slots before the group.
constexpr int kUpdTile = kSortTile;
constexpr int kGroupsPerTile = kUpdTile / kWave;
constexpr int kWindowCap = 2048;  // changed pairs a workgroup stages in LDS

// Key of the particle at slot i, as the full sort computes it: the Morton code
// of its base node (of the clamped base node when !ok), with the scene index
// above bit mbits in a batch.  s: a scene at or before slot i's (advanced here).
template <class Scenes>
__device__ __forceinline__ uint32_t cell_key(const Scenes& sc, int mbits,
                                             const float* __restrict__ x, size_t Ps, int64_t i,
                                             int& s, bool& ok) {
  s = sc.of(i, s);
  const SceneGrid g = sc.grid(s);
  int b0, b1, b2;
  float t0, t1, t2;
  ok = stencil_axis(x[i], g.ox, g.inv_dx, g.nx, b0, t0);
  ok &= stencil_axis(x[Ps + i], g.oy, g.inv_dx, g.ny, b1, t1);
  ok &= stencil_axis(x[2 * Ps + i], g.oz, g.inv_dx, g.nz, b2, t2);
  return ((uint32_t)s << mbits) | morton3(b0, b1, b2);
}

// changed-slot masks, per-workgroup counts, and the order check of keys_prev;
// the first workgroups also clear the digit totals (every copy) and the tile
// counters of the changed-list sort (nothing reads them before the compaction)
template <class Scenes>
__global__ __launch_bounds__(kSortBS) void upd_mask_kernel(Scenes sc, int mbits, int64_t P,
                                                         const float* __restrict__ x,
                                                         const uint32_t* __restrict__ keys_prev,
                                                         unsigned long long* __restrict__ mask,
                                                         uint32_t* __restrict__ blk_count,
                                                         uint32_t* __restrict__ totals,
                                                         uint32_t* __restrict__ tile_ctr,
                                                         int32_t* __restrict__ status) {
  __shared__ uint32_t wcount[kSortWaves];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const size_t Ps = (size_t)P;
  for (int r = blockIdx.x; r < kTotalsRep; r += gridDim.x)
#pragma unroll
    for (int q = 0; q < kMaxPasses; ++q) totals[r * kTotalsStride + q * kRadix + threadIdx.x] = 0u;
  if (blockIdx.x == 0 && threadIdx.x < kMaxPasses) tile_ctr[threadIdx.x] = 0u;
  int s = sc.first((int64_t)blockIdx.x * kUpdTile);  // slots only grow along the rounds
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < kSortIPT; ++j) {
    const int64_t grp = (int64_t)blockIdx.x * kGroupsPerTile + j * kSortWaves + wv;
    const int64_t i = grp * kWave + lane;
    bool changed = false;
    if (i < P) {
      bool ok;
      const uint32_t key = cell_key(sc, mbits, x, Ps, i, s, ok);
      if (!ok) raise_flag(status, kFlagRange);
      const uint32_t prev = keys_prev[i];
      if (i > 0 && keys_prev[i - 1] > prev) raise_flag(status, kFlagOrder);
      changed = key != prev;
    }
    const unsigned long long m = __ballot(changed);
    if (lane == 0 && grp * kWave < P) mask[grp] = m;
    c += (uint32_t)__popcll(m);
  }
  if (lane == 0) wcount[wv] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) t += wcount[w];
    blk_count[blockIdx.x] = t;
  }
}

// Beyond this many workgroups, summing every count in every workgroup (a cost
// that grows with their square: 0.03 -> 0.08 ms at 12.5 K workgroups) loses to a
// separate one-workgroup scan.
constexpr int kFoldedScanMaxTiles = 4096;

// one workgroup: exclusive scan of the per-workgroup counts in place, total to
// *count (for more than kFoldedScanMaxTiles workgroups)
__global__ __launch_bounds__(1024) void upd_scan_kernel(uint32_t* __restrict__ blk, int n,
                                                        uint32_t* __restrict__ count) {
  __shared__ uint32_t wsum[1024 / kWave];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  uint32_t running = 0;
  for (int base = 0; base < n; base += 1024) {
    const int k = base + tid;
    const uint32_t v = k < n ? blk[k] : 0u;
    uint32_t s = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t o = __shfl_up(s, off, kWave);
      if (lane >= off) s += o;
    }
    if (lane == kWave - 1) wsum[wv] = s;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 1024 / kWave; ++w) {
      pre += (w < wv) ? wsum[w] : 0u;
      tot += wsum[w];
    }
    if (k < n) blk[k] = running + pre + s - v;
    running += tot;
    __syncthreads();
  }
  if (tid == 0) *count = running;
}

// Changed (key, index) pairs in index order, gpre[grp] = changed slots before
// the group, and what the changed list's radix sort needs: *count, the digit
// totals of every pass (added to copy b % kTotalsRep of totals, cleared by the
// mask kernel) and the
// look-back words of every tile of the changed list, cleared.  Up to
// kFoldedScanMaxTiles workgroups, each sums the per-workgroup counts itself
// (n_tiles words, a few KB, read from L2), which saves a launch for their scan;
// with `scanned`, upd_scan_kernel has already turned them into prefixes and
// written *count.
template <class Scenes>
__global__ __launch_bounds__(kSortBS) void upd_compact_kernel(
    Scenes sc, int mbits, int64_t P, int passes, const float* __restrict__ x,
    const unsigned long long* __restrict__ mask, const uint32_t* __restrict__ blk_count,
    int n_tiles, bool scanned, uint32_t* __restrict__ gpre, uint32_t* __restrict__ count,
    uint32_t* __restrict__ look, uint32_t* __restrict__ totals, uint32_t* __restrict__ ck,
    int32_t* __restrict__ cv) {
  __shared__ uint32_t pre_sh[kGroupsPerTile];
  __shared__ uint32_t wsum[2][kSortWaves];
  __shared__ uint32_t hist[kMaxPasses * kRadix];
  __shared__ int any_sh;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  const int b = (int)blockIdx.x;

  // changed slots in the workgroups before this one, and in all
  uint32_t before = 0, all = 0;
  if (scanned) {
    before = blk_count[b];
    all = *count;
  } else {
    for (int k0 = 0; k0 < n_tiles; k0 += 4 * kSortBS) {
      uint32_t c[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + u * kSortBS + tid;
        c[u] = k < n_tiles ? blk_count[k] : 0u;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        all += c[u];
        before += k0 + u * kSortBS + tid < b ? c[u] : 0u;
      }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
      before += __shfl_xor(before, off, kWave);
      all += __shfl_xor(all, off, kWave);
    }
    if (lane == 0) {
      wsum[0][wv] = before;
      wsum[1][wv] = all;
    }
    __syncthreads();
    before = 0;
    all = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) {
      before += wsum[0][w];
      all += wsum[1][w];
    }
    if (b == 0 && tid == 0) *count = all;
  }
  // tile b of the changed list exists: clear its look-back words
  if ((int64_t)b * kSortTile < (int64_t)all)
    for (int q = 0; q < passes; ++q) look[((size_t)q * n_tiles + b) * kRadix + tid] = 0u;

  const int64_t n_groups = (P + kWave - 1) / kWave;
  const int64_t g0 = (int64_t)b * kGroupsPerTile;
  if (wv == 0) {
    const bool in = lane < kGroupsPerTile && g0 + lane < n_groups;
    const uint32_t c = in ? (uint32_t)__popcll(mask[g0 + lane]) : 0u;
    const bool any = __ballot(c != 0u) != 0ull;  // every lane of wave 0 takes part
    if (lane == 0) any_sh = any;
    uint32_t s = c;
#pragma unroll
    for (int off = 1; off < kGroupsPerTile; off <<= 1) {
      const uint32_t o = __shfl_up(s, off, kWave);
      if (lane >= off) s += o;
    }
    const uint32_t p = before + s - c;
    if (lane < kGroupsPerTile) pre_sh[lane] = p;
    if (in) gpre[g0 + lane] = p;
  }
#pragma unroll
  for (int q = 0; q < kMaxPasses; ++q) hist[q * kRadix + tid] = 0u;
  __syncthreads();
  if (!any_sh) return;  // uniform: no changed slot in this workgroup
  const size_t Ps = (size_t)P;
  int s = sc.first(g0 * kWave);
  unsigned long long m[kSortIPT];
#pragma unroll
  for (int j = 0; j < kSortIPT; ++j) {
    const int64_t grp = g0 + j * kSortWaves + wv;
    m[j] = grp < n_groups ? mask[grp] : 0ull;
  }
#pragma unroll
  for (int j = 0; j < kSortIPT; ++j) {
    if ((m[j] >> lane) & 1ull) {
      const int k = j * kSortWaves + wv;
      const int64_t i = (g0 + k) * kWave + lane;
      bool ok;
      const uint32_t pos = pre_sh[k] + (uint32_t)lanes_below(m[j]);
      const uint32_t key = cell_key(sc, mbits, x, Ps, i, s, ok);
      ck[pos] = key;
      cv[pos] = (int32_t)i;
      for (int q = 0; q < passes; ++q) atomicAdd(&hist[q * kRadix + ((key >> (8 * q)) & 255u)], 1u);
    }
  }
  __syncthreads();
  uint32_t* copy = totals + (size_t)(b % kTotalsRep) * kTotalsStride;
  for (int q = 0; q < passes; ++q) {
    const uint32_t c = hist[q * kRadix + tid];
    if (c) atomicAdd(&copy[q * kRadix + tid], c);
  }
}

// changed slots before slot s (0 <= s <= P)
__device__ __forceinline__ int64_t changed_before(int64_t s, int64_t P, uint32_t M,
                                                  const unsigned long long* __restrict__ mask,
                                                  const uint32_t* __restrict__ gpre) {
  if (s >= P) return M;
  const int64_t grp = s / kWave;
  const int bit = (int)(s % kWave);
  const unsigned long long below = bit ? (mask[grp] & ((1ull << bit) - 1ull)) : 0ull;
  return (int64_t)gpre[grp] + __popcll(below);
}

// first changed pair in [lo, hi) not below (key, idx)
template <class KeyAt, class IdxAt>
__device__ __forceinline__ int lower_pair(KeyAt kat, IdxAt iat, int lo, int hi, uint32_t key,
                                          int64_t idx) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const uint32_t k = kat(mid);
    if (k < key || (k == key && iat(mid) < idx))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// The same found by a whole wavefront (every lane calls it with the same
// arguments): each round samples 64 evenly spaced positions of the range and
// keeps the stretch between the last sample below (key, idx) and the next one,
// so a range of n shrinks to n / 64 per round trip.
template <class KeyAt, class IdxAt>
__device__ __forceinline__ int64_t wave_lower_pair(KeyAt kat, IdxAt iat, int64_t lo, int64_t hi,
                                                   uint32_t key, int64_t idx) {
  const int lane = threadIdx.x & (kWave - 1);
  while (lo < hi) {
    const int64_t stride = (hi - lo + kWave - 1) / kWave;
    const int64_t p = lo + (int64_t)lane * stride;
    bool below = false;
    if (p < hi) {
      const uint32_t k = kat(p);
      below = k < key || (k == key && (int64_t)iat(p) < idx);
    }
    const int c = __popcll(__ballot(below));  // a prefix of the samples when sorted
    if (stride == 1) return lo + c;
    if (c == 0) return lo;
    const int64_t nhi = lo + (int64_t)c * stride;
    lo = lo + (int64_t)(c - 1) * stride + 1;
    hi = nhi < hi ? nhi : hi;
  }
  return lo;
}

// Final place of every changed pair j (sorted): j changed pairs precede it,
// and so do the unchanged slots before `lo`, the first slot s whose
// (keys_prev[s], s) is not below the pair's (key, index).  Workgroup `blk` of
// `n_blk`; one pair per wavefront at a time.
__device__ __forceinline__ void place_changed(
    int blk, int n_blk, int64_t P, const uint32_t* __restrict__ keys_prev,
    const unsigned long long* __restrict__ mask, const uint32_t* __restrict__ gpre,
    const uint32_t* __restrict__ cks, const int32_t* __restrict__ cvs, uint32_t M,
    uint32_t* __restrict__ keys_out, int32_t* __restrict__ perm_out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t waves = (int64_t)n_blk * kSortWaves;
  auto pk = [&](int64_t s) { return keys_prev[s]; };
  auto ps = [&](int64_t s) { return s; };
  for (int64_t j = (int64_t)blk * kSortWaves + threadIdx.x / kWave; j < (int64_t)M;
       j += waves) {
    const uint32_t key = cks[j];
    const int32_t idx = cvs[j];
    const int64_t lo = wave_lower_pair(pk, ps, 0, P, key, idx);
    if (lane == 0) {
      int64_t pos = j + (lo - changed_before(lo, P, M, mask, gpre));
      pos = pos < 0 ? 0 : (pos >= P ? P - 1 : pos);  // in range even for unsorted keys_prev
      keys_out[pos] = key;
      perm_out[pos] = idx;
    }
  }
}

// Final place of every unchanged slot i of slot tile `blk`: its rank among the
// unchanged plus the changed pairs below (keys_prev[i], i).  The unchanged
// slots of a tile lie between (keys_prev[i0], i0) and (keys_prev[i1 - 1], i1),
// which bound the window of the changed list they can fall into; it is staged
// in LDS when it fits.
__device__ __forceinline__ void place_unchanged(
    int blk, int64_t P, const uint32_t* __restrict__ keys_prev,
    const unsigned long long* __restrict__ mask, const uint32_t* __restrict__ gpre,
    const uint32_t* __restrict__ cks, const int32_t* __restrict__ cvs, int M,
    uint32_t* __restrict__ keys_out, int32_t* __restrict__ perm_out, int* window, uint32_t* wk,
    int32_t* wi) {
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  const int64_t i0 = (int64_t)blk * kUpdTile;
  const int64_t i1 = min(i0 + (int64_t)kUpdTile, P);
  const int64_t g0 = (int64_t)blk * kGroupsPerTile;
  // The tile's own slots do not depend on the window: their loads are issued
  // first and overlap its search.  A slot past P reads as changed (skipped).
  unsigned long long mk[kSortIPT];
  uint32_t kp[kSortIPT], gp[kSortIPT];
#pragma unroll
  for (int j = 0; j < kSortIPT; ++j) {
    const int64_t grp = g0 + j * kSortWaves + wv;
    const bool in = grp * kWave + lane < P;
    mk[j] = in ? mask[grp] : ~0ull;
    kp[j] = in ? keys_prev[grp * kWave + lane] : 0u;
    gp[j] = in ? gpre[grp] : 0u;
  }
  auto gk = [&](int64_t m) { return cks[m]; };
  auto gi = [&](int64_t m) { return cvs[m]; };
  if (wv < 2) {  // waves 0 and 1: the two ends of the window
    const int64_t at = wv == 0 ? i0 : i1 - 1;
    const int64_t w = wave_lower_pair(gk, gi, 0, M, keys_prev[at], wv == 0 ? i0 : i1);
    if (lane == 0) window[wv] = (int)w;
  }
  __syncthreads();
  const int wlo = window[0];
  const int whi = max(window[0], window[1]);  // (reversed only for unsorted keys_prev)
  const int wn = whi - wlo;
  const bool staged = wn <= kWindowCap;
  if (staged) {
    for (int m = tid; m < wn; m += kSortBS) {
      wk[m] = cks[wlo + m];
      wi[m] = cvs[wlo + m];
    }
  }
  __syncthreads();
  auto sk = [&](int m) { return wk[m]; };
  auto si = [&](int m) { return wi[m]; };
#pragma unroll
  for (int j = 0; j < kSortIPT; ++j) {
    const int64_t i = (g0 + j * kSortWaves + wv) * kWave + lane;
    const unsigned long long m = mk[j];
    if ((m >> lane) & 1ull) continue;
    const uint32_t key = kp[j];
    const int below = staged ? wlo + lower_pair(sk, si, 0, wn, key, i)
                             : lower_pair(gk, gi, wlo, whi, key, i);
    const int64_t unchanged_before = i - ((int64_t)gp[j] + lanes_below(m));
    int64_t pos = unchanged_before + below;
    pos = pos < 0 ? 0 : (pos >= P ? P - 1 : pos);  // in range even for unsorted keys_prev
    keys_out[pos] = key;
    perm_out[pos] = (int32_t)i;
  }
}

// Both placements in one launch: the first kChangedBlocks workgroups place the
// changed pairs (they start first), the rest one slot tile each.
constexpr int kChangedBlocks = 1024;

__global__ __launch_bounds__(kSortBS) void upd_place_kernel(
    int64_t P, const uint32_t* __restrict__ keys_prev, const unsigned long long* __restrict__ mask,
    const uint32_t* __restrict__ gpre, const uint32_t* __restrict__ cks,
    const int32_t* __restrict__ cvs, const uint32_t* __restrict__ count,
    uint32_t* __restrict__ keys_out, int32_t* __restrict__ perm_out) {
  __shared__ int window[2];
  __shared__ uint32_t wk[kWindowCap];
  __shared__ int32_t wi[kWindowCap];
  const uint32_t M = *count;
  if ((int)blockIdx.x < kChangedBlocks)
    place_changed((int)blockIdx.x, kChangedBlocks, P, keys_prev, mask, gpre, cks, cvs, M,
                  keys_out, perm_out);
  else
    place_unchanged((int)blockIdx.x - kChangedBlocks, P, keys_prev, mask, gpre, cks, cvs, (int)M,
                    keys_out, perm_out, window, wk, wi);
}

struct UpdLayout {
  unsigned long long* mask;
  uint32_t *blk, *gpre, *count, *ck0, *ck1, *look, *totals, *tile_ctr;
  int32_t *cv0, *cv1;
  size_t bytes;
};

UpdLayout upd_layout(void* ws, int64_t P) {
  const int64_t n_tiles = (P + kSortTile - 1) / kSortTile;
  const int64_t n_groups = (P + kWave - 1) / kWave;
  char* w = (char*)ws;
  UpdLayout L;
  size_t off = 0;
  auto take = [&](size_t n) {
    char* q = w ? w + off : nullptr;
    off += align_up(n);
    return q;
  };
  L.mask = (unsigned long long*)take((size_t)n_groups * 8);
  L.blk = (uint32_t*)take((size_t)n_tiles * 4);
  L.gpre = (uint32_t*)take((size_t)n_groups * 4);
  L.count = (uint32_t*)take(4);
  L.ck0 = (uint32_t*)take((size_t)P * 4);
  L.cv0 = (int32_t*)take((size_t)P * 4);
  L.ck1 = (uint32_t*)take((size_t)P * 4);
  L.cv1 = (int32_t*)take((size_t)P * 4);
  L.look = (uint32_t*)take((size_t)kMaxPasses * n_tiles * kRadix * 4);
  L.totals = (uint32_t*)take((size_t)kTotalsRep * kTotalsStride * 4);
  L.tile_ctr = (uint32_t*)take((size_t)kMaxPasses * 4);
  L.bytes = off;
  return L;
}

}  // namespace

size_t sort_update_workspace_bytes(int64_t P) { return upd_layout(nullptr, P).bytes; }

namespace {

template <class Scenes>
hipError_t sort_update_with(const Scenes& sc, int mbits, int key_bits, int64_t P,
                            const float* x, const uint32_t* keys_prev, uint32_t* keys_out,
                            int32_t* perm_out, void* ws, int32_t* status, hipStream_t stream) {
  if (P == 0) return hipSuccess;
  const UpdLayout L = upd_layout(ws, P);
  const int n_tiles = (int)((P + kSortTile - 1) / kSortTile);
  const int passes = (key_bits + 7) / 8;
  if (passes < 1 || passes > kMaxPasses) return hipErrorInvalidValue;
  upd_mask_kernel<Scenes><<<n_tiles, kSortBS, 0, stream>>>(sc, mbits, P, x, keys_prev, L.mask,
                                                           L.blk, L.totals, L.tile_ctr, status);
  const bool scanned = n_tiles > kFoldedScanMaxTiles;
  if (scanned) upd_scan_kernel<<<1, 1024, 0, stream>>>(L.blk, n_tiles, L.count);
  upd_compact_kernel<Scenes><<<n_tiles, kSortBS, 0, stream>>>(
      sc, mbits, P, passes, x, L.mask, L.blk, n_tiles, scanned, L.gpre, L.count, L.look,
      L.totals, L.ck0, L.cv0);
  // stable radix sort of the changed pairs (their number known on the device only)
  const int counted_grid = n_tiles < kCountedGrid ? n_tiles : kCountedGrid;
  uint32_t* ks = L.ck0;
  int32_t* vs = L.cv0;
  uint32_t* kd = L.ck1;
  int32_t* vd = L.cv1;
  for (int pass = 0; pass < passes; ++pass) {
    counted_scatter_kernel<<<counted_grid, kSortBS, 0, stream>>>(
        ks, vs, kd, vd, L.count, 8 * pass, L.totals + pass * kRadix,
        L.look + (size_t)pass * n_tiles * kRadix, L.tile_ctr + pass, status);
    uint32_t* kt = ks;
    ks = kd;
    kd = kt;
    int32_t* vt = vs;
    vs = vd;
    vd = vt;
  }
  upd_place_kernel<<<kChangedBlocks + n_tiles, kSortBS, 0, stream>>>(
      P, keys_prev, L.mask, L.gpre, ks, vs, L.count, keys_out, perm_out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sort_update(const GridDev& g, int64_t P, const float* x,
                              const uint32_t* keys_prev, uint32_t* keys_out, int32_t* perm_out,
                              void* ws, int32_t* status, hipStream_t stream) {
  OneScene one;
  one.sg.nx = g.nx;
  one.sg.ny = g.ny;
  one.sg.nz = g.nz;
  one.sg.inv_dx = g.inv_dx;
  one.sg.ox = g.ox;
  one.sg.oy = g.oy;
  one.sg.oz = g.oz;
  one.sg.dx = 0.0f;
  for (int k = 0; k < 3; ++k) one.sg.lo[k] = one.sg.hi[k] = 0.0f;
  one.sg.node_off = 0;
  const int bits = sort_key_bits(g);
  return sort_update_with(one, bits, bits, P, x, keys_prev, keys_out, perm_out, ws, status,
                          stream);
}

hipError_t launch_sort_update_batch(const SceneDev* table, int n_scenes, int mbits, int key_bits,
                                    int64_t P, const float* x, const uint32_t* keys_prev,
                                    uint32_t* keys_out, int32_t* perm_out, void* ws,
                                    int32_t* status, hipStream_t stream) {
  SceneTable st{table, n_scenes};
  return sort_update_with(st, mbits, key_bits, P, x, keys_prev, keys_out, perm_out, ws, status,
                          stream);
}

}  // namespace polypic
