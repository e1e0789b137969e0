// Cell-key computation and stable LSD radix sort (8-bit digits) for gfx950.
//
// Each pass: (1) per-tile digit histograms, (2) per-digit exclusive scan over
// tiles, (3) a stable scatter in which every tile ranks its keys in input
// order -- within a wavefront by ballot matching of equal digits, across the
// wavefronts of the block through small LDS histograms.  Ties keep input
// order, so the result equals a stable argsort of the keys.
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

}  // namespace polypic
