// Counting sort of particles by grid tile (support for the tiled deposition).
//
// Tiles are kTile^3 blocks of cells (partial at the upper end of an axis); particles
// with an out-of-range cell index go to one extra bucket after the last tile so
// the sorted order has no holes (they are counted and never deposited).  Three
// launches: count per tile, exclusive scan of the counts, rank (each particle's
// slot in tile order).  Particles that share a tile within a wavefront are
// combined before touching the tile counter, so a wave issues one atomic per
// distinct tile: with particles already grouped by tile (the previous step's
// order) that is one or two atomics per wave instead of 64.
#include "kernels.h"

namespace pic {

namespace {

__device__ inline uint32_t fdiv(uint32_t n, const FastDiv& f) { return (__umulhi(n, f.m) + n) >> f.s; }

__device__ inline int tile_key(int c, const GridGeom& g, const TileGeom& t) {
  if (c < 0 || c >= g.nx * g.ny * g.nz) return t.ntiles;
  const int r = (int)fdiv((uint32_t)c, g.nz_div);
  const int k = c - r * g.nz;
  const int i = (int)fdiv((uint32_t)r, g.ny_div);
  const int j = r - i * g.ny;
  return ((i / kTile) * t.nty + j / kTile) * t.ntz + k / kTile;
}

// Adds one per valid lane to counters[key]; returns each lane's previous-value
// slot (counter value before the lane's increment, lanes of one key in lane order).
// The lanes are first grouped by key (ballots only); then the first lane of every group
// issues the group's atomic, all groups' atomics in the same instruction, so a wave waits
// for one atomic round trip however many distinct keys it holds.
__device__ inline int wave_aggregated_add(int* counters, int key, bool valid) {
  unsigned long long active = __ballot(valid);
  const int lane = __lane_id();
  int leader_of = lane, rank = 0, group = 0;
  while (active) {
    const int leader = __ffsll((unsigned long long)active) - 1;
    const int lkey = __shfl(key, leader);
    const unsigned long long same = __ballot(valid && key == lkey) & active;
    if ((same >> lane) & 1ull) {
      leader_of = leader;
      rank = __popcll(same & ((1ull << lane) - 1ull));
    }
    if (lane == leader) group = __popcll(same);
    active &= ~same;
  }
  int base = 0;
  if (valid && lane == leader_of) base = atomicAdd(&counters[key], group);
  base = __shfl(base, leader_of);
  return valid ? base + rank : -1;
}

// The same count without the slots: the atomics' results are not waited for.
__device__ inline void wave_aggregated_count(int* counters, int key, bool valid) {
  unsigned long long active = __ballot(valid);
  const int lane = __lane_id();
  int group = 0;
  while (active) {
    const int leader = __ffsll((unsigned long long)active) - 1;
    const int lkey = __shfl(key, leader);
    const unsigned long long same = __ballot(valid && key == lkey) & active;
    if (lane == leader) group = __popcll(same);
    active &= ~same;
  }
  if (group > 0) atomicAdd(&counters[key], group);
}

__global__ void __launch_bounds__(256) k_tile_count(GridGeom g, TileGeom t, const int32_t* __restrict__ cell, long long n,
                                                    int* counts) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int key = (p < n) ? tile_key(cell[p], g, t) : 0;
  wave_aggregated_count(counts, key, p < n);
}

__global__ void __launch_bounds__(256) k_tile_rank(GridGeom g, TileGeom t, const int32_t* __restrict__ cell, long long n,
                                                   int* cursor, int* dst, int* bad) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int key = (p < n) ? tile_key(cell[p], g, t) : 0;
  const int slot = wave_aggregated_add(cursor, key, p < n);
  if (p < n) {
    if (key == t.ntiles && bad) atomicAdd(bad, 1);
    dst[p] = slot;
  }
}

// The same two passes with a per-workgroup histogram in LDS (grids of at most
// kSortMaxBuckets - 1 tiles): each workgroup counts its kSortBlock * kSortPer particles
// per tile in LDS and touches each global counter once per tile it holds, so a counter
// sees a few atomics per step instead of one per wave (atomics on one address serialise).
// For the ranks, a workgroup reserves one run per tile on ``cursor`` and places its
// particles in the run by their LDS ranks.
constexpr int kSortBlock = 1024, kSortPer = 8;
constexpr int kSortMaxBuckets = 32768;  // 128 KiB of LDS counters

__global__ void __launch_bounds__(kSortBlock) k_tile_count_lds(GridGeom g, TileGeom t, const int32_t* __restrict__ cell,
                                                               long long n, int* counts) {
  extern __shared__ int hist[];
  const int nbk = t.ntiles + 1;
  for (int e = threadIdx.x; e < nbk; e += blockDim.x) hist[e] = 0;
  __syncthreads();
  const long long p0 = (long long)blockIdx.x * kSortBlock * kSortPer + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kSortPer; ++u) {
    const long long p = p0 + (long long)u * kSortBlock;
    const int key = (p < n) ? tile_key(cell[p], g, t) : 0;
    wave_aggregated_count(hist, key, p < n);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nbk; e += blockDim.x) {
    const int c = hist[e];
    if (c) atomicAdd(&counts[e], c);
  }
}

__global__ void __launch_bounds__(kSortBlock) k_tile_rank_lds(GridGeom g, TileGeom t, const int32_t* __restrict__ cell,
                                                              long long n, int* cursor, int* dst, int* bad) {
  extern __shared__ int hist[];
  const int nbk = t.ntiles + 1;
  for (int e = threadIdx.x; e < nbk; e += blockDim.x) hist[e] = 0;
  __syncthreads();
  const long long p0 = (long long)blockIdx.x * kSortBlock * kSortPer + threadIdx.x;
  int key[kSortPer], rank[kSortPer];
#pragma unroll
  for (int u = 0; u < kSortPer; ++u) {
    const long long p = p0 + (long long)u * kSortBlock;
    key[u] = (p < n) ? tile_key(cell[p], g, t) : 0;
    rank[u] = wave_aggregated_add(hist, key[u], p < n);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nbk; e += blockDim.x) {
    const int c = hist[e];
    if (c) hist[e] = atomicAdd(&cursor[e], c);  // this workgroup's run of tile e
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kSortPer; ++u) {
    const long long p = p0 + (long long)u * kSortBlock;
    if (p < n) {
      if (key[u] == t.ntiles && bad) atomicAdd(bad, 1);
      dst[p] = hist[key[u]] + rank[u];
    }
  }
}

// Exclusive scan of counts[0..m) into starts[0..m] (starts[m] = the total) and cursor[0..m)
// by blocks of 1024 threads, in chunks of 1024 x 8 entries: thread t takes the 8 adjacent
// entries at the chunk's base + 8 t (the block's loads and stores cover contiguous memory),
// and the block scans the thread sums (a scan within each wave, then over the 16 wave totals).
constexpr int kScanPer = 8;
constexpr int kScanChunk = 1024 * kScanPer;
constexpr int kScanWaves = 1024 / 64;

// One chunk from ``carry`` (the sum of everything before it); returns the chunk's total.
// Every thread of the block calls it.
__device__ inline int scan_chunk(const int* __restrict__ counts, int* starts, int* cursor, int m, int base, int carry,
                                 int* wsum) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = base + tid * kScanPer;
  int v[kScanPer];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = (i0 + k < m) ? counts[i0 + k] : 0;
    s += v[k];
  }
  int x = s;  // inclusive scan of the thread sums within the wave
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  if (wave == 0) {  // inclusive scan of the wave totals
    int w = lane < kScanWaves ? wsum[lane] : 0;
#pragma unroll
    for (int o = 1; o < kScanWaves; o <<= 1) {
      const int y = __shfl_up(w, o, 64);
      if (lane >= o) w += y;
    }
    if (lane < kScanWaves) wsum[lane] = w;
  }
  __syncthreads();
  int run = carry + (wave > 0 ? wsum[wave - 1] : 0) + x - s;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (i0 + k < m) {
      starts[i0 + k] = run;
      cursor[i0 + k] = run;
      run += v[k];
    }
  }
  const int total = wsum[kScanWaves - 1];
  __syncthreads();  // wsum is rewritten by the next chunk
  return total;
}

// Up to two chunks (m <= 2 kScanChunk), one block: thread t scans its own run of at most 16
// adjacent entries serially, the block scans the run totals (one launch beats three there).
__global__ void __launch_bounds__(1024) k_scan(const int* __restrict__ counts, int* starts, int* cursor, int m) {
  __shared__ int part[1024];
  const int tid = threadIdx.x;
  const int chunk = (m + blockDim.x - 1) / blockDim.x;
  const int lo = min(m, tid * chunk), hi = min(m, lo + chunk);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += counts[i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const int v = (tid >= off) ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int run = part[tid] - s;  // exclusive prefix of this run
  for (int i = lo; i < hi; ++i) {
    starts[i] = run;
    cursor[i] = run;
    run += counts[i];
  }
  if (tid == blockDim.x - 1) starts[m] = part[tid];
}

// Large m, first of three launches: sums[b] = the total of chunk b.
__global__ void __launch_bounds__(1024) k_scan_sums(const int* __restrict__ counts, int m, int* sums) {
  __shared__ int wsum[kScanWaves];
  const int base = blockIdx.x * kScanChunk, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int i = base + k * 1024 + (int)threadIdx.x;
    if (i < m) s += counts[i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) wsum[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kScanWaves; ++w) t += wsum[w];
    sums[blockIdx.x] = t;
  }
}

// Second launch (one block, nb <= 1024): sums -> their exclusive scan in place; *total = the sum.
__global__ void __launch_bounds__(1024) k_scan_offsets(int* sums, int nb, int* total) {
  __shared__ int wsum[kScanWaves];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int v = tid < nb ? sums[tid] : 0;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wave; ++w) before += wsum[w];
  if (tid < nb) sums[tid] = before + x - v;
  if (tid == 1023) *total = before + x;
}

// One block over every chunk in turn (the fallback without scratch).
__global__ void __launch_bounds__(1024) k_scan_apply_serial(const int* __restrict__ counts, int* starts, int* cursor,
                                                            int m) {
  __shared__ int wsum[kScanWaves];
  int carry = 0;
  for (int base = 0; base < m; base += kScanChunk) carry += scan_chunk(counts, starts, cursor, m, base, carry, wsum);
  if (threadIdx.x == 0) starts[m] = carry;
}

// Third launch: block b scans chunk b from its offset.
__global__ void __launch_bounds__(1024) k_scan_apply(const int* __restrict__ counts, int* starts, int* cursor, int m,
                                                     const int* __restrict__ offsets) {
  __shared__ int wsum[kScanWaves];
  (void)scan_chunk(counts, starts, cursor, m, blockIdx.x * kScanChunk, offsets[blockIdx.x], wsum);
}

// For every destination tile D of the new grouping: the slot runs of the particles that
// arrive from each neighbour source tile S (grouped by S in the previous step), in the
// order of the 27 offsets, from starts[D]; bases[27 S + nb] receives the start of the run
// of S's particles whose offset to D is nb, cursor[D] the first slot after all runs.
// An offset that names the same S as another (grids of one or two tiles along an axis)
// is taken once, with the index the particle kernels compute for it.
// One 32-lane group per destination tile D; lane o < 27 takes the offset o, its source
// tile and count, and a scan across the group places the runs.
__global__ void __launch_bounds__(256) k_neighbour_bases(TileGeom t, const int* __restrict__ old_starts,
                                                         const int* __restrict__ nbr_counts,
                                                         const int* __restrict__ new_starts, int* bases, int* cursor) {
  const int D = (blockIdx.x * blockDim.x + threadIdx.x) >> 5;
  const int o = threadIdx.x & 31;
  if (D >= t.ntiles) return;  // whole 32-lane groups leave together
  const int dz = D % t.ntz, dy = (D / t.ntz) % t.nty, dx = D / (t.ntz * t.nty);
  const int nt[3] = {t.ntx, t.nty, t.ntz};
  const int dc[3] = {dx, dy, dz};
  const int off[3] = {o / 9 - 1, (o / 3) % 3 - 1, o % 3 - 1};
  int sc[3], canon = 0;
  for (int a = 0; a < 3; ++a) {
    sc[a] = (dc[a] - off[a] + nt[a]) % nt[a];
    int d = dc[a] - sc[a];  // as the particle kernels wrap it
    if (d > 1) d -= nt[a];
    if (d < -1) d += nt[a];
    canon = canon * 3 + (d + 1);
  }
  const int S = (sc[0] * t.nty + sc[1]) * t.ntz + sc[2];
  const bool take = o < 27 && canon == o;
  const int Sv = take ? S : 0;
  const int s0 = old_starts[Sv], s1 = old_starts[Sv + 1];  // an empty tile published no counts
  const int cv = nbr_counts[27 * Sv + (take ? o : 0)];
  const int c = (take && s0 != s1) ? cv : 0;
  int x = c;  // inclusive scan over the group
  for (int k = 1; k < 32; k <<= 1) {
    const int y = __shfl_up(x, k, 32);
    if (o >= k) x += y;
  }
  const int run0 = new_starts[D];
  if (take && s0 != s1) bases[27 * S + o] = run0 + x - c;
  if (o == 31) cursor[D] = run0 + x;
}

__global__ void __launch_bounds__(256) k_invert(const int* __restrict__ dst, int* perm, long long n) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) perm[dst[p]] = (int)p;
}

}  // namespace

FastDiv make_fastdiv(uint32_t d) {
  FastDiv f{d, 0u, 0u};
  while ((1ull << f.s) < d) ++f.s;
  f.m = (uint32_t)((((1ull << 32) * ((1ull << f.s) - d)) / d) + 1);
  return f;
}

GridGeom make_geom(int nx, int ny, int nz, double dx, double dy, double dz, double dt, int shape_order) {
  GridGeom g{nx, ny, nz, dx, dy, dz, dt, shape_order, make_fastdiv((uint32_t)ny), make_fastdiv((uint32_t)nz),
             0.0, 0.0, 0.0, 0};
  return g;
}

TileGeom make_tiles(const GridGeom& g) {
  TileGeom t{};
  t.ntx = (g.nx + kTile - 1) / kTile;
  t.nty = (g.ny + kTile - 1) / kTile;
  t.ntz = (g.nz + kTile - 1) / kTile;
  t.ntiles = t.ntx * t.nty * t.ntz;
  return t;
}

// The exclusive scan of the ntiles + 1 bucket counts: one block for up to two chunks, else
// the three-launch form through t.scan_tmp (up to 1024 chunks: every grid pic_init accepts).
void scan_buckets(const TileGeom& t, const int* counts, int* starts, int* cursor, hipStream_t s) {
  const int m = t.ntiles + 1;
  const int nb = (m + kScanChunk - 1) / kScanChunk;
  if (nb <= 2) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, starts, cursor, m);
    return;
  }
  if (nb > 1024 || !t.scan_tmp) {  // not reached through pic_init: a chunk per block in turn would be needed
    hipLaunchKernelGGL(k_scan_apply_serial, dim3(1), dim3(1024), 0, s, counts, starts, cursor, m);
    return;
  }
  hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(1024), 0, s, counts, m, t.scan_tmp);
  hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(1024), 0, s, t.scan_tmp, nb, starts + m);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(1024), 0, s, counts, starts, cursor, m,
                     (const int*)t.scan_tmp);
}

void tile_sort(const GridGeom& g, const TileGeom& t, const int32_t* cell, int64_t n, int* counts, int* starts,
               int* cursor, int* dst, int* bad, hipStream_t s) {
  // buckets 0..ntiles-1 are tiles, bucket ntiles collects invalid cells
  (void)hipMemsetAsync(counts, 0, sizeof(int) * (t.ntiles + 1), s);
  if (t.ntiles + 1 <= kSortMaxBuckets) {
    const size_t lds = sizeof(int) * (size_t)(t.ntiles + 1);
    const unsigned nbl = (unsigned)((n + kSortBlock * kSortPer - 1) / (kSortBlock * kSortPer));
    if (lds > 64 * 1024) {
      (void)hipFuncSetAttribute((const void*)k_tile_count_lds, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      (void)hipFuncSetAttribute((const void*)k_tile_rank_lds, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    }
    if (n > 0)
      hipLaunchKernelGGL(k_tile_count_lds, dim3(nbl), dim3(kSortBlock), lds, s, g, t, cell, (long long)n, counts);
    scan_buckets(t, counts, starts, cursor, s);
    if (n > 0)
      hipLaunchKernelGGL(k_tile_rank_lds, dim3(nbl), dim3(kSortBlock), lds, s, g, t, cell, (long long)n, cursor, dst,
                         bad);
    return;
  }
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (n > 0) hipLaunchKernelGGL(k_tile_count, dim3(nb), dim3(256), 0, s, g, t, cell, (long long)n, counts);
  scan_buckets(t, counts, starts, cursor, s);
  if (n > 0) hipLaunchKernelGGL(k_tile_rank, dim3(nb), dim3(256), 0, s, g, t, cell, (long long)n, cursor, dst, bad);
}

void scan_counts(const TileGeom& t, const int* counts, int* starts, int* cursor, hipStream_t s) {
  scan_buckets(t, counts, starts, cursor, s);
}

void neighbour_bases(const TileGeom& t, const int* old_starts, const int* nbr_counts, const int* new_starts,
                     int* bases, int* cursor, hipStream_t s) {
  hipLaunchKernelGGL(k_neighbour_bases, dim3((unsigned)((t.ntiles + 7) / 8)), dim3(256), 0, s, t, old_starts,
                     nbr_counts, new_starts, bases, cursor);
}

void invert_perm(const int* dst, int* perm, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_invert, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, perm, (long long)n);
}

}  // namespace pic
