// Particle kernels of the hybrid cycle (Sec. 2): momentum-conserving gather from
// the nodal grid + relativistic Boris push, and charge/current deposition on the
// nodal grid.  Because every nodal component sits at the same points, one set of
// B-spline weights serves all six gathered components and all four deposited ones.
//
// Shapes (centred B-splines; the paper's runs use cubic splines, Sec. 5.2/5.3):
//   order 1 (CIC): nodes i, i+1 with weights 1-d, d;
//   order 3:       nodes i-1..i+2 with (1-d)^3/6, 2/3-d^2+d^3/2, 2/3-(1-d)^2+(1-d)^3/2, d^3/6,
// d in [0,1) the offset of the particle from node i along the axis.
// Positions are an integer cell plus an offset in [0,1): the offset carries the
// full precision of the dtype everywhere in the box.
#include <algorithm>

#include "kernels.h"

#ifndef PIC_GATHER_BLOCK
#define PIC_GATHER_BLOCK 512
#endif
#ifndef PIC_DEPOSIT_BLOCK
#define PIC_DEPOSIT_BLOCK 512
#endif

namespace pic {

namespace {

template <typename T, int ORDER>
struct Shape;

template <typename T>
struct Shape<T, 1> {
  static constexpr int NW = 2;
  static constexpr int BASE = 0;
  __device__ static inline void weights(T d, T* w) {
    w[0] = (T)1 - d;
    w[1] = d;
  }
};

template <typename T>
struct Shape<T, 3> {
  static constexpr int NW = 4;
  static constexpr int BASE = -1;
  __device__ static inline void weights(T d, T* w) {
    const T e = (T)1 - d;
    const T sixth = (T)1 / (T)6;
    const T twothird = (T)2 / (T)3;
    w[0] = sixth * e * e * e;
    w[1] = twothird - d * d + (T)0.5 * d * d * d;
    w[2] = twothird - e * e + (T)0.5 * e * e * e;
    w[3] = sixth * d * d * d;
  }
};

__device__ inline int wrapi(int i, int n) {
  i = (i < 0) ? i + n : i;
  return (i >= n) ? i - n : i;
}

// periodic index for any integer (used where the shift comes from caller data)
__device__ inline int modi(int i, int n) {
  i %= n;
  return (i < 0) ? i + n : i;
}

// Decodes a linear cell index; returns false (and counts the particle) when it is out of range.
__device__ inline bool decode_cell(int c, const GridGeom& g, int* bad, int& i, int& j, int& k) {
  if (c < 0 || c >= g.nx * g.ny * g.nz) {
    if (bad) atomicAdd(bad, 1);
    return false;
  }
  k = c % g.nz;
  const int t = c / g.nz;
  j = t % g.ny;
  i = t / g.ny;
  return true;
}

// offset + displacement (in cells) -> (new offset in [0,1), integer shift), |displacement| < 1.
template <typename T>
__device__ inline int advance_offset(T& off, T disp) {
  T o = off + disp;
  T f = floor(o);
  o -= f;
  // a finite, in-range offset moves by less than one cell; anything else is clamped
  int sh = (f > (T)1 || f < (T)-1 || f != f) ? 0 : (int)f;
  if (f != (T)sh) o = (T)0;
  if (o >= (T)1) {  // rounding of o - floor(o) for tiny negative o
    o -= (T)1;
    sh += 1;
  }
  off = o;
  return sh;
}

// ---------------------------------------------------------------- tiles

__device__ inline void tile_coords(int tile, const TileGeom& tg, int& tx, int& ty, int& tz) {
  tz = tile % tg.ntz;
  const int r = tile / tg.ntz;
  ty = r % tg.nty;
  tx = r / tg.nty;
}

__device__ inline int tile_of(int i, int j, int k, const TileGeom& tg) {
  return ((i / tg.ts) * tg.nty + j / tg.ts) * tg.ntz + k / tg.ts;
}

// Index 0..26 of ``key`` among the 27 tiles around (tx, ty, tz) (periodic), or -1.
__device__ inline int neighbour_index(int key, int tx, int ty, int tz, const TileGeom& tg) {
  int kx, ky, kz;
  tile_coords(key, tg, kx, ky, kz);
  int d[3] = {kx - tx, ky - ty, kz - tz};
  const int nt[3] = {tg.ntx, tg.nty, tg.ntz};
  for (int a = 0; a < 3; ++a) {
    if (d[a] > 1) d[a] -= nt[a];
    if (d[a] < -1) d[a] += nt[a];
    if (d[a] < -1 || d[a] > 1) return -1;
  }
  return ((d[0] + 1) * 3 + (d[1] + 1)) * 3 + (d[2] + 1);
}

__device__ inline int neighbour_key(int nb, int tx, int ty, int tz, const TileGeom& tg) {
  const int dx = nb / 9 - 1, dy = (nb / 3) % 3 - 1, dz = nb % 3 - 1;
  return (modi(tx + dx, tg.ntx) * tg.nty + modi(ty + dy, tg.nty)) * tg.ntz + modi(tz + dz, tg.ntz);
}

// box-local index (0 .. B-1) of the first support node of a particle in cell i of a
// tile starting at cell t0, for boxes whose node 0 is t0 - 1 + BASE (one-cell
// margin); -1 if the particle is outside the margin.
__device__ inline int box_index(int i, int t0, int n, int ts) {
  int l = (i - t0 + 1) % n;
  if (l < 0) l += n;
  return (l <= ts + 1) ? l : -1;
}

// ---------------------------------------------------------------- gather + push

// Nodal field box in LDS, node-major with the six components adjacent (8 slots for
// float: two 16-byte reads per node; 6 for double: three 16-byte reads).
template <typename T>
struct FieldSlots;
template <>
struct FieldSlots<float> {
  static constexpr int FS = 8;
  __device__ static inline void read(const float* p, float* v) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    const float2 b = *reinterpret_cast<const float2*>(p + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y;
  }
};
template <>
struct FieldSlots<double> {
  static constexpr int FS = 6;
  __device__ static inline void read(const double* p, double* v) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    const double2 c = *reinterpret_cast<const double2*>(p + 4);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y; v[4] = c.x; v[5] = c.y;
  }
};

// Stages the six nodal components over the B^3 box of tile (t0x, t0y, t0z).
template <typename T, int ORDER>
__device__ inline void load_field_box(T* box, const Batch<const T*>& F, const GridGeom& g, int t0x, int t0y, int t0z,
                                      int B) {
  using S = Shape<T, ORDER>;
  constexpr int FS = FieldSlots<T>::FS;
  const int ox0 = t0x - 1 + S::BASE, oy0 = t0y - 1 + S::BASE, oz0 = t0z - 1 + S::BASE;
  const int B3 = B * B * B;
  for (int e = threadIdx.x; e < B3; e += blockDim.x) {
    const int lx = e / (B * B), ly = (e / B) % B, lz = e % B;
    const size_t gi = ((size_t)modi(ox0 + lx, g.nx) * g.ny + modi(oy0 + ly, g.ny)) * g.nz + modi(oz0 + lz, g.nz);
#pragma unroll
    for (int c = 0; c < 6; ++c) box[e * FS + c] = F.p[c][gi];
  }
}

// Gather at one particle from the LDS box (first support node at box index l*) or,
// outside the margin, from the grid; then the relativistic Boris push and the move.
template <typename T, int ORDER>
__device__ inline void gather_push_one(const T* box, int B, const Batch<const T*>& F, const GridGeom& g, int lx, int ly,
                                       int lz, int& i, int& j, int& k, T& ox, T& oy, T& oz, T& ux, T& uy, T& uz,
                                       T qdt2m, T dtx, T dty, T dtz) {
  using S = Shape<T, ORDER>;
  constexpr int NW = S::NW;
  constexpr int FS = FieldSlots<T>::FS;
  T wx[NW], wy[NW], wz[NW];
  S::weights(ox, wx);
  S::weights(oy, wy);
  S::weights(oz, wz);
  T f[6] = {0, 0, 0, 0, 0, 0};
  if (lx >= 0 && ly >= 0 && lz >= 0) {
#pragma unroll
    for (int a = 0; a < NW; ++a) {
#pragma unroll
      for (int b = 0; b < NW; ++b) {
        const int row = ((lx + a) * B + (ly + b)) * B + lz;
        const T wab = wx[a] * wy[b];
#pragma unroll
        for (int cc = 0; cc < NW; ++cc) {
          const T w = wab * wz[cc];
          T v[6];
          FieldSlots<T>::read(box + (size_t)(row + cc) * FS, v);
#pragma unroll
          for (int m = 0; m < 6; ++m) f[m] += w * v[m];
        }
      }
    }
  } else {
    for (int a = 0; a < NW; ++a) {
      const int ii = modi(i + a + S::BASE, g.nx);
      for (int b = 0; b < NW; ++b) {
        const int jj = modi(j + b + S::BASE, g.ny);
        const size_t row = ((size_t)ii * g.ny + jj) * g.nz;
        const T wab = wx[a] * wy[b];
        for (int cc = 0; cc < NW; ++cc) {
          const T w = wab * wz[cc];
          const size_t idx = row + modi(k + cc + S::BASE, g.nz);
          for (int m = 0; m < 6; ++m) f[m] += w * F.p[m][idx];
        }
      }
    }
  }
  // relativistic Boris (c = 1)
  const T umx = ux + qdt2m * f[0], umy = uy + qdt2m * f[1], umz = uz + qdt2m * f[2];
  const T gm = sqrt((T)1 + umx * umx + umy * umy + umz * umz);
  const T tf = qdt2m / gm;
  const T tx = tf * f[3], ty = tf * f[4], tz = tf * f[5];
  const T sf = (T)2 / ((T)1 + tx * tx + ty * ty + tz * tz);
  const T sx = sf * tx, sy = sf * ty, sz = sf * tz;
  const T upx = umx + (umy * tz - umz * ty);
  const T upy = umy + (umz * tx - umx * tz);
  const T upz = umz + (umx * ty - umy * tx);
  ux = umx + (upy * sz - upz * sy) + qdt2m * f[0];
  uy = umy + (upz * sx - upx * sz) + qdt2m * f[1];
  uz = umz + (upx * sy - upy * sx) + qdt2m * f[2];
  const T ig = (T)1 / sqrt((T)1 + ux * ux + uy * uy + uz * uz);
  i = modi(i + advance_offset(ox, dtx * ux * ig), g.nx);
  j = modi(j + advance_offset(oy, dty * uy * ig), g.ny);
  k = modi(k + advance_offset(oz, dtz * uz * ig), g.nz);
}

template <typename T>
__device__ inline void copy_particle(const SpeciesView<T>& in, long long p, const SpeciesView<T>& out, long long q) {
  out.cell[q] = in.cell[p];
  for (int d = 0; d < 3; ++d) {
    out.off[d][q] = in.off[d][p];
    out.u[d][q] = in.u[d][p];
  }
  if (in.w) out.w[q] = in.w[p];
}

// Gather + push through a permutation: one block per tile t of the particles'
// current cells, slots q in [starts[t], starts[t+1]); slot q reads particle perm[q]
// of ``in`` and writes it to slot q (write_sorted) or back to perm[q] of ``out``.
// Block ntiles carries particles with invalid cells along.
template <typename T, int ORDER>
__global__ void __launch_bounds__(PIC_GATHER_BLOCK) k_gather_push_perm(GridGeom g, TileGeom tg, Batch<const T*> F,
                                                                       SpeciesView<T> in, SpeciesView<T> out,
                                                                       const int* __restrict__ perm,
                                                                       const int* __restrict__ starts, int write_sorted,
                                                                       T qdt2m, T dtx, T dty, T dtz) {
  using S = Shape<T, ORDER>;
  extern __shared__ __align__(16) unsigned char smem[];
  T* box = reinterpret_cast<T*>(smem);
  const int tile = blockIdx.x;
  const int beg = starts[tile], end = starts[tile + 1];
  if (beg == end) return;
  if (tile == tg.ntiles) {
    for (int qq = beg + threadIdx.x; qq < end; qq += blockDim.x) {
      const int p = perm[qq];
      copy_particle(in, p, out, write_sorted ? qq : p);
    }
    return;
  }
  const int B = tg.ts + S::NW + 1;
  int tx, ty, tz;
  tile_coords(tile, tg, tx, ty, tz);
  const int t0x = tx * tg.ts, t0y = ty * tg.ts, t0z = tz * tg.ts;
  load_field_box<T, ORDER>(box, F, g, t0x, t0y, t0z, B);
  __syncthreads();
  for (int qq = beg + threadIdx.x; qq < end; qq += blockDim.x) {
    const int p = perm[qq];
    const int wi = write_sorted ? qq : p;
    int i, j, k;
    (void)decode_cell(in.cell[p], g, nullptr, i, j, k);
    T ox = in.off[0][p], oy = in.off[1][p], oz = in.off[2][p];
    T ux = in.u[0][p], uy = in.u[1][p], uz = in.u[2][p];
    const int lx = box_index(i, t0x, g.nx, tg.ts), ly = box_index(j, t0y, g.ny, tg.ts),
              lz = box_index(k, t0z, g.nz, tg.ts);
    gather_push_one<T, ORDER>(box, B, F, g, lx, ly, lz, i, j, k, ox, oy, oz, ux, uy, uz, qdt2m, dtx, dty, dtz);
    out.u[0][wi] = ux;
    out.u[1][wi] = uy;
    out.u[2][wi] = uz;
    out.off[0][wi] = ox;
    out.off[1][wi] = oy;
    out.off[2][wi] = oz;
    out.cell[wi] = (i * g.ny + j) * g.nz + k;
    if (in.w && (write_sorted || out.w != in.w)) out.w[wi] = in.w[p];
  }
}

// Steady-state gather + push of pic_step.  ``in`` is grouped by home tile h (the
// tile of the previous step's positions; slots [home[h], home[h+1])), so every
// particle lies within one cell of its home tile and the LDS box of h covers it.
// Each particle is written to ``out`` grouped by the tile of its current cell
// (before the push): a block first counts its particles per neighbour tile in LDS,
// reserves one contiguous run per neighbour tile with a single atomic on ``cursor``
// (the start of each tile in the new grouping, from the counts the previous
// deposition took), then gathers, pushes and writes each particle to base + its
// rank from a second LDS count.  Block ntiles carries invalid cells to the last bucket.
template <typename T, int ORDER>
__global__ void __launch_bounds__(PIC_GATHER_BLOCK) k_gather_push_home(GridGeom g, TileGeom tg, Batch<const T*> F,
                                                                       SpeciesView<T> in, SpeciesView<T> out,
                                                                       const int* __restrict__ home, int* cursor,
                                                                       T qdt2m, T dtx, T dty, T dtz) {
  using S = Shape<T, ORDER>;
  extern __shared__ __align__(16) unsigned char smem[];
  T* box = reinterpret_cast<T*>(smem);
  __shared__ int cnt[27];
  __shared__ int base[27];
  const int tile = blockIdx.x;
  const int beg = home[tile], end = home[tile + 1];
  if (beg == end) return;
  if (tile == tg.ntiles) {
    if (threadIdx.x == 0) base[0] = atomicAdd(&cursor[tg.ntiles], end - beg);
    __syncthreads();
    for (int qq = beg + threadIdx.x; qq < end; qq += blockDim.x) copy_particle(in, qq, out, base[0] + qq - beg);
    return;
  }
  const int B = tg.ts + S::NW + 1;
  int tx, ty, tz;
  tile_coords(tile, tg, tx, ty, tz);
  const int t0x = tx * tg.ts, t0y = ty * tg.ts, t0z = tz * tg.ts;
  if (threadIdx.x < 27) cnt[threadIdx.x] = 0;
  load_field_box<T, ORDER>(box, F, g, t0x, t0y, t0z, B);
  __syncthreads();
  // pass 1: particles per neighbour tile of the new grouping
  for (int qq = beg + threadIdx.x; qq < end; qq += blockDim.x) {
    int i, j, k;
    (void)decode_cell(in.cell[qq], g, nullptr, i, j, k);
    const int nb = neighbour_index(tile_of(i, j, k, tg), tx, ty, tz, tg);
    if (nb >= 0) atomicAdd(&cnt[nb], 1);
  }
  __syncthreads();
  // one contiguous run per neighbour tile, reserved with a single atomic each
  if (threadIdx.x < 27) {
    const int n = cnt[threadIdx.x];
    base[threadIdx.x] = n > 0 ? atomicAdd(&cursor[neighbour_key(threadIdx.x, tx, ty, tz, tg)], n) : 0;
    cnt[threadIdx.x] = 0;
  }
  __syncthreads();
  // pass 2: gather, push and write each particle to its slot
  for (int qq = beg + threadIdx.x; qq < end; qq += blockDim.x) {
    int i, j, k;
    (void)decode_cell(in.cell[qq], g, nullptr, i, j, k);
    const int key = tile_of(i, j, k, tg);
    const int nb = neighbour_index(key, tx, ty, tz, tg);
    const int slot = nb >= 0 ? base[nb] + atomicAdd(&cnt[nb], 1) : atomicAdd(&cursor[key], 1);
    T ox = in.off[0][qq], oy = in.off[1][qq], oz = in.off[2][qq];
    T ux = in.u[0][qq], uy = in.u[1][qq], uz = in.u[2][qq];
    const int lx = box_index(i, t0x, g.nx, tg.ts), ly = box_index(j, t0y, g.ny, tg.ts),
              lz = box_index(k, t0z, g.nz, tg.ts);
    gather_push_one<T, ORDER>(box, B, F, g, lx, ly, lz, i, j, k, ox, oy, oz, ux, uy, uz, qdt2m, dtx, dty, dtz);
    out.u[0][slot] = ux;
    out.u[1][slot] = uy;
    out.u[2][slot] = uz;
    out.off[0][slot] = ox;
    out.off[1][slot] = oy;
    out.off[2][slot] = oz;
    out.cell[slot] = (i * g.ny + j) * g.nz + k;
    if (in.w) out.w[slot] = in.w[qq];
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_permute(SpeciesView<T> in, SpeciesView<T> out, const int* __restrict__ dst) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= in.n) return;
  const long long q = dst[p];
  out.cell[q] = in.cell[p];
  for (int d = 0; d < 3; ++d) {
    out.off[d][q] = in.off[d][p];
    out.u[d][q] = in.u[d][p];
  }
  if (in.w) out.w[q] = in.w[p];
}

template <typename T>
__device__ inline void atomic_add(T* a, T v) {
  unsafeAtomicAdd(a, v);
}

template <typename T, int ORDER>
__device__ inline void scatter(const GridGeom& g, int i, int j, int k, T ox, T oy, T oz, T* const* dst, const T* val,
                               int nval) {
  using S = Shape<T, ORDER>;
  constexpr int NW = S::NW;
  T wx[NW], wy[NW], wz[NW];
  S::weights(ox, wx);
  S::weights(oy, wy);
  S::weights(oz, wz);
  int kk[NW];
#pragma unroll
  for (int cc = 0; cc < NW; ++cc) kk[cc] = wrapi(k + cc + S::BASE, g.nz);
#pragma unroll
  for (int a = 0; a < NW; ++a) {
    const int ii = wrapi(i + a + S::BASE, g.nx);
#pragma unroll
    for (int b = 0; b < NW; ++b) {
      const int jj = wrapi(j + b + S::BASE, g.ny);
      const size_t row = ((size_t)ii * g.ny + jj) * g.nz;
      const T wab = wx[a] * wy[b];
#pragma unroll
      for (int cc = 0; cc < NW; ++cc) {
        const T w = wab * wz[cc];
        for (int q = 0; q < nval; ++q) atomic_add(dst[q] + row + kk[cc], w * val[q]);
      }
    }
  }
}

// Fixed-point accumulators of the LDS deposition box.  FP32 runs accumulate int32
// (one v_cvt per contribution, ds_add_u32) scaled so that the tile's bound on any
// node sum stays below 2^30: a resolution of about 2^-31 * 8/27 * sum|q w| per
// contribution, comparable to FP32 rounding.  FP64 runs accumulate int64 scaled
// to 2^-50 of the largest |q w|, rounded with the exact 1.5*2^52 add.
template <typename T>
struct Fixed;

// shift(): the scale exponent for a tile whose partial sums are bounded by 2^e_sum,
// whose single contributions are bounded by 2^e_max, with fewer than 2^h particles.
template <>
struct Fixed<float> {
  using acc_t = int;
  __device__ static inline int shift(int e_sum, int e_max, int h) { return 30 - e_sum; }
  __device__ static inline acc_t conv(float x) { return __float2int_rn(x); }
  __device__ static inline void add(acc_t* a, acc_t v) { atomicAdd(a, v); }
};

template <>
struct Fixed<double> {
  using acc_t = long long;
  // |sum| < 2^(h + e_max + sh) <= 2^62; each contribution < 2^50 (exact rounding below)
  __device__ static inline int shift(int e_sum, int e_max, int h) { return min(62 - e_max - h, 50 - e_max); }
  __device__ static inline acc_t conv(double x) {
    return __double_as_longlong(x + 6755399441055744.0) - 0x4338000000000000LL;
  }
  __device__ static inline void add(acc_t* a, acc_t v) {
    atomicAdd(reinterpret_cast<unsigned long long*>(a), (unsigned long long)v);
  }
};

// Largest single-node weight of the 3D shape: 1 (linear) and (2/3)^3 (cubic).
template <int ORDER>
struct MaxWeight;
template <>
struct MaxWeight<1> {
  static constexpr double value = 1.0;
};
template <>
struct MaxWeight<3> {
  static constexpr double value = 8.0 / 27.0;
};

// Adds the shape-weighted values of one particle, as fixed-point integers scaled by
// 2^sh, to a (B x B x B) LDS box whose first support node is (lx, ly, lz).
// Integer LDS atomics retire about 20x faster than float LDS atomics on gfx950.
template <typename T, int ORDER>
__device__ inline void scatter_lds(typename Fixed<T>::acc_t* box, int B, int lx, int ly, int lz, T ox, T oy, T oz,
                                   const T* val, int nval, const int* sh) {
  using S = Shape<T, ORDER>;
  constexpr int NW = S::NW;
  T wx[NW], wy[NW], wz[NW];
  S::weights(ox, wx);
  S::weights(oy, wy);
  S::weights(oz, wz);
  const int B3 = B * B * B;
  T sv[3];
  for (int q = 0; q < nval; ++q) sv[q] = ldexp(val[q], sh[q]);
#pragma unroll
  for (int a = 0; a < NW; ++a) {
#pragma unroll
    for (int b = 0; b < NW; ++b) {
      const T wab = wx[a] * wy[b];
      const int row = ((lx + a) * B + (ly + b)) * B + lz;
#pragma unroll
      for (int cc = 0; cc < NW; ++cc) {
        const T w = wab * wz[cc];
        for (int q = 0; q < nval; ++q) Fixed<T>::add(&box[q * B3 + row + cc], Fixed<T>::conv(w * sv[q]));
      }
    }
  }
}


// One block per tile: rho (at x) and J (at x - dt v/2) of the tile's particles are
// accumulated in LDS over a box of B = ts + NW + 1 nodes per axis (the tile, the
// shape support and a one-cell margin for particles that moved since the sort),
// then stored to the tile's staging slot; k_deposit_reduce adds the overlapping
// boxes on the grid.  (A particle outside the margin is added to the grid
// directly with global atomics.)
template <typename T, int ORDER>
__global__ void __launch_bounds__(PIC_DEPOSIT_BLOCK) k_deposit_tiled(GridGeom g, TileGeom tg, SpeciesView<T> sp,
                                                       const int* __restrict__ perm, const int* __restrict__ starts,
                                                       Batch<T*> out, T* __restrict__ stage, T qdv, int with_j, T hdtx,
                                                       T hdty, T hdtz, int* bad, int* next_counts) {
  using S = Shape<T, ORDER>;
  constexpr int NW = S::NW;
  using acc_t = typename Fixed<T>::acc_t;
  extern __shared__ __align__(16) unsigned char smem[];
  acc_t* box = reinterpret_cast<acc_t*>(smem);
  constexpr int kWaves = PIC_DEPOSIT_BLOCK / 64;
  __shared__ T red[4 * kWaves];
  __shared__ T redm[4 * kWaves];
  __shared__ int cnt[27];
  const int tile = blockIdx.x;
  const int beg = starts[tile], end = starts[tile + 1];
  if (beg == end) return;
  if (tile == tg.ntiles) {  // invalid cells: never deposited, kept in the last bucket
    if (next_counts && threadIdx.x == 0) atomicAdd(&next_counts[tg.ntiles], end - beg);
    return;
  }
  const int ts = tg.ts;
  const int B = ts + NW + 1;
  const int B3 = B * B * B;
  const int ncomp = with_j ? 4 : 1;
  // Fixed-point scales 2^sh[c], one per deposited component.  A node of this box
  // receives from each particle of the tile at most MaxWeight * |q w| / dV (rho) or
  // MaxWeight * |q w v_c| / dV (J^c): every partial sum is bounded by MaxWeight times the
  // tile's sum of those magnitudes (< 2^e_sum), every contribution by their max (< 2^e_max).
  // per component c (rho, J^x, J^y, J^z): sum and max over the tile of |q w| (rho) or
  // |q w v_c| (J^c), the bounds that set that component's scale
  T sw[4] = {0, 0, 0, 0}, mw[4] = {0, 0, 0, 0};
  for (int qq = beg + threadIdx.x; qq < end; qq += blockDim.x) {
    const int p = perm ? perm[qq] : qq;
    const T a = fabs(sp.w ? sp.w[p] : (T)sp.w_const);
    sw[0] += a;
    mw[0] = fmax(mw[0], a);
    if (with_j) {
      const T ux = sp.u[0][p], uy = sp.u[1][p], uz = sp.u[2][p];
      const T ig = (T)1 / sqrt((T)1 + ux * ux + uy * uy + uz * uz);
      const T v[3] = {fabs(ux * ig), fabs(uy * ig), fabs(uz * ig)};
      for (int d = 0; d < 3; ++d) {
        sw[1 + d] += a * v[d];
        mw[1 + d] = fmax(mw[1 + d], a * v[d]);
      }
    }
  }
  for (int c = 0; c < ncomp; ++c) {
    for (int o = 32; o > 0; o >>= 1) {
      sw[c] += __shfl_xor(sw[c], o, 64);
      mw[c] = fmax(mw[c], __shfl_xor(mw[c], o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
      red[c * kWaves + (threadIdx.x >> 6)] = sw[c];
      redm[c * kWaves + (threadIdx.x >> 6)] = mw[c];
    }
  }
  __syncthreads();
  __shared__ int shs[4];
  if (threadIdx.x < ncomp) {
    const int c = threadIdx.x;
    T m = 0, x = 0;
    for (int w = 0; w < kWaves; ++w) {
      m += red[c * kWaves + w];
      x = fmax(x, redm[c * kWaves + w]);
    }
    // a little slack on the bound covers the rounding of the FP sum itself
    int e_sum = 0, e_max = 0;
    (void)frexp(m * fabs(qdv) * (T)(MaxWeight<ORDER>::value * 1.001), &e_sum);
    (void)frexp(x * fabs(qdv) * (T)1.001, &e_max);
    shs[c] = Fixed<T>::shift(e_sum, e_max, 32 - __clz(end - beg));
  }
  __syncthreads();
  int sh[4];
  for (int c = 0; c < 4; ++c) sh[c] = (c < ncomp) ? shs[c] : 0;
  int ti, tj, tk;
  tile_coords(tile, tg, ti, tj, tk);
  const int t0x = ti * ts, t0y = tj * ts, t0z = tk * ts;
  for (int k = threadIdx.x; k < ncomp * B3; k += blockDim.x) box[k] = 0;
  if (threadIdx.x < 27) cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int qq = beg + threadIdx.x; qq < end; qq += blockDim.x) {
    const int p = perm ? perm[qq] : qq;
    int i, j, k;
    if (!decode_cell(sp.cell[p], g, bad, i, j, k)) continue;
    const T ox = sp.off[0][p], oy = sp.off[1][p], oz = sp.off[2][p];
    const T qw = qdv * (sp.w ? sp.w[p] : (T)sp.w_const);
    if (next_counts) {  // the tile of this position groups the particle in the next step
      const int key = tile_of(i, j, k, tg);
      const int nb = neighbour_index(key, ti, tj, tk, tg);
      if (nb >= 0) atomicAdd(&cnt[nb], 1);
      else atomicAdd(&next_counts[key], 1);
    }
    {
      const int lx = box_index(i, t0x, g.nx, ts), ly = box_index(j, t0y, g.ny, ts), lz = box_index(k, t0z, g.nz, ts);
      T val[1] = {qw};
      if (lx >= 0 && ly >= 0 && lz >= 0) {
        scatter_lds<T, ORDER>(box, B, lx, ly, lz, ox, oy, oz, val, 1, sh);
      } else {
        T* dst[1] = {out.p[0]};
        scatter<T, ORDER>(g, i, j, k, ox, oy, oz, dst, val, 1);
      }
    }
    if (with_j) {
      const T ux = sp.u[0][p], uy = sp.u[1][p], uz = sp.u[2][p];
      const T ig = (T)1 / sqrt((T)1 + ux * ux + uy * uy + uz * uz);
      const T vx = ux * ig, vy = uy * ig, vz = uz * ig;
      // x^{n+1/2} = x^{n+1} - dt v / 2
      T hx = ox, hy = oy, hz = oz;
      const int ih = modi(i + advance_offset(hx, -hdtx * vx), g.nx);
      const int jh = modi(j + advance_offset(hy, -hdty * vy), g.ny);
      const int kh = modi(k + advance_offset(hz, -hdtz * vz), g.nz);
      T val[3] = {qw * vx, qw * vy, qw * vz};
      const int lx = box_index(ih, t0x, g.nx, ts), ly = box_index(jh, t0y, g.ny, ts),
                lz = box_index(kh, t0z, g.nz, ts);
      if (lx >= 0 && ly >= 0 && lz >= 0) {
        scatter_lds<T, ORDER>(box + B3, B, lx, ly, lz, hx, hy, hz, val, 3, sh + 1);
      } else {
        T* dst[3] = {out.p[1], out.p[2], out.p[3]};
        scatter<T, ORDER>(g, ih, jh, kh, hx, hy, hz, dst, val, 3);
      }
    }
  }
  __syncthreads();
  if (next_counts && threadIdx.x < 27 && cnt[threadIdx.x] > 0)
    atomicAdd(&next_counts[neighbour_key(threadIdx.x, ti, tj, tk, tg)], cnt[threadIdx.x]);
  // the whole box goes to this tile's staging slot (plain stores, zeros included)
  T* dstage = stage + (size_t)tile * ncomp * B3;
  for (int k = threadIdx.x; k < ncomp * B3; k += blockDim.x) dstage[k] = ldexp((T)box[k], -sh[k / B3]);
}

// Sums, for every grid node, the staging boxes of all non-empty tiles that cover it
// (box node l of tile t along an axis is grid node (t*ts - 1 + BASE + l) mod n) and
// adds the sums to the nodal arrays.  Each node is owned by one thread: no atomics.
template <typename T, int ORDER>
__global__ void __launch_bounds__(256) k_deposit_reduce(GridGeom g, TileGeom tg, const int* __restrict__ starts,
                                                        const T* __restrict__ stage, Batch<T*> out, int ncomp) {
  using S = Shape<T, ORDER>;
  constexpr int NW = S::NW;
  const int ts = tg.ts;
  const int B = ts + NW + 1;
  const int B3 = B * B * B;
  const long long N = (long long)g.nx * g.ny * g.nz;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < N;
       idx += (long long)gridDim.x * blockDim.x) {
    const int z = (int)(idx % g.nz);
    const long long r = idx / g.nz;
    const int y = (int)(r % g.ny);
    const int x = (int)(r / g.ny);
    // candidate (tile, box index) pairs per axis over the periodic images x - n, x, x + n
    int ctx_[8], clx[8], cty[8], cly[8], ctz[8], clz[8];
    int nx_ = 0, ny_ = 0, nz_ = 0;
    const int pos[3] = {x, y, z};
    const int n[3] = {g.nx, g.ny, g.nz};
    const int nt[3] = {tg.ntx, tg.nty, tg.ntz};
    for (int d = 0; d < 3; ++d) {
      int* ct = d == 0 ? ctx_ : (d == 1 ? cty : ctz);
      int* cl = d == 0 ? clx : (d == 1 ? cly : clz);
      int cnt = 0;
      for (int im = -1; im <= 1; ++im) {
        const int X = pos[d] + im * n[d];
        // tiles t with 0 <= X - (t*ts - 1 + BASE) < B
        const int hi = (X + 1 - S::BASE);
        int tmax = hi >= 0 ? hi / ts : -((-hi + ts - 1) / ts);
        for (int t = tmax; t >= 0 && cnt < 8; --t) {
          const int l = X - (t * ts - 1 + S::BASE);
          if (l >= B) break;
          if (t < nt[d] && l >= 0) {
            ct[cnt] = t;
            cl[cnt] = l;
            ++cnt;
          }
        }
      }
      if (d == 0) nx_ = cnt; else if (d == 1) ny_ = cnt; else nz_ = cnt;
    }
    T acc[4] = {0, 0, 0, 0};
    for (int a = 0; a < nx_; ++a)
      for (int b = 0; b < ny_; ++b)
        for (int c = 0; c < nz_; ++c) {
          const int tile = (ctx_[a] * tg.nty + cty[b]) * tg.ntz + ctz[c];
          if (starts[tile] == starts[tile + 1]) continue;
          const T* sb = stage + (size_t)tile * ncomp * B3 + (clx[a] * B + cly[b]) * B + clz[c];
          for (int q = 0; q < ncomp; ++q) acc[q] += sb[(size_t)q * B3];
        }
    for (int q = 0; q < ncomp; ++q) out.p[q][idx] += acc[q];
  }
}


}  // namespace

template <typename T>
void permute_species(const SpeciesView<T>& in, const SpeciesView<T>& out, const int* dst, hipStream_t s) {
  if (in.n <= 0) return;
  hipLaunchKernelGGL((k_permute<T>), dim3((unsigned)((in.n + 255) / 256)), dim3(256), 0, s, in, out, dst);
}

// Raises a kernel's dynamic-LDS limit above the 64 KiB default when a launch needs it
// (gfx950 has 160 KiB of LDS per workgroup).  A refusal surfaces at the launch.
void allow_lds(const void* kernel, size_t bytes) {
  if (bytes > 64 * 1024) {
    if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
      (void)hipGetLastError();
  }
}

int deposit_box(int shape_order, int ts) { return ts + (shape_order == 1 ? 2 : 4) + 1; }
template <typename T>
void gather_push_tiled(const GridGeom& g, const TileGeom& t, const T* const E[3], const T* const B[3],
                       const SpeciesView<T>& in, const SpeciesView<T>& out, const int* perm, const int* starts,
                       bool write_sorted, int* home_cursor, hipStream_t s) {
  if (in.n <= 0) return;
  Batch<const T*> F{};
  for (int d = 0; d < 3; ++d) {
    F.p[d] = E[d];
    F.p[3 + d] = B[d];
  }
  const T qdt2m = (T)(in.q * g.dt / (2.0 * in.m));
  const T dtx = (T)(g.dt / g.dx), dty = (T)(g.dt / g.dy), dtz = (T)(g.dt / g.dz);
  const int Bx = deposit_box(g.shape_order, t.ts);
  const size_t lds = (size_t)Bx * Bx * Bx * FieldSlots<T>::FS * sizeof(T);
  const dim3 grid(t.ntiles + 1), block(PIC_GATHER_BLOCK);
  if (home_cursor) {
    if (g.shape_order == 1) {
      allow_lds((const void*)k_gather_push_home<T, 1>, lds);
      hipLaunchKernelGGL((k_gather_push_home<T, 1>), grid, block, lds, s, g, t, F, in, out, starts, home_cursor,
                         qdt2m, dtx, dty, dtz);
    } else {
      allow_lds((const void*)k_gather_push_home<T, 3>, lds);
      hipLaunchKernelGGL((k_gather_push_home<T, 3>), grid, block, lds, s, g, t, F, in, out, starts, home_cursor,
                         qdt2m, dtx, dty, dtz);
    }
  } else {
    const int ws = write_sorted ? 1 : 0;
    if (g.shape_order == 1) {
      allow_lds((const void*)k_gather_push_perm<T, 1>, lds);
      hipLaunchKernelGGL((k_gather_push_perm<T, 1>), grid, block, lds, s, g, t, F, in, out, perm, starts, ws, qdt2m,
                         dtx, dty, dtz);
    } else {
      allow_lds((const void*)k_gather_push_perm<T, 3>, lds);
      hipLaunchKernelGGL((k_gather_push_perm<T, 3>), grid, block, lds, s, g, t, F, in, out, perm, starts, ws, qdt2m,
                         dtx, dty, dtz);
    }
  }
}

template <typename T>
void deposit_tiled(const GridGeom& g, const TileGeom& t, const SpeciesView<T>& sp, const int* perm, const int* starts,
                   bool with_j, T* stage, int* bad, int* next_counts, T* rho, T* const J[3], hipStream_t s) {
  if (sp.n <= 0) return;
  Batch<T*> out{};
  out.p[0] = rho;
  for (int d = 0; d < 3; ++d) out.p[1 + d] = J ? J[d] : nullptr;
  const T qdv = (T)(sp.q / (g.dx * g.dy * g.dz));
  const T hx = (T)(0.5 * g.dt / g.dx), hy = (T)(0.5 * g.dt / g.dy), hz = (T)(0.5 * g.dt / g.dz);
  const int wj = with_j ? 1 : 0;
  const int ncomp = with_j ? 4 : 1;
  const int B = deposit_box(g.shape_order, t.ts);
  const size_t lds = (size_t)ncomp * B * B * B * sizeof(typename Fixed<T>::acc_t);
  if (g.shape_order == 1) allow_lds((const void*)k_deposit_tiled<T, 1>, lds);
  else allow_lds((const void*)k_deposit_tiled<T, 3>, lds);
  if (g.shape_order == 1)
    hipLaunchKernelGGL((k_deposit_tiled<T, 1>), dim3(t.ntiles + 1), dim3(PIC_DEPOSIT_BLOCK), lds, s, g, t, sp, perm,
                       starts, out, stage, qdv, wj, hx, hy, hz, bad, next_counts);
  else
    hipLaunchKernelGGL((k_deposit_tiled<T, 3>), dim3(t.ntiles + 1), dim3(PIC_DEPOSIT_BLOCK), lds, s, g, t, sp, perm,
                       starts, out, stage, qdv, wj, hx, hy, hz, bad, next_counts);
}

template <typename T>
void deposit_reduce(const GridGeom& g, const TileGeom& t, const int* starts, const T* stage, bool with_j, T* rho,
                    T* const J[3], hipStream_t s) {
  Batch<T*> out{};
  out.p[0] = rho;
  for (int d = 0; d < 3; ++d) out.p[1 + d] = J ? J[d] : nullptr;
  const int ncomp = with_j ? 4 : 1;
  const long long N = (long long)g.nx * g.ny * g.nz;
  const unsigned nr = (unsigned)std::min<long long>((N + 255) / 256, 65536);
  if (g.shape_order == 1)
    hipLaunchKernelGGL((k_deposit_reduce<T, 1>), dim3(nr), dim3(256), 0, s, g, t, starts, stage, out, ncomp);
  else
    hipLaunchKernelGGL((k_deposit_reduce<T, 3>), dim3(nr), dim3(256), 0, s, g, t, starts, stage, out, ncomp);
}

#define PIC_INST(T)                                                                                              \
  template void permute_species<T>(const SpeciesView<T>&, const SpeciesView<T>&, const int*, hipStream_t);       \
  template void deposit_tiled<T>(const GridGeom&, const TileGeom&, const SpeciesView<T>&, const int*, const int*, \
                                 bool, T*, int*, int*, T*, T* const*, hipStream_t);                              \
  template void deposit_reduce<T>(const GridGeom&, const TileGeom&, const int*, const T*, bool, T*, T* const*,   \
                                  hipStream_t);                                                                  \
  template void gather_push_tiled<T>(const GridGeom&, const TileGeom&, const T* const*, const T* const*,         \
                                     const SpeciesView<T>&, const SpeciesView<T>&, const int*, const int*, bool,  \
                                     int*, hipStream_t);
PIC_INST(float)
PIC_INST(double)
#undef PIC_INST

}  // namespace pic
