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
// Workgroup of the production gather + push: FP32 cubic boxes (53 KB of LDS, a few hundred
// particles per tile at the densities of the beam-driven wake) run three 256-thread
// workgroups per CU, whose box loads and particle work then overlap; every other case runs
// 512 threads (a double cubic box admits one workgroup per CU, linear tiles hold many more
// particles per box).
#ifndef PIC_GATHER_BLOCK_F32_CUBIC
#define PIC_GATHER_BLOCK_F32_CUBIC 256
#endif
template <typename T, int ORDER>
constexpr int kGatherBlock = (sizeof(T) == 4 && ORDER == 3) ? PIC_GATHER_BLOCK_F32_CUBIC : PIC_GATHER_BLOCK;
#ifndef PIC_DEPOSIT_BLOCK
#define PIC_DEPOSIT_BLOCK 256
#endif
#ifndef PIC_DEPOSIT_BOUND_LOAD
#define PIC_DEPOSIT_BOUND_LOAD 1
#endif
#ifndef PIC_DEPOSIT_CELL_KEY
#define PIC_DEPOSIT_CELL_KEY 1
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
  // d w / d d (the reverse mode's position derivatives)
  __device__ static inline void dweights(T, T* g) {
    g[0] = (T)-1;
    g[1] = (T)1;
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
  __device__ static inline void dweights(T d, T* g) {
    const T e = (T)1 - d;
    g[0] = (T)-0.5 * e * e;
    g[1] = (T)-2 * d + (T)1.5 * d * d;
    g[2] = (T)2 * e - (T)1.5 * e * e;
    g[3] = (T)0.5 * d * d;
  }
};

// 1/sqrt(x) and a/b: the hardware approximations (about 1 ulp) in FP32, exact
// rounding in FP64 (the FP64 path is held to the FP64 oracle's rounding level).
__device__ inline float inv_sqrt(float x) { return rsqrtf(x); }
__device__ inline double inv_sqrt(double x) { return 1.0 / sqrt(x); }
__device__ inline float quot(float a, float b) { return __fdividef(a, b); }
__device__ inline double quot(double a, double b) { return a / b; }

__device__ inline int wrapi(int i, int n) {
  i = (i < 0) ? i + n : i;
  return (i >= n) ? i - n : i;
}

// periodic index for any integer (used where the shift comes from caller data)
__device__ inline int modi(int i, int n) {
  i %= n;
  return (i < 0) ? i + n : i;
}

__device__ inline int fdiv(int n, const FastDiv& f) { return (int)((__umulhi((uint32_t)n, f.m) + (uint32_t)n) >> f.s); }

// Decodes a linear cell index c = (i ny + j) nz + k; returns false (and counts the
// particle when ``bad`` is given) when it is out of range.
__device__ inline bool decode_cell(int c, const GridGeom& g, int* bad, int& i, int& j, int& k) {
  if (c < 0 || c >= g.nx * g.ny * g.nz) {
    if (bad) atomicAdd(bad, 1);
    return false;
  }
  const int r = fdiv(c, g.nz_div);
  k = c - r * g.nz;
  i = fdiv(r, g.ny_div);
  j = r - i * g.ny;
  return true;
}

// offset + displacement (in cells) -> (new offset in [0,1), integer shift in -1..1),
// |displacement| < 1.
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
  return ((i / kTile) * tg.nty + j / kTile) * tg.ntz + k / kTile;
}

// Index 0..26 of the tile of cell (i, j, k) among the 27 tiles around (tx, ty, tz)
// (periodic), or -1.  13 is the tile itself.
__device__ inline int neighbour_of_cell(int i, int j, int k, int tx, int ty, int tz, const TileGeom& tg) {
  int d[3] = {i / kTile - tx, j / kTile - ty, k / kTile - tz};
  const int nt[3] = {tg.ntx, tg.nty, tg.ntz};
#pragma unroll
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

// box-local index (0 .. B-1) of the first support node of a particle in cell i
// (0 <= i < n) of a tile starting at cell t0, for boxes whose node 0 is t0 - 1 + BASE
// (one-cell margin); -1 if the particle is outside the margin.
__device__ inline int box_index(int i, int t0, int n) {
  const int l = wrapi(i - t0 + 1, n);
  return (l <= kTile + 1) ? l : -1;
}

// Box geometry of one tile for a shape of NW nodes per axis: B = kTile + NW + 1
// nodes per edge, z fastest.
template <int NW>
struct Box {
  static constexpr int B = kTile + NW + 1;
  static constexpr int B2 = B * B;
  static constexpr int B3 = B2 * B;
  __device__ static inline int at(int lx, int ly, int lz) { return (lx * B + ly) * B + lz; }
};

// Row layout of a tile's staging slot (see deposit_stage_slot): per component B x B rows of
// PZ values, box node (lx, ly, lz) at (lx * B + ly) * PZ + OFF + lz, zeros in the other positions.
template <int ORDER>
struct StageRows {
  static constexpr int B = kTile + (ORDER == 1 ? 2 : 4) + 1;
  static constexpr int BASE = ORDER == 1 ? 0 : -1;
  static constexpr int PZ = 16;
  static constexpr int OFF = (BASE + 3) & 3;
  static constexpr int SLOT = B * B * PZ;
  static_assert(OFF + B <= PZ, "a box row fits its padded row");
  __device__ static inline int at(int lx, int ly, int lz) { return (lx * B + ly) * PZ + OFF + lz; }
};

// Four consecutive values as one 16-byte (float) or two 16-byte (double) accesses.
__device__ inline void store4(float* p, const float* v) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ inline void store4(double* p, const double* v) {
  reinterpret_cast<double2*>(p)[0] = make_double2(v[0], v[1]);
  reinterpret_cast<double2*>(p)[1] = make_double2(v[2], v[3]);
}
__device__ inline void load4(const float* p, float* v) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}
__device__ inline void load4(const double* p, double* v) {
  const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}

// One particle as stored: cell, offsets, momentum (when WJ) and weight.  Loaded in one
// go, so that the loads of several particles are in flight together.
template <typename T>
struct Raw {
  int cell;
  T o[3], u[3], w;
};

// Stand-in weight array for species without per-particle weights: the weight load
// is then unconditional (a branch around it would make the compiler wait for every
// load in flight) and its value is replaced by w_const.
__device__ float g_no_weight_f[1];
__device__ double g_no_weight_d[1];
template <typename T>
__device__ inline const T* no_weight();
template <>
__device__ inline const float* no_weight<float>() { return g_no_weight_f; }
template <>
__device__ inline const double* no_weight<double>() { return g_no_weight_d; }

template <typename T, bool WJ>
__device__ inline void load_raw(const SpeciesView<T>& sp, int p, Raw<T>& r) {
  r.cell = sp.cell[p];
#pragma unroll
  for (int d = 0; d < 3; ++d) r.o[d] = sp.off[d][p];
#pragma unroll
  for (int d = 0; d < 3; ++d) r.u[d] = WJ ? sp.u[d][p] : (T)0;
  const bool has_w = sp.w != nullptr;
  const T wv = (has_w ? sp.w : no_weight<T>())[has_w ? p : 0];
  r.w = has_w ? wv : (T)sp.w_const;
}

// What the scale bounds need of a particle: its momentum (when WJ) and weight.
template <typename T, bool WJ>
__device__ inline void load_bound(const SpeciesView<T>& sp, int p, Raw<T>& r) {
#pragma unroll
  for (int d = 0; d < 3; ++d) r.u[d] = WJ ? sp.u[d][p] : (T)0;
  const bool has_w = sp.w != nullptr;
  const T wv = (has_w ? sp.w : no_weight<T>())[has_w ? p : 0];
  r.w = has_w ? wv : (T)sp.w_const;
}

// Slots -> particle indices through an optional permutation, all lookups in flight at once.
template <int U>
__device__ inline void through_perm(const int* perm, int (&q)[U]) {
  if (perm) {
    int t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) t[u] = perm[q[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = t[u];
  }
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

// The box of the hybrid gather: for float two planes, (E_x, E_y, E_z, B_x) as one float4 per
// node (16-byte stride) followed by (B_y, B_z) as one float2 per node (8-byte stride).  Lanes
// reading 16 bytes each are served eight at a time; at a 16-byte node stride those eight
// spread over every bank group, where the 32-byte stride of FieldSlots<float> reaches only
// half of them.  Double keeps FieldSlots<double> (48-byte stride, already spread).
template <typename T, int B3>
struct GatherBox {
  static constexpr int SLOTS = FieldSlots<T>::FS;
  __device__ static inline void store(T* box, int e, const T* v) {
#pragma unroll
    for (int c = 0; c < 6; ++c) box[e * SLOTS + c] = v[c];
  }
  __device__ static inline void read(const T* box, int e, T* v) { FieldSlots<T>::read(box + (size_t)e * SLOTS, v); }
};
template <int B3>
struct GatherBox<float, B3> {
  static constexpr int SLOTS = 6;
  __device__ static inline void store(float* box, int e, const float* v) {
    reinterpret_cast<float4*>(box)[e] = make_float4(v[0], v[1], v[2], v[3]);
    reinterpret_cast<float2*>(box + 4 * B3)[e] = make_float2(v[4], v[5]);
  }
  __device__ static inline void read(const float* box, int e, float* v) {
    const float4 a = reinterpret_cast<const float4*>(box)[e];
    const float2 b = reinterpret_cast<const float2*>(box + 4 * B3)[e];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y;
  }
};

// Periodic index of x in [-n, 3n).
__device__ inline int wrap3(int x, int n) {
  x += (x < 0) ? n : 0;
  x -= (x >= n) ? n : 0;
  return (x >= n) ? x - n : x;
}

// Byte offset of a grid element in the loads of load_field_box: 32-bit for float (at most
// 1024^3 cells, so below 2^32 bytes), which lets each load add it to the array's base held in
// scalar registers; 64-bit for double.
template <typename T>
struct BoxOffset {
  using type = size_t;
};
template <>
struct BoxOffset<float> {
  using type = unsigned int;
};
static_assert((size_t)1024 * 1024 * 1024 * sizeof(float) - 1 <= 0xffffffffu, "float offsets must fit 32 bits");

// Stages the six nodal components over the box of tile (t0x, t0y, t0z), in the
// FieldSlots layout or (GATHER) the GatherBox one.  Thread t takes box elements
// e = t + u * BLOCK; their coordinates (lx, ly, lz) advance by the block size
// written in base B (no division per node).  Boxes inside the grid (all but the tiles on
// its faces) skip the periodic wrap.  Each thread issues the loads of all its nodes before
// storing any, so they are in flight together.
template <typename T, int ORDER, bool GATHER = false, int BLOCK = PIC_GATHER_BLOCK>
__device__ inline void load_field_box(T* box, const Batch<const T*>& F, const GridGeom& g, int t0x, int t0y, int t0z) {
  using S = Shape<T, ORDER>;
  using X = Box<S::NW>;
  using Off = typename BoxOffset<T>::type;
  constexpr int B = X::B;
  constexpr int FS = FieldSlots<T>::FS;
  constexpr int PER = (X::B3 + BLOCK - 1) / BLOCK;
  constexpr int DX = BLOCK / X::B2, DY = (BLOCK / B) % B, DZ = BLOCK % B;
  const int ox0 = t0x - 1 + S::BASE, oy0 = t0y - 1 + S::BASE, oz0 = t0z - 1 + S::BASE;
  const bool inner = ox0 >= 0 && ox0 + B <= g.nx && oy0 >= 0 && oy0 + B <= g.ny && oz0 >= 0 && oz0 + B <= g.nz;
  const int t = threadIdx.x;
  int lx = t / X::B2, ly = (t / B) % B, lz = t % B;
  T v[PER][6];
  if (inner) {
    const int sxy = g.ny * g.nz;
    const int base = (ox0 * g.ny + oy0) * g.nz + oz0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      if (u < PER - 1 || t + u * BLOCK < X::B3) {
        const Off off = (Off)(base + lx * sxy + ly * g.nz + lz) * (Off)sizeof(T);
#pragma unroll
        for (int c = 0; c < 6; ++c) v[u][c] = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(F.p[c]) + off);
      }
      lz += DZ;
      ly += DY + (lz >= B ? 1 : 0);
      lz -= lz >= B ? B : 0;
      lx += DX + (ly >= B ? 1 : 0);
      ly -= ly >= B ? B : 0;
    }
  } else {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      if (u < PER - 1 || t + u * BLOCK < X::B3) {
        const Off off = (Off)((wrap3(ox0 + lx, g.nx) * g.ny + wrap3(oy0 + ly, g.ny)) * g.nz + wrap3(oz0 + lz, g.nz)) *
                        (Off)sizeof(T);
#pragma unroll
        for (int c = 0; c < 6; ++c) v[u][c] = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(F.p[c]) + off);
      }
      lz += DZ;
      ly += DY + (lz >= B ? 1 : 0);
      lz -= lz >= B ? B : 0;
      lx += DX + (ly >= B ? 1 : 0);
      ly -= ly >= B ? B : 0;
    }
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = t + u * BLOCK;
    if (e < X::B3) {
      if (GATHER) {
        GatherBox<T, X::B3>::store(box, e, v[u]);
      } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) box[e * FS + c] = v[u][c];
      }
    }
  }
}

// Relativistic Boris push (c = 1) of u by the gathered f = (E, B), qdt2m = q dt / (2 m):
//   u- = u + qdt2m E,  t = qdt2m B / gamma(u-),  s = 2 t / (1 + |t|^2),
//   u' = u- + u- x t,  u+ = u- + u' x s,  u_new = u+ + qdt2m E.
// The intermediates stay in ``b`` (the reverse mode reuses them).
template <typename T>
struct BorisState {
  T umx, umy, umz, tf, tx, ty, tz, sf, sx, sy, sz, upx, upy, upz;
};
template <typename T>
__device__ inline void boris(const T* f, T qdt2m, T& ux, T& uy, T& uz, BorisState<T>& b) {
  b.umx = ux + qdt2m * f[0];
  b.umy = uy + qdt2m * f[1];
  b.umz = uz + qdt2m * f[2];
  b.tf = qdt2m * inv_sqrt((T)1 + b.umx * b.umx + b.umy * b.umy + b.umz * b.umz);  // q dt / (2 m gamma)
  b.tx = b.tf * f[3];
  b.ty = b.tf * f[4];
  b.tz = b.tf * f[5];
  b.sf = quot((T)2, (T)1 + b.tx * b.tx + b.ty * b.ty + b.tz * b.tz);
  b.sx = b.sf * b.tx;
  b.sy = b.sf * b.ty;
  b.sz = b.sf * b.tz;
  b.upx = b.umx + (b.umy * b.tz - b.umz * b.ty);
  b.upy = b.umy + (b.umz * b.tx - b.umx * b.tz);
  b.upz = b.umz + (b.umx * b.ty - b.umy * b.tx);
  ux = b.umx + (b.upy * b.sz - b.upz * b.sy) + qdt2m * f[0];
  uy = b.umy + (b.upz * b.sx - b.upx * b.sz) + qdt2m * f[1];
  uz = b.umz + (b.upx * b.sy - b.upy * b.sx) + qdt2m * f[2];
}

// Gather at one particle from the LDS box (GatherBox layout; first support node at box
// index l*) or, outside the margin, from the grid; then the relativistic Boris push and the move.
template <typename T, int ORDER>
__device__ inline void gather_push_one(const T* box, const Batch<const T*>& F, const GridGeom& g, int lx, int ly,
                                       int lz, int& i, int& j, int& k, T& ox, T& oy, T& oz, T& ux, T& uy, T& uz,
                                       T qdt2m, T dtx, T dty, T dtz) {
  using S = Shape<T, ORDER>;
  using X = Box<S::NW>;
  constexpr int NW = S::NW;
  T wx[NW], wy[NW], wz[NW];
  S::weights(ox, wx);
  S::weights(oy, wy);
  S::weights(oz, wz);
  T f[6] = {0, 0, 0, 0, 0, 0};
  if (lx >= 0 && ly >= 0 && lz >= 0) {
    const int n0 = X::at(lx, ly, lz);
#pragma unroll
    for (int a = 0; a < NW; ++a) {
#pragma unroll
      for (int b = 0; b < NW; ++b) {
        const T wab = wx[a] * wy[b];
#pragma unroll
        for (int cc = 0; cc < NW; ++cc) {
          const T w = wab * wz[cc];
          T v[6];
          GatherBox<T, X::B3>::read(box, n0 + a * X::B2 + b * X::B + cc, v);
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
  BorisState<T> b;
  boris(f, qdt2m, ux, uy, uz, b);
  const T ig = inv_sqrt((T)1 + ux * ux + uy * uy + uz * uz);
  // on the grid moving with v_gal (Galilean frame) the particle moves by (v - v_gal) dt
  i = wrapi(i + advance_offset(ox, dtx * ux * ig - (T)g.sgx), g.nx);
  j = wrapi(j + advance_offset(oy, dty * uy * ig - (T)g.sgy), g.ny);
  k = wrapi(k + advance_offset(oz, dtz * uz * ig - (T)g.sgz), g.nz);
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
__global__ void __launch_bounds__((kGatherBlock<T, ORDER>)) k_gather_push_perm(GridGeom g, TileGeom tg, Batch<const T*> F,
                                                                       SpeciesView<T> in, SpeciesView<T> out,
                                                                       const int* __restrict__ perm,
                                                                       const int* __restrict__ starts, int write_sorted,
                                                                       T qdt2m, T dtx, T dty, T dtz) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* box = reinterpret_cast<T*>(smem);
  const int tile = xcd_major(blockIdx.x, gridDim.x);
  const int beg = starts[tile], end = starts[tile + 1];
  if (beg == end) return;
  if (tile == tg.ntiles) {
    for (int qq = beg + threadIdx.x; qq < end; qq += blockDim.x) {
      const int p = perm[qq];
      copy_particle(in, p, out, write_sorted ? qq : p);
    }
    return;
  }
  int tx, ty, tz;
  tile_coords(tile, tg, tx, ty, tz);
  const int t0x = tx * kTile, t0y = ty * kTile, t0z = tz * kTile;
  load_field_box<T, ORDER, true, kGatherBlock<T, ORDER>>(box, F, g, t0x, t0y, t0z);
  __syncthreads();
  for (int qq = beg + threadIdx.x; qq < end; qq += blockDim.x) {
    const int p = perm[qq];
    const int wi = write_sorted ? qq : p;
    int i, j, k;
    (void)decode_cell(in.cell[p], g, nullptr, i, j, k);
    T ox = in.off[0][p], oy = in.off[1][p], oz = in.off[2][p];
    T ux = in.u[0][p], uy = in.u[1][p], uz = in.u[2][p];
    const int lx = box_index(i, t0x, g.nx), ly = box_index(j, t0y, g.ny), lz = box_index(k, t0z, g.nz);
    gather_push_one<T, ORDER>(box, F, g, lx, ly, lz, i, j, k, ox, oy, oz, ux, uy, uz, qdt2m, dtx, dty, dtz);
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
__global__ void __launch_bounds__((kGatherBlock<T, ORDER>)) k_gather_push_home(GridGeom g, TileGeom tg, Batch<const T*> F,
                                                                       SpeciesView<T> in, SpeciesView<T> out,
                                                                       const int* __restrict__ home, int* cursor,
                                                                       const int* __restrict__ nbr_bases, T qdt2m,
                                                                       T dtx, T dty, T dtz) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* box = reinterpret_cast<T*>(smem);
  __shared__ int cnt[27];
  __shared__ int base[27];
  const int tile = xcd_major(blockIdx.x, gridDim.x);
  const int beg = home[tile], end = home[tile + 1];
  if (beg == end) return;
  if (tile == tg.ntiles) {
    if (threadIdx.x == 0) base[0] = atomicAdd(&cursor[tg.ntiles], end - beg);
    __syncthreads();
    for (int qq = beg + threadIdx.x; qq < end; qq += blockDim.x) copy_particle(in, qq, out, base[0] + qq - beg);
    return;
  }
  int tx, ty, tz;
  tile_coords(tile, tg, tx, ty, tz);
  const int t0x = tx * kTile, t0y = ty * kTile, t0z = tz * kTile;
  if (threadIdx.x < 27) {
    cnt[threadIdx.x] = 0;
    if (nbr_bases) base[threadIdx.x] = nbr_bases[27 * tile + threadIdx.x];
  }
  load_field_box<T, ORDER, true, kGatherBlock<T, ORDER>>(box, F, g, t0x, t0y, t0z);
  __syncthreads();
  if (!nbr_bases) {
    // pass 1: particles per neighbour tile of the new grouping (the home tile, the
    // common case, is counted once per wave), then one contiguous run per neighbour
    // tile, reserved with a single atomic each
    for (int qq = beg + threadIdx.x; qq < end; qq += blockDim.x) {
      int i, j, k;
      (void)decode_cell(in.cell[qq], g, nullptr, i, j, k);
      const int nb = neighbour_of_cell(i, j, k, tx, ty, tz, tg);
      const unsigned long long own = __ballot(nb == 13);
      if (nb == 13) {
        if (__lane_id() == __ffsll(own) - 1) atomicAdd(&cnt[13], __popcll(own));
      } else if (nb >= 0) {
        atomicAdd(&cnt[nb], 1);
      }
    }
    __syncthreads();
    if (threadIdx.x < 27) {
      const int n = cnt[threadIdx.x];
      base[threadIdx.x] = n > 0 ? atomicAdd(&cursor[neighbour_key(threadIdx.x, tx, ty, tz, tg)], n) : 0;
      cnt[threadIdx.x] = 0;
    }
    __syncthreads();
  }
  // pass 2: gather, push and write each particle to its slot, the next particle's
  // loads in flight meanwhile.  They are issued after the slot is reserved: the rare
  // global reservation returns into the slot's register, and the wait for it would
  // otherwise also wait for the prefetch.
  Raw<T> nxt;
  if (beg + (int)threadIdx.x < end) load_raw<T, true>(in, beg + threadIdx.x, nxt);
  for (int qq = beg + threadIdx.x; qq < end; qq += blockDim.x) {
    const Raw<T> r = nxt;
    int i, j, k;
    (void)decode_cell(r.cell, g, nullptr, i, j, k);
    const int nb = neighbour_of_cell(i, j, k, tx, ty, tz, tg);
    int slot;
    const unsigned long long own = __ballot(nb == 13);
    if (nb == 13) {
      const int lane = __lane_id();
      const int leader = __ffsll(own) - 1;
      int b0 = 0;
      if (lane == leader) b0 = atomicAdd(&cnt[13], __popcll(own));
      b0 = __shfl(b0, leader);
      slot = base[13] + b0 + __popcll(own & ((1ull << lane) - 1ull));
    } else {
      slot = nb >= 0 ? base[nb] + atomicAdd(&cnt[nb], 1) : atomicAdd(&cursor[tile_of(i, j, k, tg)], 1);
    }
    load_raw<T, true>(in, min(qq + (int)blockDim.x, end - 1), nxt);
    T ox = r.o[0], oy = r.o[1], oz = r.o[2];
    T ux = r.u[0], uy = r.u[1], uz = r.u[2];
    const int lx = box_index(i, t0x, g.nx), ly = box_index(j, t0y, g.ny), lz = box_index(k, t0z, g.nz);
    gather_push_one<T, ORDER>(box, F, g, lx, ly, lz, i, j, k, ox, oy, oz, ux, uy, uz, qdt2m, dtx, dty, dtz);
    out.u[0][slot] = ux;
    out.u[1][slot] = uy;
    out.u[2][slot] = uz;
    out.off[0][slot] = ox;
    out.off[1][slot] = oy;
    out.off[2][slot] = oz;
    out.cell[slot] = (i * g.ny + j) * g.nz + k;
    if (in.w) out.w[slot] = r.w;
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

// Fixed-point accumulators of the LDS deposition box.  A contribution (already scaled
// by 2^sh) becomes the nearest integer with one FMA and one integer subtraction:
// adding 1.5 * 2^p (p = 23 for FP32, 52 for FP64) to a value of magnitude at most
// 2^(p-1) rounds it to an integer that sits in the low bits of the sum.  FP32 runs
// accumulate int32 (ds_add_u32), FP64 runs int64 (ds_add_u64): integer LDS atomics
// retire about 20x faster than float ones on gfx950.
template <typename T>
struct Fixed;

// shift(): the scale exponent for a tile whose partial sums are bounded by 2^e_sum,
// whose single contributions are bounded by 2^e_max, with fewer than 2^h particles.
template <>
struct Fixed<float> {
  using acc_t = int;
  // node sums below 2^30, single contributions at most 2^22 (the rounding add's range)
  __device__ static inline int shift(int e_sum, int e_max, int h) { return min(30 - e_sum, 22 - e_max); }
  __device__ static inline acc_t fma_round(float a, float b) {
    return __float_as_int(fmaf(a, b, 12582912.0f)) - 0x4B400000;
  }
  __device__ static inline void add(acc_t* a, acc_t v) { atomicAdd(a, v); }
};

template <>
struct Fixed<double> {
  using acc_t = long long;
  // |sum| < 2^(h + e_max + sh) <= 2^62; each contribution at most 2^50
  __device__ static inline int shift(int e_sum, int e_max, int h) { return min(62 - e_max - h, 50 - e_max); }
  __device__ static inline acc_t fma_round(double a, double b) {
    return __double_as_longlong(fma(a, b, 6755399441055744.0)) - 0x4338000000000000LL;
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

// Adds the shape-weighted values sv[0..NVAL) (already scaled to fixed point) of one
// particle to NVAL consecutive components of the LDS box; ``at`` is the box index of
// the first support node.  Every atomic addresses ``at`` plus a constant, which the
// instruction carries as an immediate offset.
template <typename T, int ORDER, int NVAL>
__device__ inline void scatter_lds(typename Fixed<T>::acc_t* box, int at, T ox, T oy, T oz, const T* sv) {
  using S = Shape<T, ORDER>;
  using X = Box<S::NW>;
  constexpr int NW = S::NW;
  T wx[NW], wy[NW], wz[NW];
  S::weights(ox, wx);
  S::weights(oy, wy);
  S::weights(oz, wz);
  typename Fixed<T>::acc_t* b0 = box + at;
#pragma unroll
  for (int q = 0; q < NVAL; ++q) {
#pragma unroll
    for (int a = 0; a < NW; ++a) {
      const T xa = sv[q] * wx[a];
#pragma unroll
      for (int b = 0; b < NW; ++b) {
        const T xab = xa * wy[b];
#pragma unroll
        for (int cc = 0; cc < NW; ++cc)
          Fixed<T>::add(b0 + q * X::B3 + a * X::B2 + b * X::B + cc, Fixed<T>::fma_round(xab, wz[cc]));
      }
    }
  }
}

// The current of one particle into a float box whose J^x, J^y share one 64-bit word per
// node, J^y 2^32 + J^x in two's complement, followed by a J^z plane: one 64-bit LDS atomic
// stands for two 32-bit ones.  The rounding adds leave K + n in each half (K = 0x4B400000,
// |n| <= 2^22), so subtracting K 2^32 + K gives n_y 2^32 + n_x exactly, and since integer
// addition is exact the word sums to (sum n_y) 2^32 + sum n_x, from which both sums (each
// below 2^31 by the choice of scale) come back exactly (unpack_xy).
template <int ORDER>
__device__ inline void scatter_lds_packed_j(int* box, int at, float ox, float oy, float oz, const float* sv) {
  using S = Shape<float, ORDER>;
  using X = Box<S::NW>;
  constexpr int NW = S::NW;
  constexpr unsigned long long kBias = 0x4B4000004B400000ull;
  float wx[NW], wy[NW], wz[NW];
  S::weights(ox, wx);
  S::weights(oy, wy);
  S::weights(oz, wz);
  unsigned long long* xy = reinterpret_cast<unsigned long long*>(box) + at;
  int* z = box + 2 * X::B3 + at;
#pragma unroll
  for (int a = 0; a < NW; ++a) {
#pragma unroll
    for (int b = 0; b < NW; ++b) {
      const float wab = wx[a] * wy[b];
      const float xab = sv[0] * wab, yab = sv[1] * wab, zab = sv[2] * wab;
#pragma unroll
      for (int cc = 0; cc < NW; ++cc) {
        const int rel = a * X::B2 + b * X::B + cc;
        const unsigned lo = __float_as_uint(fmaf(xab, wz[cc], 12582912.0f));
        const unsigned hi = __float_as_uint(fmaf(yab, wz[cc], 12582912.0f));
        atomicAdd(xy + rel, (((unsigned long long)hi << 32) | lo) - kBias);
        atomicAdd(z + rel, Fixed<float>::fma_round(zab, wz[cc]));
      }
    }
  }
}
// NP pairs of values (sv[2 q], sv[2 q + 1]) into NP planes of packed 64-bit words, as
// scatter_lds_packed_j does for (J^x, J^y).
template <int ORDER, int NP>
__device__ inline void scatter_lds_pairs(int* box, int at, float ox, float oy, float oz, const float* sv) {
  using S = Shape<float, ORDER>;
  using X = Box<S::NW>;
  constexpr int NW = S::NW;
  constexpr unsigned long long kBias = 0x4B4000004B400000ull;
  float wx[NW], wy[NW], wz[NW];
  S::weights(ox, wx);
  S::weights(oy, wy);
  S::weights(oz, wz);
  unsigned long long* w0 = reinterpret_cast<unsigned long long*>(box) + at;
#pragma unroll
  for (int a = 0; a < NW; ++a) {
#pragma unroll
    for (int b = 0; b < NW; ++b) {
      const float wab = wx[a] * wy[b];
      float xab[2 * NP];
#pragma unroll
      for (int v = 0; v < 2 * NP; ++v) xab[v] = sv[v] * wab;
#pragma unroll
      for (int cc = 0; cc < NW; ++cc) {
        const int rel = a * X::B2 + b * X::B + cc;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          const unsigned lo = __float_as_uint(fmaf(xab[2 * q], wz[cc], 12582912.0f));
          const unsigned hi = __float_as_uint(fmaf(xab[2 * q + 1], wz[cc], 12582912.0f));
          atomicAdd(w0 + q * X::B3 + rel, (((unsigned long long)hi << 32) | lo) - kBias);
        }
      }
    }
  }
}
__device__ inline void unpack_xy(unsigned long long w, int& x, int& y) {
  x = (int)(unsigned)w;
  y = (int)((long long)(w - (unsigned long long)(long long)x) >> 32);
}

// Order of the particles inside a deposition chunk.  LDS atomics of a wave retire
// without bank conflicts when the 32 lanes of each half wave address distinct words
// modulo 32 (4-byte accumulators), or the 16 lanes of each quarter wave distinct
// 8-byte words modulo 16 (measured on gfx950).  All atomics of a particle are at its
// first support node plus a constant, so particles whose first nodes differ modulo
// KG never conflict: they are dealt round-robin over the KG residues, row r of the
// deal holding the r-th particle of every residue that has one.
template <typename T>
struct DepositOrder {
  static constexpr int KG = sizeof(typename Fixed<T>::acc_t) == 4 ? 32 : 16;
  static constexpr int CH = sizeof(typename Fixed<T>::acc_t) == 4 ? 1024 : 512;  // particles per chunk
  static constexpr int RMAX = CH / 4;  // deal rows; a chunk with more keeps its stored order
  static constexpr int U = CH / PIC_DEPOSIT_BLOCK;  // particles per thread and chunk, loaded together
  static_assert(CH % PIC_DEPOSIT_BLOCK == 0, "a chunk is a whole number of particles per thread");
};

// What the deposition needs of one particle: its cell and offsets at x, the velocity,
// the cell and offsets at x - dt v / 2, and the box indices of the first support
// node at both positions (-1 outside the box margin).
template <typename T>
struct DepositPoint {
  int i, j, k, ih, jh, kh, at_rho, at_j;
  T ox, oy, oz, hx, hy, hz, vx, vy, vz;
};

template <typename T, int ORDER, bool WJ>
__device__ inline bool locate(const Raw<T>& r, const GridGeom& g, int t0x, int t0y, int t0z, T hdtx, T hdty, T hdtz,
                              int* bad, DepositPoint<T>& d) {
  using X = Box<Shape<T, ORDER>::NW>;
  if (!decode_cell(r.cell, g, bad, d.i, d.j, d.k)) return false;
  d.ox = r.o[0];
  d.oy = r.o[1];
  d.oz = r.o[2];
  {
    const int lx = box_index(d.i, t0x, g.nx), ly = box_index(d.j, t0y, g.ny), lz = box_index(d.k, t0z, g.nz);
    d.at_rho = (lx >= 0 && ly >= 0 && lz >= 0) ? X::at(lx, ly, lz) : -1;
  }
  d.at_j = -1;
  if (WJ) {
    const T ig = inv_sqrt((T)1 + r.u[0] * r.u[0] + r.u[1] * r.u[1] + r.u[2] * r.u[2]);
    d.vx = r.u[0] * ig;
    d.vy = r.u[1] * ig;
    d.vz = r.u[2] * ig;
    // x^{n+1/2} = x^{n+1} - dt (v - v_gal) / 2
    d.hx = d.ox;
    d.hy = d.oy;
    d.hz = d.oz;
    d.ih = wrapi(d.i + advance_offset(d.hx, -hdtx * d.vx + (T)0.5 * (T)g.sgx), g.nx);
    d.jh = wrapi(d.j + advance_offset(d.hy, -hdty * d.vy + (T)0.5 * (T)g.sgy), g.ny);
    d.kh = wrapi(d.k + advance_offset(d.hz, -hdtz * d.vz + (T)0.5 * (T)g.sgz), g.nz);
    const int lx = box_index(d.ih, t0x, g.nx), ly = box_index(d.jh, t0y, g.ny), lz = box_index(d.kh, t0z, g.nz);
    d.at_j = (lx >= 0 && ly >= 0 && lz >= 0) ? X::at(lx, ly, lz) : -1;
  }
  return true;
}

// Scale bounds of one particle: |q w| (rho) and |q w v_c| (J^c), summed and maxed.
template <typename T, bool WJ>
__device__ inline void bound_add(const Raw<T>& r, T* sw, T* mw) {
  const T a = fabs(r.w);
  sw[0] += a;
  mw[0] = fmax(mw[0], a);
  if (WJ) {
    const T ig = inv_sqrt((T)1 + r.u[0] * r.u[0] + r.u[1] * r.u[1] + r.u[2] * r.u[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const T v = a * fabs(r.u[d] * ig);
      sw[1 + d] += v;
      mw[1 + d] = fmax(mw[1 + d], v);
    }
  }
}

// In-place exclusive prefix sum of a[0..n) by the whole block (wtot: one int per wave).
__device__ inline void block_exclusive_scan(int* a, int n, int* wtot) {
  const int per = (n + (int)blockDim.x - 1) / (int)blockDim.x;
  const int lo = min(n, (int)threadIdx.x * per), hi = min(n, lo + per);
  int s = 0;
  for (int e = lo; e < hi; ++e) s += a[e];
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  int x = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wtot[wave] = x;
  __syncthreads();
  int run = x - s;
  for (int w = 0; w < wave; ++w) run += wtot[w];
  for (int e = lo; e < hi; ++e) {
    const int v = a[e];
    a[e] = run;
    run += v;
  }
  __syncthreads();
}

// One block per tile: rho (at x) and J (at x - dt v/2) of the tile's particles are
// accumulated in LDS over a box of B = kTile + NW + 1 nodes per axis (the tile, the
// shape support and a one-cell margin for particles that moved since the grouping),
// then stored to the tile's staging slot; k_deposit_reduce adds the overlapping
// boxes on the grid.  (A particle outside the margin is added to the grid directly
// with global atomics.)  With next_counts, the tiles of the particles' cells (the
// next grouping) are counted: per tile in next_counts, per neighbour of this tile in
// nbr_counts[27 * tile ...] (what the next gather of this tile's particles reserves).
// LDS of a deposition workgroup besides the box.
template <typename T>
struct DepositLds {
  static constexpr int kWaves = PIC_DEPOSIT_BLOCK / 64;
  using O = DepositOrder<T>;
  T red[4 * kWaves];
  T redm[4 * kWaves];
  int shs[4];
  int cnt[27];
  int wtot[kWaves];
  int next_tile;
  int cross;  // faces of the box holding a nonzero value (see deposit_tile)
  __align__(16) int hist[O::KG];
  unsigned short kr[O::CH];
  unsigned short order[O::CH];
  unsigned rowmask[O::RMAX];
  int rowstart[O::RMAX];
};

// Deposition of one tile by the whole workgroup (see k_deposit_tiled).
template <typename T, int ORDER, bool WJ>
__device__ inline void deposit_tile(int tile, const GridGeom& g, const TileGeom& tg, const SpeciesView<T>& sp,
                                    const int* __restrict__ perm, const int* __restrict__ starts,
                                    const Batch<T*>& out, T* __restrict__ stage, T qdv, T hdtx, T hdty, T hdtz,
                                    int* bad, int* next_counts, int* nbr_counts, int* spill_flag, int* box_faces,
                                    typename Fixed<T>::acc_t* box, DepositLds<T>& L) {
  using S = Shape<T, ORDER>;
  using X = Box<S::NW>;
  using O = DepositOrder<T>;
  constexpr int ncomp = WJ ? 4 : 1;
  constexpr int kWaves = DepositLds<T>::kWaves;
  // Box planes: FP32 with J, (J^x, J^y) packed 64-bit words, J^z, then rho; otherwise rho, J^x, J^y, J^z.
  constexpr bool PACK = WJ && sizeof(T) == 4;
  typename Fixed<T>::acc_t* rbox = PACK ? box + 3 * X::B3 : box;
  T* red = L.red;
  T* redm = L.redm;
  int* shs = L.shs;
  int* cnt = L.cnt;
  int* wtot = L.wtot;
  int* hist = L.hist;
  unsigned short* kr = L.kr;
  unsigned short* order = L.order;
  unsigned* rowmask = L.rowmask;
  int* rowstart = L.rowstart;
  const int beg = starts[tile], end = starts[tile + 1];
  if (beg == end) return;
  if (tile == tg.ntiles) {  // invalid cells: never deposited, kept in the last bucket
    if (next_counts && threadIdx.x == 0) atomicAdd(&next_counts[tg.ntiles], end - beg);
    return;
  }
  int ti, tj, tk;
  tile_coords(tile, tg, ti, tj, tk);
  const int t0x = ti * kTile, t0y = tj * kTile, t0z = tk * kTile;
  // Fixed-point scales 2^sh[c], one per deposited component (rho, J^x, J^y, J^z).  A
  // node of this box receives from each particle of the tile at most MaxWeight * |q w|
  // / dV (rho) or MaxWeight * |q w v_c| / dV (J^c): every partial sum is bounded by
  // MaxWeight times the tile's sum of those magnitudes (< 2^e_sum), every contribution
  // by their max (< 2^e_max).  A tile of one chunk takes the bounds in the chunk's
  // first pass; a larger one in a pass of its own.
  const bool single = end - beg <= O::CH;
  T sw[4] = {0, 0, 0, 0}, mw[4] = {0, 0, 0, 0};
  auto publish_bounds = [&]() {  // wave partials -> red / redm
#pragma unroll
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
  };
  auto finish_bounds = [&]() {  // red / redm -> shs (threads 0..ncomp-1)
    if (threadIdx.x < ncomp) {
      const int c = threadIdx.x;
      T m = 0, x = 0;
      for (int w = 0; w < kWaves; ++w) {
        m += red[c * kWaves + w];
        x = fmax(x, redm[c * kWaves + w]);
      }
      if (g.det) m = x * (T)(end - beg);  // order-independent bound (see GridGeom::det)
      // a little slack on the bound covers the rounding of the FP sum itself
      int e_sum = 0, e_max = 0;
      (void)frexp(m * fabs(qdv) * (T)(MaxWeight<ORDER>::value * 1.001), &e_sum);
      (void)frexp(x * fabs(qdv) * (T)1.001, &e_max);
      shs[c] = Fixed<T>::shift(e_sum, e_max, 32 - __clz(end - beg));
    }
  };
  if (!single) {
    for (int q0 = beg + threadIdx.x; q0 < end; q0 += O::U * PIC_DEPOSIT_BLOCK) {
      int qi[O::U];
#pragma unroll
      for (int u = 0; u < O::U; ++u) qi[u] = min(q0 + u * PIC_DEPOSIT_BLOCK, end - 1);
      through_perm(perm, qi);
      Raw<T> r[O::U];
#pragma unroll
      for (int u = 0; u < O::U; ++u) {
        if (PIC_DEPOSIT_BOUND_LOAD)
          load_bound<T, WJ>(sp, qi[u], r[u]);
        else
          load_raw<T, WJ>(sp, qi[u], r[u]);
      }
#pragma unroll
      for (int u = 0; u < O::U; ++u)
        if (q0 + u * PIC_DEPOSIT_BLOCK < end) bound_add<T, WJ>(r[u], sw, mw);
    }
    publish_bounds();
    __syncthreads();
    finish_bounds();
  }
  {  // clear the box: 16-byte stores, then the words past the last whole 16 bytes
    constexpr int W = (int)(ncomp * X::B3 * sizeof(typename Fixed<T>::acc_t) / sizeof(int));
    int4* b4 = reinterpret_cast<int4*>(box);
#pragma unroll
    for (int k0 = 0; k0 < W / 4; k0 += PIC_DEPOSIT_BLOCK)
      if ((W / 4) % PIC_DEPOSIT_BLOCK == 0 || k0 + (int)threadIdx.x < W / 4) b4[k0 + threadIdx.x] = make_int4(0, 0, 0, 0);
    if ((int)threadIdx.x < W % 4) reinterpret_cast<int*>(box)[W / 4 * 4 + threadIdx.x] = 0;
  }
  if (threadIdx.x < 27) cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) L.cross = 0;  // read only after the chunk loop's barriers
  for (int cb = beg; cb < end; cb += O::CH) {
    const int nc = min(O::CH, end - cb);
    if (threadIdx.x < O::KG) hist[threadIdx.x] = 0;
    __syncthreads();
    // pass 1: residue of each particle's first support node and its rank among the chunk's
    // particles of that residue; all of a thread's particles in flight.  The residue is taken
    // from the particle's cell alone (rho's first node; one int per particle instead of its whole
    // record, with momentum and weight for the bounds of a single-chunk tile): the first support
    // node of the current shifts from it only when the half step crosses a cell face, and the
    // deal only orders the atomics, it does not change their sums.  PIC_DEPOSIT_CELL_KEY 0 keys
    // by the current's first node instead.
    if (PIC_DEPOSIT_CELL_KEY) {
      const int e0 = threadIdx.x;
      int qi[O::U];
#pragma unroll
      for (int u = 0; u < O::U; ++u) qi[u] = cb + min(e0 + u * PIC_DEPOSIT_BLOCK, nc - 1);
      through_perm(perm, qi);
      int c[O::U];
      Raw<T> r[O::U];
#pragma unroll
      for (int u = 0; u < O::U; ++u) {
        c[u] = sp.cell[qi[u]];
        if (single) load_bound<T, WJ>(sp, qi[u], r[u]);
      }
#pragma unroll
      for (int u = 0; u < O::U; ++u) {
        const int e = e0 + u * PIC_DEPOSIT_BLOCK;
        if (e < nc) {
          int i, j, k, key = 0;
          if (decode_cell(c[u], g, nullptr, i, j, k)) {
            const int lx = box_index(i, t0x, g.nx), ly = box_index(j, t0y, g.ny), lz = box_index(k, t0z, g.nz);
            if (lx >= 0 && ly >= 0 && lz >= 0) key = X::at(lx, ly, lz) & (O::KG - 1);
          }
          const int rk = atomicAdd(&hist[key], 1);
          kr[e] = (unsigned short)(rk * O::KG + key);
          if (single) bound_add<T, WJ>(r[u], sw, mw);
        }
      }
    } else {
      const int e0 = threadIdx.x;
      int qi[O::U];
#pragma unroll
      for (int u = 0; u < O::U; ++u) qi[u] = cb + min(e0 + u * PIC_DEPOSIT_BLOCK, nc - 1);
      through_perm(perm, qi);
      Raw<T> r[O::U];
#pragma unroll
      for (int u = 0; u < O::U; ++u) load_raw<T, WJ>(sp, qi[u], r[u]);
#pragma unroll
      for (int u = 0; u < O::U; ++u) {
        const int e = e0 + u * PIC_DEPOSIT_BLOCK;
        if (e < nc) {
          DepositPoint<T> d;
          int key = 0;
          if (locate<T, ORDER, WJ>(r[u], g, t0x, t0y, t0z, hdtx, hdty, hdtz, nullptr, d)) {
            const int at = WJ ? d.at_j : d.at_rho;
            key = at >= 0 ? (at & (O::KG - 1)) : 0;
          }
          const int rk = atomicAdd(&hist[key], 1);
          kr[e] = (unsigned short)(rk * O::KG + key);
          if (single) bound_add<T, WJ>(r[u], sw, mw);
        }
      }
    }
    if (single) publish_bounds();
    __syncthreads();
    if (single) finish_bounds();
    // row r of the deal: a bit per residue with an r-th particle, and the row's start
    int R = 0;
#pragma unroll
    for (int k = 0; k < O::KG; k += 4) {
      const int4 h4 = *reinterpret_cast<const int4*>(&hist[k]);
      R = max(R, max(max(h4.x, h4.y), max(h4.z, h4.w)));
    }
    if (R > O::RMAX) R = 0;  // too uneven to deal: stored order
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
      unsigned m = 0;
#pragma unroll 4
      for (int k = 0; k < O::KG; ++k) m |= (hist[k] > r ? 1u : 0u) << k;
      rowmask[r] = m;
      rowstart[r] = __popc(m);
    }
    __syncthreads();
    block_exclusive_scan(rowstart, R, wtot);
    for (int e = threadIdx.x; e < nc; e += blockDim.x) {
      if (R == 0) {
        order[e] = (unsigned short)e;
      } else {
        const int v = kr[e];
        const int r = v / O::KG, key = v % O::KG;
        order[rowstart[r] + __popc(rowmask[r] & ((1u << key) - 1u))] = (unsigned short)e;
      }
    }
    __syncthreads();
    int sh[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) sh[c] = (c < ncomp) ? shs[c] : 0;
    // pass 2: deposit in the dealt order, the next particle's loads in flight meanwhile
    Raw<T> nxt;
    if ((int)threadIdx.x < nc) {
      int q[1] = {cb + order[threadIdx.x]};
      through_perm(perm, q);
      load_raw<T, WJ>(sp, q[0], nxt);
    }
    for (int pos = threadIdx.x; pos < nc; pos += blockDim.x) {
      const Raw<T> r = nxt;
      {
        int q[1] = {cb + order[min(pos + (int)blockDim.x, nc - 1)]};
        through_perm(perm, q);
        load_raw<T, WJ>(sp, q[0], nxt);
      }
      DepositPoint<T> d;
      if (!locate<T, ORDER, WJ>(r, g, t0x, t0y, t0z, hdtx, hdty, hdtz, bad, d)) continue;
      if (next_counts) {  // the tile of this position groups the particle in the next step
        const int nb = neighbour_of_cell(d.i, d.j, d.k, ti, tj, tk, tg);
        const unsigned long long own = __ballot(nb == 13);
        if (nb == 13) {
          if (__lane_id() == __ffsll(own) - 1) atomicAdd(&cnt[13], __popcll(own));
        } else if (nb >= 0) {
          atomicAdd(&cnt[nb], 1);
        } else {
          atomicAdd(&next_counts[tile_of(d.i, d.j, d.k, tg)], 1);
        }
      }
      const T qw = qdv * r.w;
      if (d.at_rho >= 0) {
        const T sv[1] = {ldexp(qw, sh[0])};
        scatter_lds<T, ORDER, 1>(rbox, d.at_rho, d.ox, d.oy, d.oz, sv);
      } else {
        T* dst[1] = {out.p[0]};
        const T val[1] = {qw};
        scatter<T, ORDER>(g, d.i, d.j, d.k, d.ox, d.oy, d.oz, dst, val, 1);
        if (spill_flag) *spill_flag = 1;
      }
      if (WJ) {
        if (d.at_j >= 0) {
          const T sv[3] = {ldexp(qw * d.vx, sh[1]), ldexp(qw * d.vy, sh[2]), ldexp(qw * d.vz, sh[3])};
          if constexpr (PACK)
            scatter_lds_packed_j<ORDER>(box, d.at_j, d.hx, d.hy, d.hz, sv);
          else
            scatter_lds<T, ORDER, 3>(box + X::B3, d.at_j, d.hx, d.hy, d.hz, sv);
        } else {
          T* dst[3] = {out.p[1], out.p[2], out.p[3]};
          const T val[3] = {qw * d.vx, qw * d.vy, qw * d.vz};
          scatter<T, ORDER>(g, d.ih, d.jh, d.kh, d.hx, d.hy, d.hz, dst, val, 3);
          if (spill_flag) *spill_flag = 1;
        }
      }
    }
    __syncthreads();
  }
  if (next_counts && threadIdx.x < 27) {
    const int n = cnt[threadIdx.x];
    if (n > 0) atomicAdd(&next_counts[neighbour_key(threadIdx.x, ti, tj, tk, tg)], n);
    if (nbr_counts) nbr_counts[27 * tile + threadIdx.x] = n;
  }
  // Only particles that left the tile since the grouping reach the outermost layers of the
  // box (in-tile particles touch layers 1 .. B - 2), so with box_faces the tile stages only
  // the x and y layers that hold a nonzero value: bit f of its face mask (faces x-, y-, z- at
  // layer 0, then at layer B - 1) is set when face f does, and the reduction reads nothing
  // outside.  z rows are always staged whole (their ends share memory sectors with the rest).
  int faces = 0x3F;
  if (box_faces) {
    int mine = 4 | 32;  // faces this thread found nonzero, then OR-reduced over the wave: one atomic per wave
    for (int e = threadIdx.x; e < 4 * X::B2; e += blockDim.x) {
      const int k = e / X::B2, uv = e - k * X::B2, u = uv / X::B, v = uv - u * X::B;
      const int f = (k & 1) + 3 * (k >> 1);  // x-, y-, x+, y+
      const int l = k < 2 ? 0 : X::B - 1;
      const int n = (k & 1) == 0 ? X::at(l, u, v) : X::at(u, l, v);
      bool nz = rbox[n] != 0;
      if (WJ) {
        if constexpr (PACK)
          nz = nz || reinterpret_cast<const unsigned long long*>(box)[n] != 0ull || box[2 * X::B3 + n] != 0;
        else
          nz = nz || box[X::B3 + n] != 0 || box[2 * X::B3 + n] != 0 || box[3 * X::B3 + n] != 0;
      }
      if (nz) mine |= 1 << f;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mine |= __shfl_xor(mine, o, 64);
    if ((threadIdx.x & 63) == 0 && mine) atomicOr(&L.cross, mine);
    __syncthreads();
    faces = L.cross;
    if (threadIdx.x == 0) box_faces[tile] = faces;
  }
  const int lo[3] = {(faces & 1) ? 0 : 1, (faces & 2) ? 0 : 1, (faces & 4) ? 0 : 1};
  const int hi[3] = {(faces & 8) ? X::B - 1 : X::B - 2, (faces & 16) ? X::B - 1 : X::B - 2,
                     (faces & 32) ? X::B - 1 : X::B - 2};
  // the tile's slot in rows (StageRows): thread t writes vectors it = t + u * PIC_DEPOSIT_BLOCK,
  // four consecutive positions of row it / 4, every component, zeros outside the box row
  using RL = StageRows<ORDER>;
  static_assert(RL::B == X::B, "stage rows match the box");
  T* const dstage = stage + (size_t)tile * ncomp * RL::SLOT;
  const int sh0 = -shs[0], sh1 = -shs[1], sh2 = -shs[2], sh3 = -shs[3];
  for (int it = threadIdx.x; it < X::B2 * (RL::PZ / 4); it += blockDim.x) {
    const int r = it >> 2, p0 = (it & 3) * 4;
    const int lx = r / X::B, ly = r - lx * X::B;
    if (lx < lo[0] || lx > hi[0] || ly < lo[1] || ly > hi[1]) continue;
    T v[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int lz = p0 + i - RL::OFF;
      const bool in = lz >= 0 && lz < X::B;
      const int n = r * X::B + (in ? lz : 0);
      v[0][i] = in ? ldexp((T)rbox[n], sh0) : (T)0;
      if constexpr (PACK) {
        int jx, jy;
        unpack_xy(reinterpret_cast<const unsigned long long*>(box)[n], jx, jy);
        v[1][i] = in ? ldexp((T)jx, sh1) : (T)0;
        v[2][i] = in ? ldexp((T)jy, sh2) : (T)0;
        v[3][i] = in ? ldexp((T)box[2 * X::B3 + n], sh3) : (T)0;
      } else if (WJ) {
        v[1][i] = in ? ldexp((T)box[X::B3 + n], sh1) : (T)0;
        v[2][i] = in ? ldexp((T)box[2 * X::B3 + n], sh2) : (T)0;
        v[3][i] = in ? ldexp((T)box[3 * X::B3 + n], sh3) : (T)0;
      }
    }
    T* const row = dstage + r * RL::PZ + p0;
#pragma unroll
    for (int q = 0; q < ncomp; ++q) store4(row + q * RL::SLOT, v[q]);
  }
}

// Waves per SIMD the register budget allows: FP32 cubic 3 (its LDS box admits three
// workgroups per CU), FP32 linear 4, FP64 unconstrained.
// Cubic shapes: persistent workgroups, each taking tiles 0..ntiles (the last one the
// invalid-cell bucket) from the work counter until none is left, so that one tile's
// loads overlap other tiles' LDS work.  Linear shapes: one workgroup per tile (their
// smaller box leaves more workgroups resident).
template <typename T, int ORDER, bool WJ>
__global__ void __launch_bounds__(PIC_DEPOSIT_BLOCK, sizeof(T) == 4 ? (ORDER == 3 ? 3 : 4) : 1)
    k_deposit_tiled(GridGeom g, TileGeom tg, SpeciesView<T> sp, const int* __restrict__ perm,
                    const int* __restrict__ starts, Batch<T*> out, T* __restrict__ stage, T qdv, T hdtx, T hdty,
                    T hdtz, int* bad, int* next_counts, int* nbr_counts, int* work, int* spill_flag,
                    int* box_faces) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ DepositLds<T> L;
  auto* box = reinterpret_cast<typename Fixed<T>::acc_t*>(smem);
  if (ORDER == 3) {
    for (;;) {
      if (threadIdx.x == 0) L.next_tile = atomicAdd(work, 1);
      __syncthreads();
      const int tile = L.next_tile;
      __syncthreads();
      if (tile > tg.ntiles) break;
      deposit_tile<T, ORDER, WJ>(tile, g, tg, sp, perm, starts, out, stage, qdv, hdtx, hdty, hdtz, bad, next_counts,
                                 nbr_counts, spill_flag, box_faces, box, L);
    }
  } else {
    deposit_tile<T, ORDER, WJ>(blockIdx.x, g, tg, sp, perm, starts, out, stage, qdv, hdtx, hdty, hdtz, bad,
                               next_counts, nbr_counts, spill_flag, box_faces, box, L);
  }
}

// Tiles along z of the largest grid (1024 / kTile): the reduction's occupancy table.
constexpr int kMaxTilesZ = 1024 / kTile;

// Per axis, the (tile, box index) pairs whose boxes hold grid node x on grids that are
// whole multiples of the tile: its own tile t at l0 = x mod kTile + 1 - BASE, and
// t - 1 at l0 + kTile or t + 1 at l0 - kTile when that index lies inside the box.
template <int ORDER>
__device__ inline int axis_candidates(int x, int nt, int* t, int* l) {
  using S = Shape<float, ORDER>;
  using X = Box<S::NW>;
  const int tt = x / kTile, l0 = x % kTile + 1 - S::BASE;
  t[0] = tt;
  l[0] = l0;
  if (l0 + kTile < X::B) {
    t[1] = tt == 0 ? nt - 1 : tt - 1;
    l[1] = l0 + kTile;
    return 2;
  }
  if (l0 - kTile >= 0) {
    t[1] = tt == nt - 1 ? 0 : tt + 1;
    l[1] = l0 - kTile;
    return 2;
  }
  return 1;
}

// Sums, for every grid node, the staging boxes of the non-empty tiles that cover it
// and adds the sums to the nodal arrays; each node is owned by one thread, so no
// atomics.  Grids that are whole multiples of the tile; grid (z blocks, ny, nx).
template <typename T, int ORDER, int NCOMP>
__global__ void __launch_bounds__(256) k_deposit_reduce_whole(GridGeom g, TileGeom tg, const int* __restrict__ starts,
                                                              const T* __restrict__ stage, Batch<T*> out,
                                                              ReduceArgs<T> ra) {
  using X = Box<Shape<T, ORDER>::NW>;
  // per candidate tile of the row, by tz: 0 if empty, else 1 + 2 x its face mask
  __shared__ unsigned char occ[4][kMaxTilesZ];
  if (ra.next_flag && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0) *ra.next_flag = 0;
  // grid (z blocks, ny, nx) flattened and renumbered XCD-major: rows next to each other
  // read the same staging lines
  const int nzb = gridDim.x;
  const int L = xcd_major(blockIdx.x + nzb * (blockIdx.y + gridDim.y * blockIdx.z), nzb * gridDim.y * gridDim.z);
  const int z = (L % nzb) * blockDim.x + threadIdx.x;
  const int y = (L / nzb) % g.ny, x = L / (nzb * g.ny);
  int tx[2], lx[2], ty[2], ly[2], tz[2], lz[2];
  const int nxc = axis_candidates<ORDER>(x, tg.ntx, tx, lx);
  const int nyc = axis_candidates<ORDER>(y, tg.nty, ty, ly);
  // which tiles of the row's candidates hold particles (empty tiles' staging slots hold
  // stale data and are skipped): loaded once per block, so that every staging load
  // below issues without waiting for another global load
  for (int e = threadIdx.x; e < 4 * tg.ntz; e += blockDim.x) {
    const int ab = e / tg.ntz, t3 = e - ab * tg.ntz;
    const int a = ab >> 1, b = ab & 1;
    if (a < nxc && b < nyc) {
      const int tile = (tx[a] * tg.nty + ty[b]) * tg.ntz + t3;
      occ[ab][t3] = starts[tile] != starts[tile + 1] ? (unsigned char)(1 + 2 * (ra.box_faces ? ra.box_faces[tile] : 0x3F))
                                                     : (unsigned char)0;
    }
  }
  __syncthreads();
  if (z >= g.nz) return;
  const int nzc = axis_candidates<ORDER>(z, tg.ntz, tz, lz);
  // the eight combinations are unrolled: first every tile's occupancy, then the
  // staging loads of the occupied ones, all in flight before any sum (empty tiles'
  // staging slots hold stale data and are skipped)
  const size_t idx = ((size_t)x * g.ny + y) * g.nz + z;
  T acc[NCOMP];
#pragma unroll
  for (int q = 0; q < NCOMP; ++q) acc[q] = ra.start(q, out.p[q], idx);
  bool use[8];
  const T* sb[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int a = m >> 2, b = (m >> 1) & 1, c = m & 1;
    const bool present = a < nxc && b < nyc && c < nzc;
    const int ia = present ? a : 0, ib = present ? b : 0, ic = present ? c : 0;
    const int tile = (tx[ia] * tg.nty + ty[ib]) * tg.ntz + tz[ic];
    const int o = occ[2 * ia + ib][tz[ic]];
    const int f = o >> 1;  // the staged layers: 1 .. B - 2, plus the faces in f
    const bool in = (lx[ia] > 0 || (f & 1)) && (lx[ia] < X::B - 1 || (f & 8)) && (ly[ib] > 0 || (f & 2)) &&
                    (ly[ib] < X::B - 1 || (f & 16)) && (lz[ic] > 0 || (f & 4)) && (lz[ic] < X::B - 1 || (f & 32));
    use[m] = present && (o & 1) && in;
    sb[m] = stage + (size_t)tile * NCOMP * X::B3 + X::at(lx[ia], ly[ib], lz[ic]);
  }
  T v[8][NCOMP];
#pragma unroll
  for (int m = 0; m < 8; ++m)
#pragma unroll
    for (int q = 0; q < NCOMP; ++q) v[m][q] = use[m] ? sb[m][q * X::B3] : (T)0;
#pragma unroll
  for (int q = 0; q < NCOMP; ++q) {
#pragma unroll
    for (int m = 0; m < 8; ++m) acc[q] += v[m][q];
  }
  if (ra.flag && *ra.flag) {
#pragma unroll
    for (int q = 0; q < NCOMP; ++q) acc[q] += ra.take_spill(q, idx);
  }
#pragma unroll
  for (int q = 0; q < NCOMP; ++q) out.p[q][idx] = acc[q];
}

// The same sums over the row layout of deposit_tiled: each thread owns four consecutive nodes
// z0 .. z0+3 (z0 a multiple of 4) of one grid row and reads each covering box's four values
// as one aligned vector (zeros where the box ends inside the group).  Along z the group lies in
// tile tz = z0 / kTile and in the box of tz - 1 (first half of the tile) or of tz + 1 (second
// half); along x and y the candidates are those of the node.  Grid (z blocks, ny, nx),
// XCD-major.
template <typename T, int ORDER, int NCOMP>
__global__ void __launch_bounds__(256) k_deposit_reduce_rows(GridGeom g, TileGeom tg, const int* __restrict__ starts,
                                                             const T* __restrict__ stage, Batch<T*> out,
                                                             ReduceArgs<T> ra) {
  using RL = StageRows<ORDER>;
  static_assert(kTile == 8, "two groups of four nodes per tile along z");
  __shared__ unsigned char occ[4][kMaxTilesZ];
  if (ra.next_flag && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0) *ra.next_flag = 0;
  const int nzb = gridDim.x;
  const int L = xcd_major(blockIdx.x + nzb * (blockIdx.y + gridDim.y * blockIdx.z), nzb * gridDim.y * gridDim.z);
  const int z0 = 4 * ((L % nzb) * blockDim.x + threadIdx.x);
  const int y = (L / nzb) % g.ny, x = L / (nzb * g.ny);
  int tx[2], lx[2], ty[2], ly[2];
  const int nxc = axis_candidates<ORDER>(x, tg.ntx, tx, lx);
  const int nyc = axis_candidates<ORDER>(y, tg.nty, ty, ly);
  for (int e = threadIdx.x; e < 4 * tg.ntz; e += blockDim.x) {
    const int ab = e / tg.ntz, t3 = e - ab * tg.ntz;
    const int a = ab >> 1, b = ab & 1;
    if (a < nxc && b < nyc) {
      const int tile = (tx[a] * tg.nty + ty[b]) * tg.ntz + t3;
      occ[ab][t3] = starts[tile] != starts[tile + 1] ? (unsigned char)(1 + 2 * (ra.box_faces ? ra.box_faces[tile] : 0x3F))
                                                     : (unsigned char)0;
    }
  }
  __syncthreads();
  if (z0 >= g.nz) return;
  const int tzc = z0 / kTile, dz = z0 - tzc * kTile;  // dz = 0 or 4
  // the two z candidates (tile, position of z0 in its rows): c = tzc - 1, tzc or tzc, tzc + 1
  int tz[2], pz[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int c = (dz == 0 ? -1 : 0) + k;  // candidate tile offset from tzc
    tz[k] = tzc + c < 0 ? tg.ntz - 1 : (tzc + c >= tg.ntz ? 0 : tzc + c);
    pz[k] = dz - c * kTile + 1 - RL::BASE + RL::OFF;  // lz of z0 in that box, plus the row offset
  }
  const size_t idx = ((size_t)x * g.ny + y) * g.nz + z0;
  bool use[8];
  const T* sb[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int a = m >> 2, b = (m >> 1) & 1, c = m & 1;
    const bool present = a < nxc && b < nyc;
    const int ia = present ? a : 0, ib = present ? b : 0;
    const int tile = (tx[ia] * tg.nty + ty[ib]) * tg.ntz + tz[c];
    const int o = occ[2 * ia + ib][tz[c]];
    const int f = o >> 1;  // staged x, y layers: 1 .. B - 2, plus the faces in f (z rows whole)
    const bool in = (lx[ia] > 0 || (f & 1)) && (lx[ia] < RL::B - 1 || (f & 8)) && (ly[ib] > 0 || (f & 2)) &&
                    (ly[ib] < RL::B - 1 || (f & 16));
    use[m] = present && (o & 1) && in;
    sb[m] = stage + (size_t)tile * NCOMP * RL::SLOT + (lx[ia] * RL::B + ly[ib]) * RL::PZ + pz[c];
  }
  const bool spilled = ra.flag && *ra.flag;
  // one component at a time (its eight vectors in flight together); the empty asm keeps the
  // compiler from hoisting the next component's loads, which would multiply the registers held
#pragma unroll
  for (int q = 0; q < NCOMP; ++q) {
    T acc[4], v[8][4];
    if (ra.acc_mask & (q == 0 ? 1 : 2)) load4(out.p[q] + idx, acc);
    else if (q == 0 && ra.base) load4(ra.base + idx, acc);
    else
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] = (T)0;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      if (use[m]) load4(sb[m] + (size_t)q * RL::SLOT, v[m]);
      else
#pragma unroll
        for (int i = 0; i < 4; ++i) v[m][i] = (T)0;
    }
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] += v[m][i];
    if (spilled)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] += ra.take_spill(q, idx + i);
    store4(out.p[q] + idx, acc);
    asm volatile("" ::: "memory");
  }
}

// The same for any grid (partial tiles at the upper ends): candidate (tile, box index)
// pairs per axis over the periodic images x - n, x, x + n, box node l of tile t being
// grid node (t * kTile - 1 + BASE + l) mod n.
template <typename T, int ORDER>
__global__ void __launch_bounds__(256) k_deposit_reduce(GridGeom g, TileGeom tg, const int* __restrict__ starts,
                                                        const T* __restrict__ stage, Batch<T*> out, int ncomp,
                                                        ReduceArgs<T> ra) {
  using S = Shape<T, ORDER>;
  using X = Box<S::NW>;
  if (ra.next_flag && blockIdx.x == 0 && threadIdx.x == 0) *ra.next_flag = 0;
  const bool spilled = ra.flag && *ra.flag;
  const long long N = (long long)g.nx * g.ny * g.nz;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < N;
       idx += (long long)gridDim.x * blockDim.x) {
    const int z = (int)(idx % g.nz);
    const long long r = idx / g.nz;
    const int y = (int)(r % g.ny);
    const int x = (int)(r / g.ny);
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
        const int X0 = pos[d] + im * n[d];
        // tiles t with 0 <= X0 - (t*kTile - 1 + BASE) < B
        const int hi = (X0 + 1 - S::BASE);
        int tmax = hi >= 0 ? hi / kTile : -((-hi + kTile - 1) / kTile);
        for (int t = tmax; t >= 0 && cnt < 8; --t) {
          const int l = X0 - (t * kTile - 1 + S::BASE);
          if (l >= X::B) break;
          if (t < nt[d] && l >= 0) {
            ct[cnt] = t;
            cl[cnt] = l;
            ++cnt;
          }
        }
      }
      if (d == 0) nx_ = cnt; else if (d == 1) ny_ = cnt; else nz_ = cnt;
    }
    T acc[6] = {0, 0, 0, 0, 0, 0};
    for (int a = 0; a < nx_; ++a)
      for (int b = 0; b < ny_; ++b)
        for (int c = 0; c < nz_; ++c) {
          const int tile = (ctx_[a] * tg.nty + cty[b]) * tg.ntz + ctz[c];
          if (starts[tile] == starts[tile + 1]) continue;
          const int slot = ra.rows ? StageRows<ORDER>::SLOT : X::B3;
          const int at = ra.rows ? StageRows<ORDER>::at(clx[a], cly[b], clz[c]) : X::at(clx[a], cly[b], clz[c]);
          const T* sb = stage + (size_t)tile * ncomp * slot + at;
          for (int q = 0; q < ncomp; ++q) acc[q] += sb[(size_t)q * slot];
        }
    for (int q = 0; q < ncomp; ++q) out.p[q][idx] = ra.start(q, out.p[q], idx) + acc[q] + (spilled ? ra.take_spill(q, idx) : (T)0);
  }
}

// ---------------------------------------------------------------- reverse mode

// Over the S^3 support nodes of a particle in cell (i, j, k) with offsets o (cells), the
// shape-weighted sums val[v] = sum_n S_n A_v[n] and the position gradients
// grad[v][a] = sum_n dS_n/dx_a A_v[n] (x in cells) of NV nodal arrays.
template <typename T, int ORDER, int NV>
__device__ inline void stencil_sums(const GridGeom& g, int i, int j, int k, T ox, T oy, T oz, const T* const* A,
                                    T* val, T (*grad)[3]) {
  using S = Shape<T, ORDER>;
  constexpr int NW = S::NW;
  T wx[NW], wy[NW], wz[NW], gx[NW], gy[NW], gz[NW];
  S::weights(ox, wx);
  S::weights(oy, wy);
  S::weights(oz, wz);
  S::dweights(ox, gx);
  S::dweights(oy, gy);
  S::dweights(oz, gz);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    val[v] = 0;
    grad[v][0] = grad[v][1] = grad[v][2] = 0;
  }
  int kk[NW];
#pragma unroll
  for (int c = 0; c < NW; ++c) kk[c] = wrapi(k + c + S::BASE, g.nz);
#pragma unroll
  for (int a = 0; a < NW; ++a) {
    const int ii = wrapi(i + a + S::BASE, g.nx);
#pragma unroll
    for (int b = 0; b < NW; ++b) {
      const int jj = wrapi(j + b + S::BASE, g.ny);
      const size_t row = ((size_t)ii * g.ny + jj) * g.nz;
      const T wab = wx[a] * wy[b], gxab = gx[a] * wy[b], gyab = wx[a] * gy[b];
#pragma unroll
      for (int c = 0; c < NW; ++c) {
        const T w = wab * wz[c], dx = gxab * wz[c], dy = gyab * wz[c], dz = wab * gz[c];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const T x = A[v][row + kk[c]];
          val[v] += w * x;
          grad[v][0] += dx * x;
          grad[v][1] += dy * x;
          grad[v][2] += dz * x;
        }
      }
    }
  }
}

// The same sums from an LDS box; ``rd(n, v)`` reads the NV values of box node n and ``at``
// is the box index of the first support node.
template <typename T, int ORDER, int NV, typename RD>
__device__ inline void box_stencil_sums(RD rd, int at, T ox, T oy, T oz, T* val, T (*grad)[3]) {
  using S = Shape<T, ORDER>;
  using X = Box<S::NW>;
  constexpr int NW = S::NW;
  T wx[NW], wy[NW], wz[NW], gx[NW], gy[NW], gz[NW];
  S::weights(ox, wx);
  S::weights(oy, wy);
  S::weights(oz, wz);
  S::dweights(ox, gx);
  S::dweights(oy, gy);
  S::dweights(oz, gz);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    val[v] = 0;
    grad[v][0] = grad[v][1] = grad[v][2] = 0;
  }
#pragma unroll
  for (int a = 0; a < NW; ++a) {
#pragma unroll
    for (int b = 0; b < NW; ++b) {
      const T wab = wx[a] * wy[b], gxab = gx[a] * wy[b], gyab = wx[a] * gy[b];
#pragma unroll
      for (int c = 0; c < NW; ++c) {
        const T w = wab * wz[c], dx = gxab * wz[c], dy = gyab * wz[c], dz = wab * gz[c];
        T x[NV];
        rd(at + a * X::B2 + b * X::B + c, x);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          val[v] += w * x[v];
          grad[v][0] += dx * x[v];
          grad[v][1] += dy * x[v];
          grad[v][2] += dz * x[v];
        }
      }
    }
  }
}

// The three adjoint current components of box node n from 4-slot nodes (16 bytes for float).
__device__ inline void read_lj(const float* p, int n, float* v) {
  const float4 a = reinterpret_cast<const float4*>(p)[n];
  v[0] = a.x; v[1] = a.y; v[2] = a.z;
}
__device__ inline void read_lj(const double* p, int n, double* v) {
  const double2 a = reinterpret_cast<const double2*>(p)[2 * n];
  v[0] = a.x; v[1] = a.y; v[2] = p[4 * n + 2];
}

// Reverse mode of gather + Boris push + move + deposition of particle p at time n (cell
// (i, j, k) decoded).  The forward quantities are recomputed with the forward's own
// functions; then, with c = q w / dV, hdt = dt / (2 dx) and dtc = dt / dx per axis
// (positions in cells):
//   deposition: rho^{n+1} = c S(x^{n+1}), J^{n+1/2} = c v S(x^{n+1} - hdt v)
//     lx1 = lx + c sum lrho grad S(x^{n+1}) + G,   G = c sum (lJ . v) grad S(x^{n+1/2})
//     lv  = c sum lJ S(x^{n+1/2}) - hdt G + dtc lx1          (x^{n+1} = x^n + dtc v)
//     lu' = lu + (lv - v (v . lv)) / gamma                   (v = u'/gamma)
//   Boris (a = lu'):  lE = qdt2m (a + lum), lB = tf lt, lu^{n-1/2} = lum with
//     lup = s x a, ls = a x up, lum = a + lup + t x lup - (tf / gamma_-^2) (B . lt) um,
//     lt = lup x um + sf ls - sf^2 t (t . ls)
//   gather: lx^n = lx1 + sum_m lF_m grad F_m(x^n);  lF = (lE, lB) goes to lamF for the
//   scatter onto the nodal grids.
// Immobile species (never pushed, rho only): lx += c sum lrho grad S(x).
// The stencil sums come from the samplers: sF(i, j, k, o.., f, gf) over E, B (6) and
// sL<C0, NV>(i, j, k, o.., val, grad) over the adjoint sources (rho 0, J 1..3).
template <typename T, int ORDER, class SF, class SL1, class SL3>
__device__ inline void adjoint_one(const GridGeom& g, const SpeciesView<T>& sp, const Batch<T*>& lam,
                                   const Batch<T*>& lamF, int p, int i, int j, int k, T qdt2m, T qdv, T dtx, T dty,
                                   T dtz, bool mobile, SF sF, SL1 sRho, SL3 sJ) {
  const T ox = sp.off[0][p], oy = sp.off[1][p], oz = sp.off[2][p];
  const T c = qdv * (sp.w ? sp.w[p] : (T)sp.w_const);
  T lx[3] = {lam.p[0][p], lam.p[1][p], lam.p[2][p]};
  if (!mobile) {
    T rv[1], rg[1][3];
    sRho(i, j, k, ox, oy, oz, rv, rg);
#pragma unroll
    for (int a = 0; a < 3; ++a) lam.p[a][p] = lx[a] + c * rg[0][a];
#pragma unroll
    for (int m = 0; m < 6; ++m) lamF.p[m][p] = 0;
    return;
  }
  const T lu[3] = {lam.p[3][p], lam.p[4][p], lam.p[5][p]};
  // forward: gather at x^n (with gradients), push, move
  T f[6], gf[6][3];
  sF(i, j, k, ox, oy, oz, f, gf);
  T ux = sp.u[0][p], uy = sp.u[1][p], uz = sp.u[2][p];
  BorisState<T> b;
  boris(f, qdt2m, ux, uy, uz, b);
  const T ig = inv_sqrt((T)1 + ux * ux + uy * uy + uz * uz);
  const T v[3] = {ux * ig, uy * ig, uz * ig};
  T o1x = ox, o1y = oy, o1z = oz;  // the forward's move and half position (g.sg* = 0: no Galilean reverse mode)
  const int i1 = wrapi(i + advance_offset(o1x, dtx * ux * ig - (T)g.sgx), g.nx);
  const int j1 = wrapi(j + advance_offset(o1y, dty * uy * ig - (T)g.sgy), g.ny);
  const int k1 = wrapi(k + advance_offset(o1z, dtz * uz * ig - (T)g.sgz), g.nz);
  const T hd[3] = {(T)0.5 * dtx, (T)0.5 * dty, (T)0.5 * dtz};
  T hx = o1x, hy = o1y, hz = o1z;
  const int ih = wrapi(i1 + advance_offset(hx, -hd[0] * v[0] + (T)0.5 * (T)g.sgx), g.nx);
  const int jh = wrapi(j1 + advance_offset(hy, -hd[1] * v[1] + (T)0.5 * (T)g.sgy), g.ny);
  const int kh = wrapi(k1 + advance_offset(hz, -hd[2] * v[2] + (T)0.5 * (T)g.sgz), g.nz);
  // deposition
  T rv[1], rg[1][3], jv[3], jg[3][3];
  sRho(i1, j1, k1, o1x, o1y, o1z, rv, rg);
  sJ(ih, jh, kh, hx, hy, hz, jv, jg);
  const T dtc[3] = {dtx, dty, dtz};
  T lx1[3], lv[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T G = c * (v[0] * jg[0][a] + v[1] * jg[1][a] + v[2] * jg[2][a]);
    lx1[a] = lx[a] + c * rg[0][a] + G;
    lv[a] = c * jv[a] - hd[a] * G;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) lv[a] += dtc[a] * lx1[a];
  const T vl = v[0] * lv[0] + v[1] * lv[1] + v[2] * lv[2];
  T ax = lu[0] + (lv[0] - v[0] * vl) * ig;
  T ay = lu[1] + (lv[1] - v[1] * vl) * ig;
  T az = lu[2] + (lv[2] - v[2] * vl) * ig;
  // Boris, reversed
  const T lupx = b.sy * az - b.sz * ay, lupy = b.sz * ax - b.sx * az, lupz = b.sx * ay - b.sy * ax;  // s x a
  const T lsx = ay * b.upz - az * b.upy, lsy = az * b.upx - ax * b.upz, lsz = ax * b.upy - ay * b.upx;  // a x up
  const T tls = b.tx * lsx + b.ty * lsy + b.tz * lsz;
  const T sf2 = b.sf * b.sf;
  const T ltx = (lupy * b.umz - lupz * b.umy) + b.sf * lsx - sf2 * b.tx * tls;
  const T lty = (lupz * b.umx - lupx * b.umz) + b.sf * lsy - sf2 * b.ty * tls;
  const T ltz = (lupx * b.umy - lupy * b.umx) + b.sf * lsz - sf2 * b.tz * tls;
  const T ig2 = inv_sqrt((T)1 + b.umx * b.umx + b.umy * b.umy + b.umz * b.umz);
  const T ktf = -b.tf * ig2 * ig2 * (f[3] * ltx + f[4] * lty + f[5] * ltz);
  const T lumx = ax + lupx + (b.ty * lupz - b.tz * lupy) + ktf * b.umx;
  const T lumy = ay + lupy + (b.tz * lupx - b.tx * lupz) + ktf * b.umy;
  const T lumz = az + lupz + (b.tx * lupy - b.ty * lupx) + ktf * b.umz;
  const T lF[6] = {qdt2m * (ax + lumx), qdt2m * (ay + lumy), qdt2m * (az + lumz),
                   b.tf * ltx,          b.tf * lty,          b.tf * ltz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T x = lx1[a];
#pragma unroll
    for (int m = 0; m < 6; ++m) x += lF[m] * gf[m][a];
    lam.p[a][p] = x;
  }
  lam.p[3][p] = lumx;
  lam.p[4][p] = lumy;
  lam.p[5][p] = lumz;
#pragma unroll
  for (int m = 0; m < 6; ++m) lamF.p[m][p] = lF[m];
}

// One particle per thread (slot q -> particle perm[q]), every stencil read from the grids.
template <typename T, int ORDER>
__global__ void __launch_bounds__(256) k_particle_adjoint(GridGeom g, SpeciesView<T> sp, Batch<T*> lam,
                                                          const int* __restrict__ perm, Batch<const T*> F,
                                                          Batch<const T*> L, Batch<T*> lamF, T qdt2m, T qdv, T dtx,
                                                          T dty, T dtz, int mobile) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= sp.n) return;
  const int p = perm ? perm[q] : (int)q;
  int i, j, k;
  if (!decode_cell(sp.cell[p], g, nullptr, i, j, k)) {  // never pushed nor deposited: adjoint passes through
#pragma unroll
    for (int m = 0; m < 6; ++m) lamF.p[m][p] = 0;
    return;
  }
  const T* LJ[3] = {L.p[1], L.p[2], L.p[3]};
  auto sF = [&](int a, int b, int c, T x, T y, T z, T* val, T (*grad)[3]) {
    stencil_sums<T, ORDER, 6>(g, a, b, c, x, y, z, F.p, val, grad);
  };
  auto sRho = [&](int a, int b, int c, T x, T y, T z, T* val, T (*grad)[3]) {
    stencil_sums<T, ORDER, 1>(g, a, b, c, x, y, z, L.p, val, grad);
  };
  auto sJ = [&](int a, int b, int c, T x, T y, T z, T* val, T (*grad)[3]) {
    stencil_sums<T, ORDER, 3>(g, a, b, c, x, y, z, LJ, val, grad);
  };
  adjoint_one<T, ORDER>(g, sp, lam, lamF, p, i, j, k, qdt2m, qdv, dtx, dty, dtz, mobile != 0, sF, sRho, sJ);
}

// One block per tile of the grouping of the particles' cells at n (slots [starts[t],
// starts[t+1]) through perm): the adjoint currents (4 slots per node), E, B (GatherBox
// layout) and the adjoint charge (a plane of its own) staged over the tile's box in LDS, in
// that order, so that every plane starts aligned to its widest read.  x^n, x^{n+1} and x^{n+1/2} lie
// within one cell of the tile, inside the box; anything outside is read from the grids.
// Block ntiles passes the particles with invalid cells through.
template <typename T, int ORDER>
__global__ void __launch_bounds__(PIC_GATHER_BLOCK) k_particle_adjoint_tiled(
    GridGeom g, TileGeom tg, SpeciesView<T> sp, Batch<T*> lam, const int* __restrict__ perm,
    const int* __restrict__ starts, Batch<const T*> F, Batch<const T*> L, Batch<T*> lamF, T qdt2m, T qdv, T dtx,
    T dty, T dtz, int mobile) {
  using S = Shape<T, ORDER>;
  using X = Box<S::NW>;
  using GB = GatherBox<T, X::B3>;
  extern __shared__ __align__(16) unsigned char smem[];
  T* ljbox = reinterpret_cast<T*>(smem);
  T* fbox = ljbox + (size_t)X::B3 * 4;
  T* lrbox = fbox + (size_t)X::B3 * GB::SLOTS;
  const int tile = xcd_major(blockIdx.x, gridDim.x);
  const int beg = starts[tile], end = starts[tile + 1];
  if (beg == end) return;
  if (tile == tg.ntiles) {
    for (int q = beg + threadIdx.x; q < end; q += blockDim.x) {
      const int p = perm[q];
#pragma unroll
      for (int m = 0; m < 6; ++m) lamF.p[m][p] = 0;
    }
    return;
  }
  int tx, ty, tz;
  tile_coords(tile, tg, tx, ty, tz);
  const int t0x = tx * kTile, t0y = ty * kTile, t0z = tz * kTile;
  if (mobile) load_field_box<T, ORDER, true>(fbox, F, g, t0x, t0y, t0z);
  {
    constexpr int PER = (X::B3 + PIC_GATHER_BLOCK - 1) / PIC_GATHER_BLOCK;
    const int ox0 = t0x - 1 + S::BASE, oy0 = t0y - 1 + S::BASE, oz0 = t0z - 1 + S::BASE;
    T v[PER][4];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = min((int)threadIdx.x + u * PIC_GATHER_BLOCK, X::B3 - 1);
      const int lx = e / X::B2, ly = (e / X::B) % X::B, lz = e % X::B;
      const size_t gi = ((size_t)wrap3(ox0 + lx, g.nx) * g.ny + wrap3(oy0 + ly, g.ny)) * g.nz + wrap3(oz0 + lz, g.nz);
#pragma unroll
      for (int c = 0; c < 4; ++c) v[u][c] = L.p[c][gi];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = (int)threadIdx.x + u * PIC_GATHER_BLOCK;
      if (e < X::B3) {
        lrbox[e] = v[u][0];
#pragma unroll
        for (int c = 0; c < 3; ++c) ljbox[e * 4 + c] = v[u][1 + c];
      }
    }
  }
  __syncthreads();
  const T* LJ[3] = {L.p[1], L.p[2], L.p[3]};
  auto at_of = [&](int a, int b, int c) {
    const int lx = box_index(a, t0x, g.nx), ly = box_index(b, t0y, g.ny), lz = box_index(c, t0z, g.nz);
    return (lx >= 0 && ly >= 0 && lz >= 0) ? X::at(lx, ly, lz) : -1;
  };
  auto sF = [&](int a, int b, int c, T x, T y, T z, T* val, T (*grad)[3]) {
    const int at = at_of(a, b, c);
    if (at >= 0) box_stencil_sums<T, ORDER, 6>([&](int n, T* v) { GB::read(fbox, n, v); }, at, x, y, z, val, grad);
    else stencil_sums<T, ORDER, 6>(g, a, b, c, x, y, z, F.p, val, grad);
  };
  auto sRho = [&](int a, int b, int c, T x, T y, T z, T* val, T (*grad)[3]) {
    const int at = at_of(a, b, c);
    if (at >= 0) box_stencil_sums<T, ORDER, 1>([&](int n, T* v) { v[0] = lrbox[n]; }, at, x, y, z, val, grad);
    else stencil_sums<T, ORDER, 1>(g, a, b, c, x, y, z, L.p, val, grad);
  };
  auto sJ = [&](int a, int b, int c, T x, T y, T z, T* val, T (*grad)[3]) {
    const int at = at_of(a, b, c);
    if (at >= 0) box_stencil_sums<T, ORDER, 3>([&](int n, T* v) { read_lj(ljbox, n, v); }, at, x, y, z, val, grad);
    else stencil_sums<T, ORDER, 3>(g, a, b, c, x, y, z, LJ, val, grad);
  };
  for (int q = beg + threadIdx.x; q < end; q += blockDim.x) {
    const int p = perm[q];
    int i, j, k;
    (void)decode_cell(sp.cell[p], g, nullptr, i, j, k);
    adjoint_one<T, ORDER>(g, sp, lam, lamF, p, i, j, k, qdt2m, qdv, dtx, dty, dtz, mobile != 0, sF, sRho, sJ);
  }
}

// Six per-particle values val_v[p] spread with the particle's shape at its position onto
// nodal grids: one block per tile of the grouping (slots [starts[t], starts[t+1]) through
// perm), accumulated in a fixed-point LDS box per component (scales from the tile's sum and
// max of |val_v|, as in the deposition) and stored to the tile's staging slot for
// k_deposit_reduce*; a particle outside the box margin goes to the grids with atomics.
// The particles of each chunk are dealt over the residues of their first support node, as
// in the deposition, so that the lanes of a wave hit distinct LDS banks.  FP32 packs the
// components pairwise into 64-bit words (scatter_lds_pairs).
template <typename T, int ORDER>
__global__ void __launch_bounds__(256) k_scatter_tiled(GridGeom g, TileGeom tg, SpeciesView<T> sp,
                                                       const int* __restrict__ perm, const int* __restrict__ starts,
                                                       Batch<const T*> val, Batch<T*> out, T* __restrict__ stage) {
  using S = Shape<T, ORDER>;
  using X = Box<S::NW>;
  using O = DepositOrder<T>;
  constexpr int NV = 6;
  constexpr int kWaves = 256 / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  auto* box = reinterpret_cast<typename Fixed<T>::acc_t*>(smem);
  __shared__ T red[NV * kWaves], redm[NV * kWaves];
  __shared__ int shs[NV];
  __shared__ int wtot[kWaves];
  __shared__ __align__(16) int hist[O::KG];
  __shared__ unsigned short kr[O::CH];
  __shared__ unsigned short order[O::CH];
  __shared__ unsigned rowmask[O::RMAX];
  __shared__ int rowstart[O::RMAX];
  const int tile = xcd_major(blockIdx.x, gridDim.x);
  const int beg = starts[tile], end = starts[tile + 1];
  if (beg == end) return;
  int ti, tj, tk;
  tile_coords(tile, tg, ti, tj, tk);
  const int t0x = ti * kTile, t0y = tj * kTile, t0z = tk * kTile;
  T sw[NV], mw[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) sw[v] = mw[v] = 0;
  for (int q = beg + threadIdx.x; q < end; q += blockDim.x) {
    const int p = perm ? perm[q] : q;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T a = fabs(val.p[v][p]);
      sw[v] += a;
      mw[v] = fmax(mw[v], a);
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    for (int o = 32; o > 0; o >>= 1) {
      sw[v] += __shfl_xor(sw[v], o, 64);
      mw[v] = fmax(mw[v], __shfl_xor(mw[v], o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
      red[v * kWaves + (threadIdx.x >> 6)] = sw[v];
      redm[v * kWaves + (threadIdx.x >> 6)] = mw[v];
    }
  }
  for (int e = threadIdx.x; e < NV * X::B3; e += blockDim.x) box[e] = 0;
  __syncthreads();
  if (threadIdx.x < NV) {
    const int v = threadIdx.x;
    T m = 0, x = 0;
    for (int w = 0; w < kWaves; ++w) {
      m += red[v * kWaves + w];
      x = fmax(x, redm[v * kWaves + w]);
    }
    if (g.det) m = x * (T)(end - beg);  // order-independent bound (see GridGeom::det)
    int e_sum = 0, e_max = 0;
    (void)frexp(m * (T)(MaxWeight<ORDER>::value * 1.001), &e_sum);
    (void)frexp(x * (T)1.001, &e_max);
    shs[v] = Fixed<T>::shift(e_sum, e_max, 32 - __clz(end - beg));
  }
  __syncthreads();
  int sh[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) sh[v] = shs[v];
  auto box_at = [&](int p, int& i, int& j, int& k) {  // -2: invalid cell, -1: outside the box
    if (!decode_cell(sp.cell[p], g, nullptr, i, j, k)) return -2;
    const int lx = box_index(i, t0x, g.nx), ly = box_index(j, t0y, g.ny), lz = box_index(k, t0z, g.nz);
    return (lx >= 0 && ly >= 0 && lz >= 0) ? X::at(lx, ly, lz) : -1;
  };
  for (int cb = beg; cb < end; cb += O::CH) {
    const int nc = min(O::CH, end - cb);
    if (threadIdx.x < O::KG) hist[threadIdx.x] = 0;
    __syncthreads();
    for (int e = threadIdx.x; e < nc; e += blockDim.x) {
      const int p = perm ? perm[cb + e] : cb + e;
      int i, j, k;
      const int at = box_at(p, i, j, k);
      const int key = at >= 0 ? (at & (O::KG - 1)) : 0;
      const int rk = atomicAdd(&hist[key], 1);
      kr[e] = (unsigned short)(rk * O::KG + key);
    }
    __syncthreads();
    int R = 0;
#pragma unroll
    for (int k = 0; k < O::KG; k += 4) {
      const int4 h4 = *reinterpret_cast<const int4*>(&hist[k]);
      R = max(R, max(max(h4.x, h4.y), max(h4.z, h4.w)));
    }
    if (R > O::RMAX) R = 0;  // too uneven to deal: stored order
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
      unsigned m = 0;
#pragma unroll 4
      for (int k = 0; k < O::KG; ++k) m |= (hist[k] > r ? 1u : 0u) << k;
      rowmask[r] = m;
      rowstart[r] = __popc(m);
    }
    __syncthreads();
    block_exclusive_scan(rowstart, R, wtot);
    for (int e = threadIdx.x; e < nc; e += blockDim.x) {
      if (R == 0) {
        order[e] = (unsigned short)e;
      } else {
        const int v = kr[e];
        const int r = v / O::KG, key = v % O::KG;
        order[rowstart[r] + __popc(rowmask[r] & ((1u << key) - 1u))] = (unsigned short)e;
      }
    }
    __syncthreads();
    for (int pos = threadIdx.x; pos < nc; pos += blockDim.x) {
      const int e = order[pos];
      const int p = perm ? perm[cb + e] : cb + e;
      int i, j, k;
      const int at = box_at(p, i, j, k);
      if (at == -2) continue;
      const T ox = sp.off[0][p], oy = sp.off[1][p], oz = sp.off[2][p];
      T x[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) x[v] = val.p[v][p];
      if (at >= 0) {
        T sv[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) sv[v] = ldexp(x[v], sh[v]);
        if constexpr (sizeof(T) == 4)
          scatter_lds_pairs<ORDER, NV / 2>(box, at, ox, oy, oz, sv);
        else
          scatter_lds<T, ORDER, NV>(box, at, ox, oy, oz, sv);
      } else {
        scatter<T, ORDER>(g, i, j, k, ox, oy, oz, out.p, x, NV);
      }
    }
    __syncthreads();
  }
  T* dstage = stage + (size_t)tile * NV * X::B3;
  if constexpr (sizeof(T) == 4) {
    const unsigned long long* w = reinterpret_cast<const unsigned long long*>(box);
    for (int e = threadIdx.x; e < (NV / 2) * X::B3; e += blockDim.x) {
      const int q = e / X::B3, n = e - q * X::B3;
      int lo, hi;
      unpack_xy(w[e], lo, hi);
      dstage[2 * q * X::B3 + n] = ldexp((T)lo, -shs[2 * q]);
      dstage[(2 * q + 1) * X::B3 + n] = ldexp((T)hi, -shs[2 * q + 1]);
    }
  } else {
    for (int e = threadIdx.x; e < NV * X::B3; e += blockDim.x) dstage[e] = ldexp((T)box[e], -shs[e / X::B3]);
  }
}

// ---------------------------------------------------------------- fully staggered comparison cycle

// Half-cell Yee offsets (x, y, z) of E^x, E^y, E^z, B^x, B^y, B^z (J as E), in half cells.
__constant__ int kYee[6][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {0, 1, 1}, {1, 0, 1}, {1, 1, 0}};

// Cell and offset of x - 1/2 cell along one axis (h = 1) or of x itself (h = 0).
template <typename T>
__device__ inline void half_back(int& i, T& o, int h, int n) {
  if (h) {
    o -= (T)0.5;
    if (o < (T)0) {
      o += (T)1;
      i = (i == 0) ? n - 1 : i - 1;
    }
  }
}

// sum_n S(x - x_n) A[n] over the S^3 support nodes (from the grid).
template <typename T, int ORDER>
__device__ inline T stencil_value(const GridGeom& g, int i, int j, int k, T ox, T oy, T oz, const T* __restrict__ A) {
  using S = Shape<T, ORDER>;
  constexpr int NW = S::NW;
  T wx[NW], wy[NW], wz[NW];
  S::weights(ox, wx);
  S::weights(oy, wy);
  S::weights(oz, wz);
  int kk[NW];
#pragma unroll
  for (int c = 0; c < NW; ++c) kk[c] = wrapi(k + c + S::BASE, g.nz);
  T acc = 0;
#pragma unroll
  for (int a = 0; a < NW; ++a) {
    const int ii = wrapi(i + a + S::BASE, g.nx);
#pragma unroll
    for (int b = 0; b < NW; ++b) {
      const size_t row = ((size_t)ii * g.ny + wrapi(j + b + S::BASE, g.ny)) * g.nz;
      const T wab = wx[a] * wy[b];
#pragma unroll
      for (int c = 0; c < NW; ++c) acc += wab * wz[c] * A[row + kk[c]];
    }
  }
  return acc;
}

// Gather + push of the staggered cycle, one particle per thread, in place: each component of
// E, B interpolated from its own Yee positions (the shape centred on x_i + delta_c, i.e. at
// x - delta_c from the nodes), then the same Boris push and move as the hybrid cycle.
template <typename T, int ORDER>
__global__ void __launch_bounds__(256) k_gather_push_yee(GridGeom g, Batch<const T*> F, SpeciesView<T> sp, T qdt2m,
                                                         T dtx, T dty, T dtz) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= sp.n) return;
  int i, j, k;
  if (!decode_cell(sp.cell[p], g, nullptr, i, j, k)) return;
  T ox = sp.off[0][p], oy = sp.off[1][p], oz = sp.off[2][p];
  T f[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    int a = i, b = j, d = k;
    T x = ox, y = oy, z = oz;
    half_back(a, x, kYee[c][0], g.nx);
    half_back(b, y, kYee[c][1], g.ny);
    half_back(d, z, kYee[c][2], g.nz);
    f[c] = stencil_value<T, ORDER>(g, a, b, d, x, y, z, F.p[c]);
  }
  T ux = sp.u[0][p], uy = sp.u[1][p], uz = sp.u[2][p];
  BorisState<T> bs;
  boris(f, qdt2m, ux, uy, uz, bs);
  const T ig = inv_sqrt((T)1 + ux * ux + uy * uy + uz * uz);
  i = wrapi(i + advance_offset(ox, dtx * ux * ig - (T)g.sgx), g.nx);
  j = wrapi(j + advance_offset(oy, dty * uy * ig - (T)g.sgy), g.ny);
  k = wrapi(k + advance_offset(oz, dtz * uz * ig - (T)g.sgz), g.nz);
  sp.u[0][p] = ux;
  sp.u[1][p] = uy;
  sp.u[2][p] = uz;
  sp.off[0][p] = ox;
  sp.off[1][p] = oy;
  sp.off[2][p] = oz;
  sp.cell[p] = (i * g.ny + j) * g.nz + k;
}

// Deposition of the staggered cycle, one particle per thread, with global atomics: rho^{n+1} on
// the nodes at x^{n+1}; J^d = q w v_d onto its own Yee positions at x^{n+1/2} (the hybrid cycle's
// half position), i.e. at x^{n+1/2} - delta_d from the nodes.
template <typename T, int ORDER>
__global__ void __launch_bounds__(256) k_deposit_yee(GridGeom g, SpeciesView<T> sp, Batch<T*> out, T qdv, T hdtx,
                                                     T hdty, T hdtz, int with_j) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= sp.n) return;
  int i, j, k;
  if (!decode_cell(sp.cell[p], g, nullptr, i, j, k)) return;
  const T ox = sp.off[0][p], oy = sp.off[1][p], oz = sp.off[2][p];
  const T qw = qdv * (sp.w ? sp.w[p] : (T)sp.w_const);
  {
    T* dst[1] = {out.p[0]};
    const T val[1] = {qw};
    scatter<T, ORDER>(g, i, j, k, ox, oy, oz, dst, val, 1);
  }
  if (!with_j) return;
  const T ux = sp.u[0][p], uy = sp.u[1][p], uz = sp.u[2][p];
  const T ig = inv_sqrt((T)1 + ux * ux + uy * uy + uz * uz);
  const T v[3] = {ux * ig, uy * ig, uz * ig};
  T hx = ox, hy = oy, hz = oz;
  const int ih = wrapi(i + advance_offset(hx, -hdtx * v[0] + (T)0.5 * (T)g.sgx), g.nx);
  const int jh = wrapi(j + advance_offset(hy, -hdty * v[1] + (T)0.5 * (T)g.sgy), g.ny);
  const int kh = wrapi(k + advance_offset(hz, -hdtz * v[2] + (T)0.5 * (T)g.sgz), g.nz);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int a = ih, b = jh, c = kh;
    T x = hx, y = hy, z = hz;
    half_back(a, x, kYee[d][0], g.nx);
    half_back(b, y, kYee[d][1], g.ny);
    half_back(c, z, kYee[d][2], g.nz);
    T* dst[1] = {out.p[1 + d]};
    const T val[1] = {qw * v[d]};
    scatter<T, ORDER>(g, a, b, c, x, y, z, dst, val, 1);
  }
}

// Tiled gather + push of the staggered cycle: one block per tile of the grouping of the particles'
// cells (slots [starts[t], starts[t+1]) through perm), E, B staged over the tile's box in LDS
// (FieldSlots layout); each component read at its own shifted stencil; particles updated in
// place.  Block ntiles (invalid cells) does nothing.
template <typename T, int ORDER>
__global__ void __launch_bounds__(PIC_GATHER_BLOCK) k_gather_push_yee_tiled(GridGeom g, TileGeom tg, Batch<const T*> F,
                                                                            SpeciesView<T> sp,
                                                                            const int* __restrict__ perm,
                                                                            const int* __restrict__ starts, T qdt2m,
                                                                            T dtx, T dty, T dtz) {
  using S = Shape<T, ORDER>;
  using X = Box<S::NW>;
  constexpr int NW = S::NW;
  constexpr int FS = FieldSlots<T>::FS;
  extern __shared__ __align__(16) unsigned char smem[];
  T* box = reinterpret_cast<T*>(smem);
  const int tile = xcd_major(blockIdx.x, gridDim.x);
  const int beg = starts[tile], end = starts[tile + 1];
  if (beg == end || tile == tg.ntiles) return;
  int tx, ty, tz;
  tile_coords(tile, tg, tx, ty, tz);
  const int t0x = tx * kTile, t0y = ty * kTile, t0z = tz * kTile;
  load_field_box<T, ORDER>(box, F, g, t0x, t0y, t0z);
  __syncthreads();
  for (int q = beg + threadIdx.x; q < end; q += blockDim.x) {
    const int p = perm[q];
    int i, j, k;
    (void)decode_cell(sp.cell[p], g, nullptr, i, j, k);
    T ox = sp.off[0][p], oy = sp.off[1][p], oz = sp.off[2][p];
    T f[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      int a = i, b = j, d = k;
      T x = ox, y = oy, z = oz;
      half_back(a, x, kYee[c][0], g.nx);
      half_back(b, y, kYee[c][1], g.ny);
      half_back(d, z, kYee[c][2], g.nz);
      const int lx = box_index(a, t0x, g.nx), ly = box_index(b, t0y, g.ny), lz = box_index(d, t0z, g.nz);
      if (lx >= 0 && ly >= 0 && lz >= 0) {
        T wx[NW], wy[NW], wz[NW];
        S::weights(x, wx);
        S::weights(y, wy);
        S::weights(z, wz);
        const T* b0 = box + (size_t)X::at(lx, ly, lz) * FS + c;
        T acc = 0;
#pragma unroll
        for (int u = 0; u < NW; ++u)
#pragma unroll
          for (int v = 0; v < NW; ++v) {
            const T wuv = wx[u] * wy[v];
#pragma unroll
            for (int w = 0; w < NW; ++w) acc += wuv * wz[w] * b0[(u * X::B2 + v * X::B + w) * FS];
          }
        f[c] = acc;
      } else {
        f[c] = stencil_value<T, ORDER>(g, a, b, d, x, y, z, F.p[c]);
      }
    }
    T ux = sp.u[0][p], uy = sp.u[1][p], uz = sp.u[2][p];
    BorisState<T> bs;
    boris(f, qdt2m, ux, uy, uz, bs);
    const T ig = inv_sqrt((T)1 + ux * ux + uy * uy + uz * uz);
    i = wrapi(i + advance_offset(ox, dtx * ux * ig - (T)g.sgx), g.nx);
    j = wrapi(j + advance_offset(oy, dty * uy * ig - (T)g.sgy), g.ny);
    k = wrapi(k + advance_offset(oz, dtz * uz * ig - (T)g.sgz), g.nz);
    sp.u[0][p] = ux;
    sp.u[1][p] = uy;
    sp.u[2][p] = uz;
    sp.off[0][p] = ox;
    sp.off[1][p] = oy;
    sp.off[2][p] = oz;
    sp.cell[p] = (i * g.ny + j) * g.nz + k;
  }
}

// Tiled deposition of the staggered cycle: one block per tile of the grouping of the particles'
// current cells (x^{n+1}), rho at x^{n+1} and each J^d at x^{n+1/2} - delta_d (all within one
// cell of the tile) accumulated in a fixed-point LDS box per component, as in k_scatter_tiled,
// then staged for the deposition's box reduction.
template <typename T, int ORDER>
__global__ void __launch_bounds__(256) k_deposit_yee_tiled(GridGeom g, TileGeom tg, SpeciesView<T> sp,
                                                           const int* __restrict__ perm,
                                                           const int* __restrict__ starts, Batch<T*> out,
                                                           T* __restrict__ stage, T qdv, T hdtx, T hdty, T hdtz,
                                                           int with_j) {
  using S = Shape<T, ORDER>;
  using X = Box<S::NW>;
  constexpr int NV = 4;
  constexpr int kWaves = 256 / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  auto* box = reinterpret_cast<typename Fixed<T>::acc_t*>(smem);
  __shared__ T red[NV * kWaves], redm[NV * kWaves];
  __shared__ int shs[NV];
  const int tile = xcd_major(blockIdx.x, gridDim.x);
  const int beg = starts[tile], end = starts[tile + 1];
  if (beg == end) return;
  int ti, tj, tk;
  tile_coords(tile, tg, ti, tj, tk);
  const int t0x = ti * kTile, t0y = tj * kTile, t0z = tk * kTile;
  // the values: q w / dV and q w v_d / dV
  auto values = [&](int p, T* val, T* v) {
    const T qw = qdv * (sp.w ? sp.w[p] : (T)sp.w_const);
    const T ux = sp.u[0][p], uy = sp.u[1][p], uz = sp.u[2][p];
    const T ig = inv_sqrt((T)1 + ux * ux + uy * uy + uz * uz);
    v[0] = ux * ig;
    v[1] = uy * ig;
    v[2] = uz * ig;
    val[0] = qw;
#pragma unroll
    for (int d = 0; d < 3; ++d) val[1 + d] = with_j ? qw * v[d] : (T)0;
  };
  T sw[NV], mw[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) sw[c] = mw[c] = 0;
  for (int q = beg + threadIdx.x; q < end; q += blockDim.x) {
    T val[NV], v[3];
    values(perm[q], val, v);
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      sw[c] += fabs(val[c]);
      mw[c] = fmax(mw[c], fabs(val[c]));
    }
  }
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    for (int o = 32; o > 0; o >>= 1) {
      sw[c] += __shfl_xor(sw[c], o, 64);
      mw[c] = fmax(mw[c], __shfl_xor(mw[c], o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
      red[c * kWaves + (threadIdx.x >> 6)] = sw[c];
      redm[c * kWaves + (threadIdx.x >> 6)] = mw[c];
    }
  }
  for (int e = threadIdx.x; e < NV * X::B3; e += blockDim.x) box[e] = 0;
  __syncthreads();
  if (threadIdx.x < NV) {
    const int c = threadIdx.x;
    T m = 0, x = 0;
    for (int w = 0; w < kWaves; ++w) {
      m += red[c * kWaves + w];
      x = fmax(x, redm[c * kWaves + w]);
    }
    if (g.det) m = x * (T)(end - beg);  // order-independent bound (see GridGeom::det)
    int e_sum = 0, e_max = 0;
    (void)frexp(m * (T)(MaxWeight<ORDER>::value * 1.001), &e_sum);
    (void)frexp(x * (T)1.001, &e_max);
    shs[c] = Fixed<T>::shift(e_sum, e_max, 32 - __clz(end - beg));
  }
  __syncthreads();
  int sh[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) sh[c] = shs[c];
  auto put = [&](int comp, int i, int j, int k, T ox, T oy, T oz, T val) {
    const int lx = box_index(i, t0x, g.nx), ly = box_index(j, t0y, g.ny), lz = box_index(k, t0z, g.nz);
    if (lx >= 0 && ly >= 0 && lz >= 0) {
      const T sv[1] = {(T)ldexp(val, sh[comp])};
      scatter_lds<T, ORDER, 1>(box + comp * X::B3, X::at(lx, ly, lz), ox, oy, oz, sv);
    } else {
      T* dst[1] = {out.p[comp]};
      const T v1[1] = {val};
      scatter<T, ORDER>(g, i, j, k, ox, oy, oz, dst, v1, 1);
    }
  };
  for (int q = beg + threadIdx.x; q < end; q += blockDim.x) {
    const int p = perm[q];
    int i, j, k;
    if (!decode_cell(sp.cell[p], g, nullptr, i, j, k)) continue;
    const T ox = sp.off[0][p], oy = sp.off[1][p], oz = sp.off[2][p];
    T val[NV], v[3];
    values(p, val, v);
    put(0, i, j, k, ox, oy, oz, val[0]);
    if (!with_j) continue;
    T hx = ox, hy = oy, hz = oz;
    const int ih = wrapi(i + advance_offset(hx, -hdtx * v[0] + (T)0.5 * (T)g.sgx), g.nx);
    const int jh = wrapi(j + advance_offset(hy, -hdty * v[1] + (T)0.5 * (T)g.sgy), g.ny);
    const int kh = wrapi(k + advance_offset(hz, -hdtz * v[2] + (T)0.5 * (T)g.sgz), g.nz);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int a = ih, b = jh, c = kh;
      T x = hx, y = hy, z = hz;
      half_back(a, x, kYee[d][0], g.nx);
      half_back(b, y, kYee[d][1], g.ny);
      half_back(c, z, kYee[d][2], g.nz);
      put(1 + d, a, b, c, x, y, z, val[1 + d]);
    }
  }
  __syncthreads();
  T* dstage = stage + (size_t)tile * NV * X::B3;
  for (int e = threadIdx.x; e < NV * X::B3; e += blockDim.x) dstage[e] = ldexp((T)box[e], -shs[e / X::B3]);
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

int deposit_box(int shape_order) { return kTile + (shape_order == 1 ? 2 : 4) + 1; }
int deposit_stage_slot(int shape_order) { return shape_order == 1 ? StageRows<1>::SLOT : StageRows<3>::SLOT; }
template <typename T>
void gather_push_tiled(const GridGeom& g, const TileGeom& t, const T* const E[3], const T* const B[3],
                       const SpeciesView<T>& in, const SpeciesView<T>& out, const int* perm, const int* starts,
                       bool write_sorted, int* home_cursor, const int* nbr_bases, hipStream_t s) {
  if (in.n <= 0) return;
  Batch<const T*> F{};
  for (int d = 0; d < 3; ++d) {
    F.p[d] = E[d];
    F.p[3 + d] = B[d];
  }
  const T qdt2m = (T)(in.q * g.dt / (2.0 * in.m));
  const T dtx = (T)(g.dt / g.dx), dty = (T)(g.dt / g.dy), dtz = (T)(g.dt / g.dz);
  const int Bx = deposit_box(g.shape_order);
  const size_t lds = (size_t)Bx * Bx * Bx * GatherBox<T, 1>::SLOTS * sizeof(T);
  const dim3 grid(t.ntiles + 1);
  const dim3 block(g.shape_order == 1 ? kGatherBlock<T, 1> : kGatherBlock<T, 3>);
  if (home_cursor) {
    if (g.shape_order == 1) {
      allow_lds((const void*)k_gather_push_home<T, 1>, lds);
      hipLaunchKernelGGL((k_gather_push_home<T, 1>), grid, block, lds, s, g, t, F, in, out, starts, home_cursor,
                         nbr_bases, qdt2m, dtx, dty, dtz);
    } else {
      allow_lds((const void*)k_gather_push_home<T, 3>, lds);
      hipLaunchKernelGGL((k_gather_push_home<T, 3>), grid, block, lds, s, g, t, F, in, out, starts, home_cursor,
                         nbr_bases, qdt2m, dtx, dty, dtz);
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

// Resident workgroups of ``kernel`` the device holds at once (occupancy x compute units).
int resident_blocks(const void* kernel, int block, size_t lds) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, block, lds) != hipSuccess || per <= 0 || cus <= 0) {
    (void)hipGetLastError();
    return 1024;
  }
  return per * cus;
}

template <typename T, int ORDER, bool WJ>
void launch_deposit(const GridGeom& g, const TileGeom& t, const SpeciesView<T>& sp, const int* perm, const int* starts,
                    T* stage, int* bad, int* next_counts, int* nbr_counts, int* work, int* spill_flag,
                    int* box_faces, const Batch<T*>& out, hipStream_t s) {
  const T qdv = (T)(sp.q / (g.dx * g.dy * g.dz));
  const T hx = (T)(0.5 * g.dt / g.dx), hy = (T)(0.5 * g.dt / g.dy), hz = (T)(0.5 * g.dt / g.dz);
  constexpr int B = Box<Shape<T, ORDER>::NW>::B;
  const size_t lds = (size_t)(WJ ? 4 : 1) * B * B * B * sizeof(typename Fixed<T>::acc_t);
  const void* k = (const void*)k_deposit_tiled<T, ORDER, WJ>;
  allow_lds(k, lds);
  int nb = t.ntiles + 1;
  if (ORDER == 3) {  // persistent launch (see k_deposit_tiled)
    static int resident = 0;  // per instantiation; the device's occupancy does not change
    if (resident == 0) resident = resident_blocks(k, PIC_DEPOSIT_BLOCK, lds);
    nb = std::min(nb, resident);
    (void)hipMemsetAsync(work, 0, sizeof(int), s);
  }
  hipLaunchKernelGGL((k_deposit_tiled<T, ORDER, WJ>), dim3(nb), dim3(PIC_DEPOSIT_BLOCK), lds, s, g, t, sp, perm,
                     starts, out, stage, qdv, hx, hy, hz, bad, next_counts, nbr_counts, work, spill_flag, box_faces);
}

template <typename T>
void deposit_tiled(const GridGeom& g, const TileGeom& t, const SpeciesView<T>& sp, const int* perm, const int* starts,
                   bool with_j, T* stage, int* bad, int* next_counts, int* nbr_counts, int* work, T* rho,
                   T* const J[3], hipStream_t s, int* spill_flag, int* box_faces) {
  if (sp.n <= 0) return;
  // the face masks serve the whole-tile reduction only; the other one reads whole boxes
  if (!(g.nx % kTile == 0 && g.ny % kTile == 0 && g.nz % kTile == 0)) box_faces = nullptr;
  Batch<T*> out{};
  out.p[0] = rho;
  for (int d = 0; d < 3; ++d) out.p[1 + d] = J ? J[d] : nullptr;
  if (g.shape_order == 1) {
    if (with_j) launch_deposit<T, 1, true>(g, t, sp, perm, starts, stage, bad, next_counts, nbr_counts, work, spill_flag, box_faces, out, s);
    else launch_deposit<T, 1, false>(g, t, sp, perm, starts, stage, bad, next_counts, nbr_counts, work, spill_flag, box_faces, out, s);
  } else {
    if (with_j) launch_deposit<T, 3, true>(g, t, sp, perm, starts, stage, bad, next_counts, nbr_counts, work, spill_flag, box_faces, out, s);
    else launch_deposit<T, 3, false>(g, t, sp, perm, starts, stage, bad, next_counts, nbr_counts, work, spill_flag, box_faces, out, s);
  }
}

template <typename T>
void deposit_reduce(const GridGeom& g, const TileGeom& t, const int* starts, const T* stage, bool with_j, T* rho,
                    T* const J[3], hipStream_t s, const ReduceArgs<T>& ra) {
  Batch<T*> out{};
  out.p[0] = rho;
  for (int d = 0; d < 3; ++d) out.p[1 + d] = J ? J[d] : nullptr;
  const int ncomp = with_j ? 4 : 1;
  if (ra.rows && g.nx % kTile == 0 && g.ny % kTile == 0 && g.nz % kTile == 0) {
    const int groups = g.nz / 4;
    const unsigned bz = (unsigned)std::min(256, (groups + 63) / 64 * 64);
    const dim3 grid((unsigned)((groups + bz - 1) / bz), (unsigned)g.ny, (unsigned)g.nx);
    if (g.shape_order == 1) {
      if (with_j) hipLaunchKernelGGL((k_deposit_reduce_rows<T, 1, 4>), grid, dim3(bz), 0, s, g, t, starts, stage, out, ra);
      else hipLaunchKernelGGL((k_deposit_reduce_rows<T, 1, 1>), grid, dim3(bz), 0, s, g, t, starts, stage, out, ra);
    } else {
      if (with_j) hipLaunchKernelGGL((k_deposit_reduce_rows<T, 3, 4>), grid, dim3(bz), 0, s, g, t, starts, stage, out, ra);
      else hipLaunchKernelGGL((k_deposit_reduce_rows<T, 3, 1>), grid, dim3(bz), 0, s, g, t, starts, stage, out, ra);
    }
    return;
  }
  if (g.nx % kTile == 0 && g.ny % kTile == 0 && g.nz % kTile == 0) {
    const unsigned bz = (unsigned)std::min(256, (g.nz + 63) / 64 * 64);
    const dim3 grid((unsigned)((g.nz + bz - 1) / bz), (unsigned)g.ny, (unsigned)g.nx);
    if (g.shape_order == 1) {
      if (with_j) hipLaunchKernelGGL((k_deposit_reduce_whole<T, 1, 4>), grid, dim3(bz), 0, s, g, t, starts, stage, out, ra);
      else hipLaunchKernelGGL((k_deposit_reduce_whole<T, 1, 1>), grid, dim3(bz), 0, s, g, t, starts, stage, out, ra);
    } else {
      if (with_j) hipLaunchKernelGGL((k_deposit_reduce_whole<T, 3, 4>), grid, dim3(bz), 0, s, g, t, starts, stage, out, ra);
      else hipLaunchKernelGGL((k_deposit_reduce_whole<T, 3, 1>), grid, dim3(bz), 0, s, g, t, starts, stage, out, ra);
    }
    return;
  }
  const long long N = (long long)g.nx * g.ny * g.nz;
  const unsigned nr = (unsigned)std::min<long long>((N + 255) / 256, 65536);
  if (g.shape_order == 1)
    hipLaunchKernelGGL((k_deposit_reduce<T, 1>), dim3(nr), dim3(256), 0, s, g, t, starts, stage, out, ncomp, ra);
  else
    hipLaunchKernelGGL((k_deposit_reduce<T, 3>), dim3(nr), dim3(256), 0, s, g, t, starts, stage, out, ncomp, ra);
}

template <typename T>
void particle_adjoint(const GridGeom& g, const TileGeom& t, const SpeciesView<T>& sp, const Batch<T*>& lam,
                      const int* perm, const int* starts, const T* const F[6], const T* const L[4],
                      const Batch<T*>& lamF, hipStream_t s) {
  if (sp.n <= 0) return;
  Batch<const T*> f{}, l{};
  for (int m = 0; m < 6; ++m) f.p[m] = F[m];
  for (int m = 0; m < 4; ++m) l.p[m] = L[m];
  const bool mobile = std::isfinite(sp.m);
  const T qdt2m = mobile ? (T)(sp.q * g.dt / (2.0 * sp.m)) : (T)0;
  const T qdv = (T)(sp.q / (g.dx * g.dy * g.dz));
  const T dtx = (T)(g.dt / g.dx), dty = (T)(g.dt / g.dy), dtz = (T)(g.dt / g.dz);
  const int mob = mobile ? 1 : 0;
  // LDS-staged boxes (E, B and the 4 adjoint sources) when they fit a workgroup's LDS
  const int Bx = deposit_box(g.shape_order);
  const size_t lds = (size_t)Bx * Bx * Bx * (4 + GatherBox<T, 1>::SLOTS + 1) * sizeof(T);
  if (starts && lds <= 160 * 1024) {
    const dim3 grid((unsigned)t.ntiles + 1);
    if (g.shape_order == 1) {
      allow_lds((const void*)k_particle_adjoint_tiled<T, 1>, lds);
      hipLaunchKernelGGL((k_particle_adjoint_tiled<T, 1>), grid, dim3(PIC_GATHER_BLOCK), lds, s, g, t, sp, lam, perm,
                         starts, f, l, lamF, qdt2m, qdv, dtx, dty, dtz, mob);
    } else {
      allow_lds((const void*)k_particle_adjoint_tiled<T, 3>, lds);
      hipLaunchKernelGGL((k_particle_adjoint_tiled<T, 3>), grid, dim3(PIC_GATHER_BLOCK), lds, s, g, t, sp, lam, perm,
                         starts, f, l, lamF, qdt2m, qdv, dtx, dty, dtz, mob);
    }
    return;
  }
  const dim3 grid((unsigned)((sp.n + 255) / 256));
  if (g.shape_order == 1)
    hipLaunchKernelGGL((k_particle_adjoint<T, 1>), grid, dim3(256), 0, s, g, sp, lam, perm, f, l, lamF, qdt2m, qdv,
                       dtx, dty, dtz, mob);
  else
    hipLaunchKernelGGL((k_particle_adjoint<T, 3>), grid, dim3(256), 0, s, g, sp, lam, perm, f, l, lamF, qdt2m, qdv,
                       dtx, dty, dtz, mob);
}

template <typename T>
void scatter_tiled(const GridGeom& g, const TileGeom& t, const SpeciesView<T>& sp, const int* perm, const int* starts,
                   const T* const val[6], T* const out[6], T* stage, hipStream_t s) {
  if (sp.n <= 0) return;
  Batch<const T*> v{};
  Batch<T*> o{};
  for (int m = 0; m < 6; ++m) {
    v.p[m] = val[m];
    o.p[m] = out[m];
  }
  const int B = deposit_box(g.shape_order);
  const size_t lds = (size_t)6 * B * B * B * sizeof(typename Fixed<T>::acc_t);
  const dim3 grid((unsigned)t.ntiles);
  if (g.shape_order == 1) {
    allow_lds((const void*)k_scatter_tiled<T, 1>, lds);
    hipLaunchKernelGGL((k_scatter_tiled<T, 1>), grid, dim3(256), lds, s, g, t, sp, perm, starts, v, o, stage);
  } else {
    allow_lds((const void*)k_scatter_tiled<T, 3>, lds);
    hipLaunchKernelGGL((k_scatter_tiled<T, 3>), grid, dim3(256), lds, s, g, t, sp, perm, starts, v, o, stage);
  }
  // the overlapping boxes onto the grids (as the deposition's second launch)
  if (g.nx % kTile == 0 && g.ny % kTile == 0 && g.nz % kTile == 0) {
    const unsigned bz = (unsigned)std::min(256, (g.nz + 63) / 64 * 64);
    const dim3 rgrid((unsigned)((g.nz + bz - 1) / bz), (unsigned)g.ny, (unsigned)g.nx);
    if (g.shape_order == 1)
      hipLaunchKernelGGL((k_deposit_reduce_whole<T, 1, 6>), rgrid, dim3(bz), 0, s, g, t, starts, stage, o, ReduceArgs<T>());
    else
      hipLaunchKernelGGL((k_deposit_reduce_whole<T, 3, 6>), rgrid, dim3(bz), 0, s, g, t, starts, stage, o, ReduceArgs<T>());
    return;
  }
  const long long N = (long long)g.nx * g.ny * g.nz;
  const unsigned nr = (unsigned)std::min<long long>((N + 255) / 256, 65536);
  if (g.shape_order == 1)
    hipLaunchKernelGGL((k_deposit_reduce<T, 1>), dim3(nr), dim3(256), 0, s, g, t, starts, stage, o, 6, ReduceArgs<T>());
  else
    hipLaunchKernelGGL((k_deposit_reduce<T, 3>), dim3(nr), dim3(256), 0, s, g, t, starts, stage, o, 6, ReduceArgs<T>());
}

template <typename T>
void gather_push_yee(const GridGeom& g, const T* const E[3], const T* const B[3], const SpeciesView<T>& sp,
                     hipStream_t s) {
  if (sp.n <= 0 || !std::isfinite(sp.m)) return;
  Batch<const T*> F{};
  for (int d = 0; d < 3; ++d) {
    F.p[d] = E[d];
    F.p[3 + d] = B[d];
  }
  const T qdt2m = (T)(sp.q * g.dt / (2.0 * sp.m));
  const T dtx = (T)(g.dt / g.dx), dty = (T)(g.dt / g.dy), dtz = (T)(g.dt / g.dz);
  const dim3 grid((unsigned)((sp.n + 255) / 256));
  if (g.shape_order == 1)
    hipLaunchKernelGGL((k_gather_push_yee<T, 1>), grid, dim3(256), 0, s, g, F, sp, qdt2m, dtx, dty, dtz);
  else
    hipLaunchKernelGGL((k_gather_push_yee<T, 3>), grid, dim3(256), 0, s, g, F, sp, qdt2m, dtx, dty, dtz);
}

template <typename T>
void gather_push_yee_tiled(const GridGeom& g, const TileGeom& t, const T* const E[3], const T* const B[3],
                           const SpeciesView<T>& sp, const int* perm, const int* starts, hipStream_t s) {
  if (sp.n <= 0 || !std::isfinite(sp.m)) return;
  Batch<const T*> F{};
  for (int d = 0; d < 3; ++d) {
    F.p[d] = E[d];
    F.p[3 + d] = B[d];
  }
  const T qdt2m = (T)(sp.q * g.dt / (2.0 * sp.m));
  const T dtx = (T)(g.dt / g.dx), dty = (T)(g.dt / g.dy), dtz = (T)(g.dt / g.dz);
  const int Bx = deposit_box(g.shape_order);
  const size_t lds = (size_t)Bx * Bx * Bx * FieldSlots<T>::FS * sizeof(T);
  const dim3 grid(t.ntiles + 1), block(PIC_GATHER_BLOCK);
  if (g.shape_order == 1) {
    allow_lds((const void*)k_gather_push_yee_tiled<T, 1>, lds);
    hipLaunchKernelGGL((k_gather_push_yee_tiled<T, 1>), grid, block, lds, s, g, t, F, sp, perm, starts, qdt2m, dtx,
                       dty, dtz);
  } else {
    allow_lds((const void*)k_gather_push_yee_tiled<T, 3>, lds);
    hipLaunchKernelGGL((k_gather_push_yee_tiled<T, 3>), grid, block, lds, s, g, t, F, sp, perm, starts, qdt2m, dtx,
                       dty, dtz);
  }
}

template <typename T>
void deposit_yee_tiled(const GridGeom& g, const TileGeom& t, const SpeciesView<T>& sp, const int* perm,
                       const int* starts, bool with_j, T* stage, T* rho, T* const J[3], hipStream_t s) {
  if (sp.n <= 0) return;
  Batch<T*> out{};
  out.p[0] = rho;
  for (int d = 0; d < 3; ++d) out.p[1 + d] = J[d];
  const T qdv = (T)(sp.q / (g.dx * g.dy * g.dz));
  const T hx = (T)(0.5 * g.dt / g.dx), hy = (T)(0.5 * g.dt / g.dy), hz = (T)(0.5 * g.dt / g.dz);
  const int B = deposit_box(g.shape_order);
  const size_t lds = (size_t)4 * B * B * B * sizeof(typename Fixed<T>::acc_t);
  const dim3 grid((unsigned)t.ntiles);
  if (g.shape_order == 1) {
    allow_lds((const void*)k_deposit_yee_tiled<T, 1>, lds);
    hipLaunchKernelGGL((k_deposit_yee_tiled<T, 1>), grid, dim3(256), lds, s, g, t, sp, perm, starts, out, stage, qdv,
                       hx, hy, hz, with_j ? 1 : 0);
  } else {
    allow_lds((const void*)k_deposit_yee_tiled<T, 3>, lds);
    hipLaunchKernelGGL((k_deposit_yee_tiled<T, 3>), grid, dim3(256), lds, s, g, t, sp, perm, starts, out, stage, qdv,
                       hx, hy, hz, with_j ? 1 : 0);
  }
  deposit_reduce<T>(g, t, starts, stage, true, rho, J, s, ReduceArgs<T>());
}

template <typename T>
void deposit_yee(const GridGeom& g, const SpeciesView<T>& sp, bool with_j, T* rho, T* const J[3], hipStream_t s) {
  if (sp.n <= 0) return;
  Batch<T*> out{};
  out.p[0] = rho;
  for (int d = 0; d < 3; ++d) out.p[1 + d] = J ? J[d] : nullptr;
  const T qdv = (T)(sp.q / (g.dx * g.dy * g.dz));
  const T hx = (T)(0.5 * g.dt / g.dx), hy = (T)(0.5 * g.dt / g.dy), hz = (T)(0.5 * g.dt / g.dz);
  const dim3 grid((unsigned)((sp.n + 255) / 256));
  if (g.shape_order == 1)
    hipLaunchKernelGGL((k_deposit_yee<T, 1>), grid, dim3(256), 0, s, g, sp, out, qdv, hx, hy, hz, with_j ? 1 : 0);
  else
    hipLaunchKernelGGL((k_deposit_yee<T, 3>), grid, dim3(256), 0, s, g, sp, out, qdv, hx, hy, hz, with_j ? 1 : 0);
}

#define PIC_INST(T)                                                                                              \
  template void permute_species<T>(const SpeciesView<T>&, const SpeciesView<T>&, const int*, hipStream_t);       \
  template void deposit_tiled<T>(const GridGeom&, const TileGeom&, const SpeciesView<T>&, const int*, const int*, \
                                 bool, T*, int*, int*, int*, int*, T*, T* const*, hipStream_t, int*, int*);      \
  template void deposit_reduce<T>(const GridGeom&, const TileGeom&, const int*, const T*, bool, T*, T* const*,   \
                                  hipStream_t, const ReduceArgs<T>&);                                            \
  template void gather_push_tiled<T>(const GridGeom&, const TileGeom&, const T* const*, const T* const*,         \
                                     const SpeciesView<T>&, const SpeciesView<T>&, const int*, const int*, bool,  \
                                     int*, const int*, hipStream_t);                                              \
  template void particle_adjoint<T>(const GridGeom&, const TileGeom&, const SpeciesView<T>&, const Batch<T*>&,    \
                                    const int*, const int*, const T* const*, const T* const*, const Batch<T*>&,   \
                                    hipStream_t);                                                                 \
  template void scatter_tiled<T>(const GridGeom&, const TileGeom&, const SpeciesView<T>&, const int*, const int*, \
                                 const T* const*, T* const*, T*, hipStream_t);                                    \
  template void gather_push_yee<T>(const GridGeom&, const T* const*, const T* const*, const SpeciesView<T>&,      \
                                   hipStream_t);                                                                  \
  template void deposit_yee<T>(const GridGeom&, const SpeciesView<T>&, bool, T*, T* const*, hipStream_t);        \
  template void deposit_yee_tiled<T>(const GridGeom&, const TileGeom&, const SpeciesView<T>&, const int*,         \
                                     const int*, bool, T*, T*, T* const*, hipStream_t);                           \
  template void gather_push_yee_tiled<T>(const GridGeom&, const TileGeom&, const T* const*, const T* const*,      \
                                         const SpeciesView<T>&, const int*, const int*, hipStream_t);
PIC_INST(float)
PIC_INST(double)
#undef PIC_INST

}  // namespace pic
