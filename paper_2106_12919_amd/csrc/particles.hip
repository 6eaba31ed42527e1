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
#include "kernels.h"

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

template <typename T, int ORDER>
__global__ void __launch_bounds__(256) k_gather_push(GridGeom g, Batch<const T*> F, SpeciesView<T> sp, T qdt2m,
                                                     T dtx, T dty, T dtz, int* bad) {
  using S = Shape<T, ORDER>;
  constexpr int NW = S::NW;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= sp.n) return;
  int i, j, k;
  if (!decode_cell(sp.cell[p], g, bad, i, j, k)) return;
  T ox = sp.off[0][p], oy = sp.off[1][p], oz = sp.off[2][p];
  T wx[NW], wy[NW], wz[NW];
  S::weights(ox, wx);
  S::weights(oy, wy);
  S::weights(oz, wz);
  int kk[NW];
#pragma unroll
  for (int cc = 0; cc < NW; ++cc) kk[cc] = wrapi(k + cc + S::BASE, g.nz);
  T f[6] = {0, 0, 0, 0, 0, 0};
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
        const size_t idx = row + kk[cc];
#pragma unroll
        for (int q = 0; q < 6; ++q) f[q] += w * F.p[q][idx];
      }
    }
  }
  // relativistic Boris (c = 1)
  const T ux = sp.u[0][p], uy = sp.u[1][p], uz = sp.u[2][p];
  const T umx = ux + qdt2m * f[0], umy = uy + qdt2m * f[1], umz = uz + qdt2m * f[2];
  const T gm = sqrt((T)1 + umx * umx + umy * umy + umz * umz);
  const T tf = qdt2m / gm;
  const T tx = tf * f[3], ty = tf * f[4], tz = tf * f[5];
  const T sf = (T)2 / ((T)1 + tx * tx + ty * ty + tz * tz);
  const T sx = sf * tx, sy = sf * ty, sz = sf * tz;
  const T upx = umx + (umy * tz - umz * ty);
  const T upy = umy + (umz * tx - umx * tz);
  const T upz = umz + (umx * ty - umy * tx);
  const T npx = umx + (upy * sz - upz * sy) + qdt2m * f[0];
  const T npy = umy + (upz * sx - upx * sz) + qdt2m * f[1];
  const T npz = umz + (upx * sy - upy * sx) + qdt2m * f[2];
  const T ig = (T)1 / sqrt((T)1 + npx * npx + npy * npy + npz * npz);
  i = modi(i + advance_offset(ox, dtx * npx * ig), g.nx);
  j = modi(j + advance_offset(oy, dty * npy * ig), g.ny);
  k = modi(k + advance_offset(oz, dtz * npz * ig), g.nz);
  sp.u[0][p] = npx;
  sp.u[1][p] = npy;
  sp.u[2][p] = npz;
  sp.off[0][p] = ox;
  sp.off[1][p] = oy;
  sp.off[2][p] = oz;
  sp.cell[p] = (i * g.ny + j) * g.nz + k;
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

template <typename T, int ORDER>
__global__ void __launch_bounds__(256) k_deposit(GridGeom g, SpeciesView<T> sp, Batch<T*> out, T qdv, int with_j,
                                                 T hdtx, T hdty, T hdtz, int* bad) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= sp.n) return;
  int i, j, k;
  if (!decode_cell(sp.cell[p], g, bad, i, j, k)) return;
  const T ox = sp.off[0][p], oy = sp.off[1][p], oz = sp.off[2][p];
  const T qw = qdv * (sp.w ? sp.w[p] : (T)sp.w_const);
  {
    T* dst[1] = {out.p[0]};
    T val[1] = {qw};
    scatter<T, ORDER>(g, i, j, k, ox, oy, oz, dst, val, 1);
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
    T* dst[3] = {out.p[1], out.p[2], out.p[3]};
    T val[3] = {qw * vx, qw * vy, qw * vz};
    scatter<T, ORDER>(g, ih, jh, kh, hx, hy, hz, dst, val, 3);
  }
}

}  // namespace

template <typename T>
void gather_push(const GridGeom& g, const T* const E[3], const T* const B[3], const SpeciesView<T>& sp, int* bad,
                 hipStream_t s) {
  if (sp.n <= 0) return;
  Batch<const T*> F{};
  for (int d = 0; d < 3; ++d) {
    F.p[d] = E[d];
    F.p[3 + d] = B[d];
  }
  const T qdt2m = (T)(sp.q * g.dt / (2.0 * sp.m));
  const T dtx = (T)(g.dt / g.dx), dty = (T)(g.dt / g.dy), dtz = (T)(g.dt / g.dz);
  const unsigned nb = (unsigned)((sp.n + 255) / 256);
  if (g.shape_order == 1)
    hipLaunchKernelGGL((k_gather_push<T, 1>), dim3(nb), dim3(256), 0, s, g, F, sp, qdt2m, dtx, dty, dtz, bad);
  else
    hipLaunchKernelGGL((k_gather_push<T, 3>), dim3(nb), dim3(256), 0, s, g, F, sp, qdt2m, dtx, dty, dtz, bad);
}

template <typename T>
void deposit(const GridGeom& g, const SpeciesView<T>& sp, T* rho, T* const J[3], bool with_j, int* bad,
             hipStream_t s) {
  if (sp.n <= 0) return;
  Batch<T*> out{};
  out.p[0] = rho;
  for (int d = 0; d < 3; ++d) out.p[1 + d] = J ? J[d] : nullptr;
  const T qdv = (T)(sp.q / (g.dx * g.dy * g.dz));
  const T hx = (T)(0.5 * g.dt / g.dx), hy = (T)(0.5 * g.dt / g.dy), hz = (T)(0.5 * g.dt / g.dz);
  const unsigned nb = (unsigned)((sp.n + 255) / 256);
  const int wj = with_j ? 1 : 0;
  if (g.shape_order == 1)
    hipLaunchKernelGGL((k_deposit<T, 1>), dim3(nb), dim3(256), 0, s, g, sp, out, qdv, wj, hx, hy, hz, bad);
  else
    hipLaunchKernelGGL((k_deposit<T, 3>), dim3(nb), dim3(256), 0, s, g, sp, out, qdv, wj, hx, hy, hz, bad);
}

template void gather_push<float>(const GridGeom&, const float* const*, const float* const*,
                                 const SpeciesView<float>&, int*, hipStream_t);
template void gather_push<double>(const GridGeom&, const double* const*, const double* const*,
                                  const SpeciesView<double>&, int*, hipStream_t);
template void deposit<float>(const GridGeom&, const SpeciesView<float>&, float*, float* const*, bool, int*,
                             hipStream_t);
template void deposit<double>(const GridGeom&, const SpeciesView<double>&, double*, double* const*, bool, int*,
                              hipStream_t);

}  // namespace pic
