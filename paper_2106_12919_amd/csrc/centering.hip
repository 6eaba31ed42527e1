// Finite-order centering between the nodal grid and the Yee grid (Sec. 3,
// eq. staggered_finite_sum; the staggered-to-nodal form is also App. C).
//
//   nodes -> centres:  f_{j+1/2} = sum_{n=1}^{m} alpha^s_{m,n} (f_{j+n} + f_{j+1-n}) / 2
//   centres -> nodes:  f_j       = sum_{n=1}^{m} alpha^s_{m,n} (f_{j+n-1/2} + f_{j-n+1/2}) / 2
// With a staggered array holding f_{j+1/2} at index j, both are
//   out[j] = sum_n c_n (in[j+n+shift] + in[j-n+1+shift]),  c_n = alpha^s_{m,n}/2,
// with shift = 0 (nodes -> centres) or -1 (centres -> nodes); periodic in j.
//
// Strided axes (x, y): one thread per contiguous column element marches over L
// outputs along the axis with a register window of L + 2m - 1 inputs (each input
// loaded once per window, loads coalesced across the column index).  Contiguous
// axis (z): a block stages whole z-lines plus the periodic halo in LDS.  Both are
// specialised on m, so the stencil is unrolled.
#include "kernels.h"

namespace pic {

namespace {

template <typename T>
struct Coef {
  T c[16];
};

// Strided axis: grid (column blocks, row blocks, outer) flattened and renumbered
// XCD-major, row blocks next to each other (which share halo rows) on one XCD.
template <typename T, int M, int L>
__global__ void __launch_bounds__(256) k_center_strided(const T* __restrict__ in, T* __restrict__ out, Coef<T> cf,
                                                        int Na, long long sa, int C, long long outer_stride,
                                                        int shift, int accumulate) {
  const int nb = gridDim.x * gridDim.y * gridDim.z;
  const int lb = xcd_major(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nb);
  const int bx = lb % gridDim.x, by = (lb / gridDim.x) % gridDim.y, bz = lb / (gridDim.x * gridDim.y);
  const int c = bx * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int j0 = by * L;
  const size_t base = (size_t)bz * outer_stride + c;
  constexpr int W = L + 2 * M - 1;
  T w[W];
#pragma unroll
  for (int i = 0; i < W; ++i) {
    int row = j0 - M + 1 + shift + i;
    row %= Na;
    if (row < 0) row += Na;
    w[i] = in[base + (size_t)row * sa];
  }
#pragma unroll
  for (int q = 0; q < L; ++q) {
    if (j0 + q < Na) {
      T acc = 0;
#pragma unroll
      for (int n = 1; n <= M; ++n) acc += cf.c[n - 1] * (w[q + n + M - 1] + w[q - n + M]);
      T* o = out + base + (size_t)(j0 + q) * sa;
      *o = accumulate ? *o + acc : acc;
    }
  }
}

// Two axes in one pass, for the staggered-to-nodal centering of B^x (y, then z) and B^y (x,
// then z): a block takes L rows along the strided axis (outer index fixed) for every z,
// centres them along that axis in registers as k_center_strided does, stages the L centred
// rows with their periodic z halo in LDS (row q at s[q * W + i] holds z = i + 1 - M + shift_z),
// then centres along z as k_center_z does.  The same sums in the same order as the two passes,
// without writing and re-reading the intermediate array.  Grid (row blocks, outer), XCD-major.
template <typename T, int M, int L>
__global__ void __launch_bounds__(256) k_center_strided_z(const T* __restrict__ in, T* __restrict__ out, Coef<T> cf,
                                                          int Na, long long sa, long long outer_stride, int nz,
                                                          int shift_a, int shift_z) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* s = reinterpret_cast<T*>(smem);
  constexpr int H = 2 * M - 1;  // halo elements per row
  constexpr int WIN = L + 2 * M - 1;
  const int W = nz + H;
  const int off = M - 1 - shift_z;  // index of z = 0
  const int lb = xcd_major(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int j0 = (lb % gridDim.x) * L;
  const size_t obase = (size_t)(lb / gridDim.x) * outer_stride;
  for (int z = threadIdx.x; z < nz; z += blockDim.x) {
    T w[WIN];
#pragma unroll
    for (int i = 0; i < WIN; ++i) {
      int row = (j0 - M + 1 + shift_a + i) % Na;
      if (row < 0) row += Na;
      w[i] = in[obase + (size_t)row * sa + z];
    }
#pragma unroll
    for (int q = 0; q < L; ++q) {  // rows past Na (a partial last block) are formed but never stored
      T acc = 0;
#pragma unroll
      for (int n = 1; n <= M; ++n) acc += cf.c[n - 1] * (w[q + n + M - 1] + w[q - n + M]);
      s[q * W + off + z] = acc;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < L * H; e += blockDim.x) {
    const int q = e / H, h = e - q * H;
    const int i = h < off ? h : nz + h;  // below z = 0, or beyond z = nz - 1
    int z = (i - off) % nz;
    if (z < 0) z += nz;
    s[q * W + i] = s[q * W + off + z];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < L * nz; e += blockDim.x) {
    const int q = e / nz, z = e - q * nz;
    if (j0 + q >= Na) continue;
    const T* sl = s + q * W + z;
    T acc = 0;
#pragma unroll
    for (int n = 1; n <= M; ++n) acc += cf.c[n - 1] * (sl[n + M - 1] + sl[M - n]);
    out[obase + (size_t)(j0 + q) * sa + z] = acc;
  }
}

// 16-byte vector of T (four floats or two doubles).
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int n = 4;
  __device__ static inline void put(float* d, const float4& v) {
    d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
  }
};
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int n = 2;
  __device__ static inline void put(double* d, const double2& v) {
    d[0] = v.x; d[1] = v.y;
  }
};

// Contiguous axis: a block stages lpb whole z-lines plus the periodic halo in LDS (line
// l at s[l * W + i] holds z = i + 1 - M + shift, W = nz + 2M - 1), the line bodies with
// 16-byte loads, then every thread forms outputs from LDS.
template <typename T, int M>
__global__ void __launch_bounds__(256) k_center_z(const T* __restrict__ in, T* __restrict__ out, Coef<T> cf, int nz,
                                                  int nlines, int lpb, int shift, int accumulate) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* s = reinterpret_cast<T*>(smem);
  constexpr int H = 2 * M - 1;  // halo elements per line
  constexpr int VN = Vec16<T>::n;
  const int W = nz + H;
  const int off = M - 1 - shift;  // index of z = 0
  const int line0 = blockIdx.x * lpb;
  const int nl = min(lpb, nlines - line0);
  const T* src = in + (size_t)line0 * nz;
  if (nz % VN == 0) {
    const int nv = nz / VN;
    for (int e = threadIdx.x; e < nl * nv; e += blockDim.x) {
      const int l = e / nv, v = e - l * nv;
      Vec16<T>::put(s + l * W + off + v * VN, reinterpret_cast<const typename Vec16<T>::type*>(src + (size_t)l * nz)[v]);
    }
  } else {
    for (int e = threadIdx.x; e < nl * nz; e += blockDim.x) {
      const int l = e / nz, z = e - l * nz;
      s[l * W + off + z] = src[(size_t)l * nz + z];
    }
  }
  for (int e = threadIdx.x; e < nl * H; e += blockDim.x) {
    const int l = e / H, h = e - l * H;
    const int i = h < off ? h : nz + h;  // below z = 0, or beyond z = nz - 1
    int z = (i - off) % nz;
    if (z < 0) z += nz;
    s[l * W + i] = src[(size_t)l * nz + z];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nl * nz; e += blockDim.x) {
    const int l = e / nz, z = e - l * nz;
    const T* sl = s + l * W + z;
    T acc = 0;
#pragma unroll
    for (int n = 1; n <= M; ++n) acc += cf.c[n - 1] * (sl[n + M - 1] + sl[M - n]);
    T* o = out + (size_t)(line0 + l) * nz + z;
    *o = accumulate ? *o + acc : acc;
  }
}

// Outputs per thread along the axis: FP32 the longest window of 32, 16 or 8 that still gives
// at least two workgroups per compute unit (a longer window re-reads fewer halo rows, but
// small grids need the workgroups); FP64 8.
template <typename T, int M>
void launch_strided(const T* in, T* out, const Coef<T>& cf, int Na, long long sa, int C, int O, long long os,
                    int shift, int acc, hipStream_t s) {
  const long long cols = (C + 255) / 256;
  auto blocks = [&](int L) { return cols * ((Na + L - 1) / L) * O; };
  constexpr long long kMinBlocks = 512;
  if (sizeof(T) == 4 && blocks(32) >= kMinBlocks) {
    dim3 grid((unsigned)cols, (Na + 31) / 32, O);
    hipLaunchKernelGGL((k_center_strided<T, M, 32>), grid, dim3(256), 0, s, in, out, cf, Na, sa, C, os, shift, acc);
  } else if (sizeof(T) == 4 && blocks(16) >= kMinBlocks) {
    dim3 grid((unsigned)cols, (Na + 15) / 16, O);
    hipLaunchKernelGGL((k_center_strided<T, M, 16>), grid, dim3(256), 0, s, in, out, cf, Na, sa, C, os, shift, acc);
  } else {
    dim3 grid((unsigned)cols, (Na + 7) / 8, O);
    hipLaunchKernelGGL((k_center_strided<T, M, 8>), grid, dim3(256), 0, s, in, out, cf, Na, sa, C, os, shift, acc);
  }
}

template <typename T>
void dispatch_strided(int m, const T* in, T* out, const Coef<T>& cf, int Na, long long sa, int C, int O,
                      long long os, int shift, int acc, hipStream_t s) {
  switch (m) {
#define PIC_CASE(MM) \
  case MM: launch_strided<T, MM>(in, out, cf, Na, sa, C, O, os, shift, acc, s); break;
    PIC_CASE(1) PIC_CASE(2) PIC_CASE(3) PIC_CASE(4) PIC_CASE(5) PIC_CASE(6) PIC_CASE(7) PIC_CASE(8)
    PIC_CASE(9) PIC_CASE(10) PIC_CASE(11) PIC_CASE(12) PIC_CASE(13) PIC_CASE(14) PIC_CASE(15) PIC_CASE(16)
#undef PIC_CASE
    default: break;
  }
}

template <typename T, int M, int L>
void launch_strided_z(const T* in, T* out, const Coef<T>& cf, int Na, long long sa, int O, long long os, int nz,
                      int shift, hipStream_t s) {
  const size_t lds = (size_t)L * (nz + 2 * M - 1) * sizeof(T);
  hipLaunchKernelGGL((k_center_strided_z<T, M, L>), dim3((Na + L - 1) / L, O), dim3(256), lds, s, in, out, cf, Na,
                     sa, os, nz, shift, shift);
}

// Rows per block of the fused pass: the longest of 32, 16, 8 (FP64: 8) whose LDS rows fit the
// default 64 KiB and that still gives two workgroups per compute unit; 0 if none fits.
template <typename T>
int strided_z_rows(int m, int Na, int O, int nz) {
  const int cand[3] = {32, 16, 8};
  int best = 0;
  for (int L : cand) {
    if (sizeof(T) == 8 && L != 8) continue;
    if ((size_t)L * (nz + 2 * m - 1) * sizeof(T) > 64 * 1024) continue;
    if (best == 0) best = L;  // the longest that fits
    if ((long long)((Na + L - 1) / L) * O >= 512) return L;
  }
  return best;
}

template <typename T, int M>
bool dispatch_strided_z_m(const T* in, T* out, const Coef<T>& cf, int Na, long long sa, int O, long long os, int nz,
                          int shift, hipStream_t s) {
  switch (strided_z_rows<T>(M, Na, O, nz)) {
    case 32: launch_strided_z<T, M, 32>(in, out, cf, Na, sa, O, os, nz, shift, s); return true;
    case 16: launch_strided_z<T, M, 16>(in, out, cf, Na, sa, O, os, nz, shift, s); return true;
    case 8: launch_strided_z<T, M, 8>(in, out, cf, Na, sa, O, os, nz, shift, s); return true;
    default: return false;
  }
}

}  // namespace

template <typename T>
bool center_axis_then_z(const T* in, T* out, int nx, int ny, int nz, int axis, int shift, int m, const double* c,
                        hipStream_t s) {
  Coef<T> cf{};
  for (int n = 0; n < m && n < 16; ++n) cf.c[n] = (T)c[n];
  const int Na = axis == 0 ? nx : ny, O = axis == 0 ? ny : nx;
  const long long sa = axis == 0 ? (long long)ny * nz : nz, os = axis == 0 ? nz : (long long)ny * nz;
  switch (m) {
#define PIC_CASE(MM) \
  case MM: return dispatch_strided_z_m<T, MM>(in, out, cf, Na, sa, O, os, nz, shift, s);
    PIC_CASE(1) PIC_CASE(2) PIC_CASE(3) PIC_CASE(4) PIC_CASE(5) PIC_CASE(6) PIC_CASE(7) PIC_CASE(8)
    PIC_CASE(9) PIC_CASE(10) PIC_CASE(11) PIC_CASE(12) PIC_CASE(13) PIC_CASE(14) PIC_CASE(15) PIC_CASE(16)
#undef PIC_CASE
    default: return false;
  }
}

template <typename T>
void center_axis(const T* in, T* out, int nx, int ny, int nz, int axis, int shift, int m, const double* c,
                 hipStream_t s, bool accumulate) {
  const int acc = accumulate ? 1 : 0;
  Coef<T> cf{};
  for (int n = 0; n < m && n < 16; ++n) cf.c[n] = (T)c[n];
  if (axis == 0) {
    dispatch_strided<T>(m, in, out, cf, nx, (long long)ny * nz, ny * nz, 1, 0, shift, acc, s);
  } else if (axis == 1) {
    dispatch_strided<T>(m, in, out, cf, ny, nz, nz, nx, (long long)ny * nz, shift, acc, s);
  } else {
    const int nlines = nx * ny;
    const int lpb = nz >= 1024 ? 1 : 1024 / nz;
    const size_t lds = (size_t)lpb * (nz + 2 * m - 1) * sizeof(T);
    const dim3 grid((nlines + lpb - 1) / lpb);
    switch (m) {
#define PIC_CASE(MM)                                                                                              \
  case MM:                                                                                                        \
    hipLaunchKernelGGL((k_center_z<T, MM>), grid, dim3(256), lds, s, in, out, cf, nz, nlines, lpb, shift, acc); \
    break;
      PIC_CASE(1) PIC_CASE(2) PIC_CASE(3) PIC_CASE(4) PIC_CASE(5) PIC_CASE(6) PIC_CASE(7) PIC_CASE(8)
      PIC_CASE(9) PIC_CASE(10) PIC_CASE(11) PIC_CASE(12) PIC_CASE(13) PIC_CASE(14) PIC_CASE(15) PIC_CASE(16)
#undef PIC_CASE
      default: break;
    }
  }
}

template void center_axis<float>(const float*, float*, int, int, int, int, int, int, const double*, hipStream_t,
                                  bool);
template void center_axis<double>(const double*, double*, int, int, int, int, int, int, const double*, hipStream_t,
                                   bool);

template bool center_axis_then_z<float>(const float*, float*, int, int, int, int, int, int, const double*,
                                         hipStream_t);
template bool center_axis_then_z<double>(const double*, double*, int, int, int, int, int, int, const double*,
                                          hipStream_t);

}  // namespace pic
