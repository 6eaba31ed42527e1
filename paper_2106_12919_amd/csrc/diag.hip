// Grid reductions accumulated in FP64 (field energy of Sec. 2 item iii, total
// charge, the Gauss's-law and continuity residuals of the spectra) and element-wise helpers.
#include "kernels.h"

namespace pic {

namespace {

__device__ inline double block_sum(double v) {
  __shared__ double red[32];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) r += red[w];
  return r;
}

template <typename T>
__global__ void __launch_bounds__(256) k_sum_squares(Batch<const T*> a, int count, long long n, double* acc) {
  double v = 0;
  for (int c = 0; c < count; ++c)
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
      const double x = (double)a.p[c][i];
      v += x * x;
    }
  v = block_sum(v);
  if (threadIdx.x == 0) atomicAdd(acc, v);
}

template <typename T>
__global__ void __launch_bounds__(256) k_sum_plain(const T* a, long long n, double* acc) {
  double v = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    v += (double)a[i];
  v = block_sum(v);
  if (threadIdx.x == 0) atomicAdd(acc, v);
}

// Residual of a divergence law in the paper's Fourier convention (App. A; derivative <-> i k):
// r = i [k]_s . V_hat + ca A_hat + cb B_hat.  With index-space spectra v_d of the Yee components
// and D-_d = i [k_d]_s exp(-i k_d dx_d / 2), i [k_d]_s V_hat_d = D-_d v_d.  Gauss's law (the
// update's derivation assumes it, eps0 = 1): V = E, A = rho, ca = -1, no B.  Continuity:
// V = J, A = rho^{n+1}, ca = 1/dt, B = rho^n, cb = -1/dt.  acc[0] += |r|^2 and
// acc[1] += |ca A + cb B|^2 over the half spectrum, each mode weighted by the number of
// full-spectrum modes it stands for (1 at kz = 0 and at the Nyquist index of an even nz, 2 otherwise).
template <typename T>
__global__ void __launch_bounds__(256) k_div_residual(Batch<const cplx<T>*> S, const cplx<T>* __restrict__ dmx,
                                                      const cplx<T>* __restrict__ dmy, const cplx<T>* __restrict__ dmz,
                                                      double ca, double cb, int nx, int ny, int nzh, int pz, int nz,
                                                      double* acc) {
  double num = 0, den = 0;
  const long long total = (long long)nx * ny * nzh;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int kz = (int)(idx % nzh);
    const long long r = idx / nzh;
    const int j = (int)(r % ny), i = (int)(r / ny);
    const size_t a = (size_t)r * pz + kz;
    const cplx<T> e0 = S.p[0][a], e1 = S.p[1][a], e2 = S.p[2][a], ah = S.p[3][a];
    double sx = ca * (double)ah.x, sy = ca * (double)ah.y;
    if (S.p[4]) {
      const cplx<T> bh = S.p[4][a];
      sx += cb * (double)bh.x;
      sy += cb * (double)bh.y;
    }
    const cplx<T> px = dmx[i], py = dmy[j], pzz = dmz[kz];
    const double rx = (double)px.x * e0.x - (double)px.y * e0.y + (double)py.x * e1.x - (double)py.y * e1.y +
                      (double)pzz.x * e2.x - (double)pzz.y * e2.y + sx;
    const double ry = (double)px.x * e0.y + (double)px.y * e0.x + (double)py.x * e1.y + (double)py.y * e1.x +
                      (double)pzz.x * e2.y + (double)pzz.y * e2.x + sy;
    const double w = (kz == 0 || 2 * kz == nz) ? 1.0 : 2.0;
    num += w * (rx * rx + ry * ry);
    den += w * (sx * sx + sy * sy);
  }
  num = block_sum(num);
  __syncthreads();
  den = block_sum(den);
  if (threadIdx.x == 0) {
    atomicAdd(acc, num);
    atomicAdd(acc + 1, den);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_add_into(T* dst, const T* src, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] += src[i];
}

template <typename T>
__global__ void __launch_bounds__(256) k_zero_arrays(Batch<T*> arrs, long long n) {
  T* __restrict__ d = arrs.p[blockIdx.y];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    d[i] = (T)0;
}

}  // namespace

template <typename T>
void sum_squares(const Batch<const T*>& arrs, int count, int64_t n, double* acc, hipStream_t s) {
  hipLaunchKernelGGL((k_sum_squares<T>), dim3(1024), dim3(256), 0, s, arrs, count, (long long)n, acc);
}
template <typename T>
void sum_plain(const T* arr, int64_t n, double* acc, hipStream_t s) {
  hipLaunchKernelGGL((k_sum_plain<T>), dim3(1024), dim3(256), 0, s, arr, (long long)n, acc);
}
template <typename T>
void div_residual(const PsatdTables<T>& t, const cplx<T>* const V[3], const cplx<T>* A, double ca, const cplx<T>* B,
                  double cb, int nx, int ny, int nzh, int pz, int nz, double* acc, hipStream_t s) {
  Batch<const cplx<T>*> S{};
  for (int d = 0; d < 3; ++d) S.p[d] = V[d];
  S.p[3] = A;
  S.p[4] = B;
  hipLaunchKernelGGL((k_div_residual<T>), dim3(1024), dim3(256), 0, s, S, t.Dm[0], t.Dm[1], t.Dm[2], ca, cb, nx, ny,
                     nzh, pz, nz, acc);
}
template <typename T>
void zero_arrays(const Batch<T*>& arrs, int count, int64_t n, hipStream_t s) {
  if (count <= 0 || n <= 0) return;
  hipLaunchKernelGGL((k_zero_arrays<T>), dim3(512, count), dim3(256), 0, s, arrs, (long long)n);
}
template <typename T>
void add_into(T* dst, const T* src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_add_into<T>), dim3(2048), dim3(256), 0, s, dst, src, (long long)n);
}

template void sum_squares<float>(const Batch<const float*>&, int, int64_t, double*, hipStream_t);
template void sum_squares<double>(const Batch<const double*>&, int, int64_t, double*, hipStream_t);
template void sum_plain<float>(const float*, int64_t, double*, hipStream_t);
template void sum_plain<double>(const double*, int64_t, double*, hipStream_t);
template void div_residual<float>(const PsatdTables<float>&, const cplx<float>* const*, const cplx<float>*, double,
                                 const cplx<float>*, double, int, int, int, int, int, double*, hipStream_t);
template void div_residual<double>(const PsatdTables<double>&, const cplx<double>* const*, const cplx<double>*, double,
                                  const cplx<double>*, double, int, int, int, int, int, double*, hipStream_t);
template void zero_arrays<float>(const Batch<float*>&, int, int64_t, hipStream_t);
template void zero_arrays<double>(const Batch<double*>&, int, int64_t, hipStream_t);
template void add_into<float>(float*, const float*, int64_t, hipStream_t);
template void add_into<double>(double*, const double*, int64_t, hipStream_t);

}  // namespace pic
