// Grid reductions accumulated in FP64 (field energy of Sec. 2 item iii, total
// charge) and a plain element-wise add used for the static charge background.
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

template <typename T>
__global__ void __launch_bounds__(256) k_add_into(T* dst, const T* src, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] += src[i];
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
void add_into(T* dst, const T* src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_add_into<T>), dim3(2048), dim3(256), 0, s, dst, src, (long long)n);
}

template void sum_squares<float>(const Batch<const float*>&, int, int64_t, double*, hipStream_t);
template void sum_squares<double>(const Batch<const double*>&, int, int64_t, double*, hipStream_t);
template void sum_plain<float>(const float*, int64_t, double*, hipStream_t);
template void sum_plain<double>(const double*, int64_t, double*, hipStream_t);
template void add_into<float>(float*, const float*, int64_t, hipStream_t);
template void add_into<double>(double*, const double*, int64_t, hipStream_t);

}  // namespace pic
