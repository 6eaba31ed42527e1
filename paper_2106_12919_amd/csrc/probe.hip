// Measurement support: the throughput of integer LDS atomics on this device, the bound of the
// fixed-point deposition (bench.py sets the deposition's time against it).  Each workgroup adds
// into a private LDS array with the address patterns the deposition's dealt order produces: for
// 32-bit adds the 32 lanes of each half wave on distinct words modulo 32, for 64-bit adds the 16
// lanes of each quarter wave on distinct words modulo 16.  Every address is a lane constant plus
// an immediate, as in the deposition.
#include "kernels.h"

#include <string>

#include "../../include/pic.h"

namespace pic {
namespace {

constexpr int kProbeWords = 4096;  // 16 KiB (u32) / 32 KiB (u64) per workgroup
constexpr int kProbeUnroll = 16;

template <typename A>
__global__ void __launch_bounds__(256) k_probe_lds_atomics(int iters, A* __restrict__ sink) {
  __shared__ A box[kProbeWords];
  for (int e = threadIdx.x; e < kProbeWords; e += blockDim.x) box[e] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // distinct residues inside each group of lanes the LDS serves together; waves on separate rows
  const int base = sizeof(A) == 4 ? (lane & 31) + 32 * (lane >> 5) : (lane & 15) + 16 * (lane >> 4);
  A* row = box + (wave * 512 + base);
  for (int it = 0; it < iters; it += kProbeUnroll) {
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) atomicAdd(row + 64 * (u & 7), (A)1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    A s = 0;
    for (int e = 0; e < 64; ++e) s += box[e];
    sink[blockIdx.x] = s;  // keeps the adds observable
  }
}

template <typename A>
hipError_t probe(int iters, double* rate) {
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int blocks = 8 * cus;
  A* sink = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if ((e = hipMalloc(&sink, blocks * sizeof(A))) != hipSuccess) return e;
  if ((e = hipEventCreate(&t0)) == hipSuccess && (e = hipEventCreate(&t1)) == hipSuccess) {
    hipLaunchKernelGGL(k_probe_lds_atomics<A>, dim3(blocks), dim3(256), 0, nullptr, kProbeUnroll, sink);  // warm-up
    (void)hipEventRecord(t0, nullptr);
    hipLaunchKernelGGL(k_probe_lds_atomics<A>, dim3(blocks), dim3(256), 0, nullptr, iters, sink);
    (void)hipEventRecord(t1, nullptr);
    e = hipEventSynchronize(t1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) *rate = (double)blocks * 256.0 * (double)iters / (ms * 1e-3) / (double)cus;
  }
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  (void)hipFree(sink);
  return e;
}

}  // namespace
}  // namespace pic

extern "C" pic_status pic_probe_lds_atomics(int width_bits, int iters, double* lane_ops_per_s_per_cu) {
  if (!lane_ops_per_s_per_cu || (width_bits != 32 && width_bits != 64) || iters < 16 || iters % 16 ||
      iters > (1 << 20))
    return PIC_EINVAL;
  const hipError_t e = width_bits == 32 ? pic::probe<unsigned int>(iters, lane_ops_per_s_per_cu)
                                        : pic::probe<unsigned long long>(iters, lane_ops_per_s_per_cu);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return PIC_EHIP;
  }
  return PIC_OK;
}
