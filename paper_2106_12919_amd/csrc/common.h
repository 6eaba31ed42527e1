// Internal declarations shared by the HIP translation units of libpic.
// Nothing here is part of the public ABI (include/pic.h).
#pragma once
#include <complex>

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>

namespace pic {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T x, y;
};

template <typename T>
__host__ __device__ inline cplx<T> cmake(T x, T y) { cplx<T> c; c.x = x; c.y = y; return c; }
template <typename T>
__host__ __device__ inline cplx<T> cadd(cplx<T> a, cplx<T> b) { return cmake(a.x + b.x, a.y + b.y); }
template <typename T>
__host__ __device__ inline cplx<T> csub(cplx<T> a, cplx<T> b) { return cmake(a.x - b.x, a.y - b.y); }
template <typename T>
__host__ __device__ inline cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return cmake(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__host__ __device__ inline cplx<T> cscale(cplx<T> a, T s) { return cmake(a.x * s, a.y * s); }
template <typename T>
__host__ __device__ inline cplx<T> cconj(cplx<T> a) { return cmake(a.x, -a.y); }
// multiply by -i (sign < 0) or +i (sign > 0)
template <typename T, int SIGN>
__host__ __device__ inline cplx<T> cmul_i(cplx<T> a) {
  return SIGN > 0 ? cmake(-a.y, a.x) : cmake(a.y, -a.x);
}

constexpr int kMaxStages = 12;
constexpr int kMaxBatch = 12;

// One axis of the mixed-radix Stockham FFT.  Stage s has radix radix[s]; ns[s] is
// the product of the radices of the stages before it; the twiddles of stage s,
// exp(-2 pi i k r / (ns R)) for k < ns and 1 <= r < R, start at twoff[s] of the
// table (entry k*(R-1) + r-1).
struct FftPlan {
  int n;
  int nstages;
  int radix[kMaxStages];
  int ns[kMaxStages];
  int twoff[kMaxStages];
  int twcount;
};

// The plan of an axis of n = 2^a 3^b points: the radix-3 stages first, then radix 8 with
// a 4 x 4 or a 4 or a 2 for the rest of the power of two (nstages = -1 for other n).  A
// constant expression, so that kernels specialised for an axis length take the same stages
// and twiddle offsets as the table the host builds from it.
constexpr FftPlan plan_of(int n) {
  FftPlan p{};
  p.n = n;
  int rest = n, n3 = 0, n2 = 0;
  while (rest > 0 && rest % 3 == 0) { rest /= 3; ++n3; }
  while (rest > 0 && rest % 2 == 0) { rest /= 2; ++n2; }
  int r[64] = {};
  int k = 0;
  if (rest == 1) {
    for (int i = 0; i < n3; ++i) r[k++] = 3;
    int n8 = n2 / 3;
    const int rem = n2 % 3;
    if (rem == 1 && n8 > 0) {
      n8 -= 1;
      for (int i = 0; i < n8; ++i) r[k++] = 8;
      r[k++] = 4;
      r[k++] = 4;
    } else {
      for (int i = 0; i < n8; ++i) r[k++] = 8;
      if (rem == 2) r[k++] = 4;
      if (rem == 1) r[k++] = 2;
    }
  }
  if (rest != 1 || k > kMaxStages) {
    p.nstages = -1;
    return p;
  }
  p.nstages = k;
  int ns = 1, off = 0;
  for (int s = 0; s < k; ++s) {
    p.radix[s] = r[s];
    p.ns[s] = ns;
    p.twoff[s] = off;
    off += ns * (r[s] - 1);
    ns *= r[s];
  }
  p.twcount = off;
  return p;
}
inline FftPlan make_fft_plan(int n) { return plan_of(n); }
// FP64 twiddles of a plan, 2*twcount doubles (re, im) of exp(-2 pi i k r/(ns R)).
void fft_twiddles(const FftPlan& p, double* out);

// Pointer batches passed to kernels by value.
template <typename P>
struct Batch {
  P p[kMaxBatch];
};

// Host FP64 tables (tables.cpp).
void alpha_staggered(int m, double* out);                  // out[n-1], n = 1..m
void k_staggered_axis(int n, double d, int order, double* out);  // [k]_s on fftfreq order
// Standard Galilean PSATD coefficients of one mode (Sec. 4.3), w = c |[k]_s|, W = v_gal . [k]_c:
// out = theta^2 C, theta^2 S/w, X1, X2, theta^2 X3, X4 (complex, FP64).
void galilean_coefficients(double w, double W, double dt, std::complex<double>* out);
// Averaged Galilean PSATD coefficients of one mode (Sec. 4.4): Psi1, Psi2, Y1, Y2, Y3, Y4.
void averaged_coefficients(double w, double W, double dt, std::complex<double>* out);
void alpha_centered(int m, double* out);                   // out[n-1], n = 1..m
void k_centered_axis(int n, double d, int order, double* out);   // [k]_c on fftfreq order
void psatd_coefficients(double w, double dt, double* C, double* S_over_w, double* X1, double* X2, double* X3);

}  // namespace pic
