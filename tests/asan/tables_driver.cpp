// Host driver for the AddressSanitizer / UndefinedBehaviorSanitizer run of the library's FP64 table
// builders (paper_2106_12919_amd/csrc/tables.cpp), compiled with g++ for the host only.  It calls
// every builder over the ranges pic_init accepts and prints the values, one "name args : values"
// line each, for tests/test_host_sanitizers.py to compare with the oracle.
#include <complex>
#include <cstdio>
#include <vector>

#include "../../paper_2106_12919_amd/csrc/common.h"

using namespace pic;

static void print_vec(const char* name, const std::vector<double>& v, int a, int b, int c) {
  std::printf("%s %d %d %d :", name, a, b, c);
  for (double x : v) std::printf(" %.17g", x);
  std::printf("\n");
}

int main() {
  for (int m = 1; m <= 32; ++m) {
    std::vector<double> s(m), c(m);
    alpha_staggered(m, s.data());
    alpha_centered(m, c.data());
    print_vec("alpha_staggered", s, m, 0, 0);
    print_vec("alpha_centered", c, m, 0, 0);
  }
  const int ns[] = {8, 12, 18, 96, 384, 768, 1024};
  const int orders[] = {0, 2, 4, 16, 64};
  for (int n : ns)
    for (int order : orders) {
      std::vector<double> ks(n), kc(n);
      k_staggered_axis(n, 0.75, order, ks.data());
      k_centered_axis(n, 0.75, order, kc.data());
      print_vec("k_staggered", ks, n, order, 0);
      print_vec("k_centered", kc, n, order, 0);
    }
  const double ws[] = {0.0, 1e-9, 1e-3, 0.05, 0.39, 0.41, 1.0, 3.0, 5.4};
  const double dts[] = {0.5, 1.0, -0.5};
  int i = 0;
  for (double w : ws)
    for (double dt : dts) {
      std::vector<double> v(5);
      psatd_coefficients(w, dt, &v[0], &v[1], &v[2], &v[3], &v[4]);
      std::printf("psatd %d 0 0 : %.17g %.17g", i++, w, dt);
      for (double x : v) std::printf(" %.17g", x);
      std::printf("\n");
    }
  const double gal[][2] = {{1.0, 0.0}, {1.0, 0.3}, {2.5, -0.9}, {0.05, 0.01}, {3.0, 2.99}, {0.0, 0.0}};
  i = 0;
  for (const auto& g : gal) {
    std::complex<double> out[6];
    galilean_coefficients(g[0], g[1], 0.5, out);
    std::printf("galilean %d 0 0 : %.17g %.17g", i, g[0], g[1]);
    for (auto z : out) std::printf(" %.17g %.17g", z.real(), z.imag());
    std::printf("\n");
    averaged_coefficients(g[0], g[1], 0.5, out);
    std::printf("averaged %d 0 0 : %.17g %.17g", i++, g[0], g[1]);
    for (auto z : out) std::printf(" %.17g %.17g", z.real(), z.imag());
    std::printf("\n");
  }
  const int fn[] = {8, 12, 16, 24, 48, 96, 128, 256, 384, 512, 768, 1024, 729, 1000};
  for (int n : fn) {
    FftPlan p = make_fft_plan(n);
    std::printf("plan %d %d 0 :", n, p.nstages);
    if (p.nstages < 0) {
      std::printf("\n");
      continue;
    }
    std::vector<double> tw(2 * (size_t)(p.twcount > 0 ? p.twcount : 1));
    fft_twiddles(p, tw.data());
    int prod = 1;
    for (int s = 0; s < p.nstages; ++s) prod *= p.radix[s];
    std::printf(" %d %d\n", prod, p.twcount);
  }
  return 0;
}
