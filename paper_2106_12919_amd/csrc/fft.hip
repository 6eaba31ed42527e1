// LDS-staged mixed-radix Stockham FFT for gfx950 (radices 2, 3, 4, 8).
//
// The paper's field solve transforms every grid quantity to Fourier space and
// back (Sec. 2, "solve Maxwell's equations on the Yee grid in Fourier space";
// discrete transform of App. A).  The staggered half-cell phase factors are not
// applied here: they are folded into the per-mode update (psatd.hip), so these
// kernels compute the plain index-space DFT.
//
// A real 3D transform runs three passes, each one read and one write of the
// array in HBM:
//   z pass  (r2c/c2r): two real z-lines packed as one complex line, one
//           workgroup per group of line pairs, lines contiguous in LDS;
//   y, x    (c2c):     a tile of TL lines that are adjacent in memory (the kz
//           index, or the flattened (ky,kz) index for x), so every global
//           access is a TL-wide contiguous row; in LDS the tile is stored
//           element-major with the line index fastest, which keeps the
//           butterfly reads and writes free of bank conflicts.
// Each Stockham stage reads its radix-R butterfly inputs from one LDS buffer and
// writes the outputs in autosorted order to the other buffer.
#include <type_traits>

#include "kernels.h"

namespace pic {

namespace {

constexpr int kBlock = 256;

template <typename T, int SIGN>
__device__ inline void dft2(cplx<T>* v) {
  cplx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

// x times an irrational constant c = hi + lo (hi the nearest T, lo the remainder), rounded once:
// the product carries c to twice the precision of T.  A constant rounded to T alone scales the
// modes it touches by |fl(c)/c| != 1 on every pass, and in FP32 that is a systematic loss or gain
// of field energy of ~1e-8 per butterfly stage, the same for every mode that goes through it.
template <typename T>
__device__ inline T mul_const(T x, T hi, T lo) {
  return fma(hi, x, lo * x);
}

template <typename T, int SIGN>
__device__ inline void dft3(cplx<T>* v) {
  // X1 = v0 - (v1+v2)/2 + SIGN i (sqrt3/2)(v1 - v2), X2 = conjugate combination.
  constexpr double hd = 0.86602540378443864676372317075294;
  const T hh = (T)hd, hl = (T)(hd - (double)(T)hd);
  cplx<T> t = cadd(v[1], v[2]);
  cplx<T> d = csub(v[1], v[2]);
  cplx<T> m = cmake(v[0].x - (T)0.5 * t.x, v[0].y - (T)0.5 * t.y);
  const cplx<T> id = cmul_i<T, SIGN>(d);
  cplx<T> r = cmake(mul_const(id.x, hh, hl), mul_const(id.y, hh, hl));
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, r);
  v[2] = csub(m, r);
}

template <typename T, int SIGN>
__device__ inline void dft4(cplx<T>* v) {
  cplx<T> t0 = cadd(v[0], v[2]);
  cplx<T> t1 = csub(v[0], v[2]);
  cplx<T> t2 = cadd(v[1], v[3]);
  cplx<T> t3 = cmul_i<T, SIGN>(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <typename T, int SIGN>
__device__ inline void dft8(cplx<T>* v) {
  constexpr double sd = 0.70710678118654752440084436210485;
  const T sh = (T)sd, sl = (T)(sd - (double)(T)sd);
  cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, SIGN>(e);
  dft4<T, SIGN>(o);
  // twiddles w^k = exp(SIGN i 2 pi k / 8), k = 0..3
  cplx<T> o1 = cmake(mul_const(o[1].x - (T)SIGN * o[1].y, sh, sl), mul_const(o[1].y + (T)SIGN * o[1].x, sh, sl));
  cplx<T> o2 = cmul_i<T, SIGN>(o[2]);
  cplx<T> o3 = cmake(mul_const(-o[3].x - (T)SIGN * o[3].y, sh, sl), mul_const(-o[3].y + (T)SIGN * o[3].x, sh, sl));
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

template <typename T, int SIGN, int R>
__device__ inline void dft(cplx<T>* v) {
  if constexpr (R == 2) dft2<T, SIGN>(v);
  else if constexpr (R == 3) dft3<T, SIGN>(v);
  else if constexpr (R == 4) dft4<T, SIGN>(v);
  else dft8<T, SIGN>(v);
}

// One butterfly of a Stockham stage: reads src[(b + r*nb)] and writes dst[j0 + r*ns].
template <typename T, int SIGN, int R>
__device__ inline void butterfly(const cplx<T>* __restrict__ src, cplx<T>* __restrict__ dst, int lbase, int js,
                                 int b, int nb, int ns, const cplx<T>* __restrict__ tw) {
  cplx<T> v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = src[lbase + (b + r * nb) * js];
  const int k = b % ns;
  if (ns > 1) {
#pragma unroll
    for (int r = 1; r < R; ++r) {
      cplx<T> w = tw[k * (R - 1) + r - 1];
      if (SIGN > 0) w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
  }
  dft<T, SIGN, R>(v);
  const int j0 = (b / ns) * ns * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) dst[lbase + (j0 + r * ns) * js] = v[r];
}

// Transforms ``nlines`` lines held in LDS buffer a (element (l, j) at l*ls + j*js),
// using b as the second buffer.  Returns the buffer holding the result.
template <typename T, int SIGN>
__device__ cplx<T>* fft_lds(cplx<T>* a, cplx<T>* b, int nlines, int ls, int js, const FftPlan& p,
                            const cplx<T>* __restrict__ tw, bool line_fastest) {
  const int N = p.n;
  for (int s = 0; s < p.nstages; ++s) {
    const int R = p.radix[s], ns = p.ns[s];
    const int nb = N / R;
    const int total = nlines * nb;
    const cplx<T>* tws = tw + p.twoff[s];
    for (int w = threadIdx.x; w < total; w += blockDim.x) {
      int l, bi;
      if (line_fastest) { l = w % nlines; bi = w / nlines; }
      else { bi = w % nb; l = w / nb; }
      const int lbase = l * ls;
      switch (R) {
        case 2: butterfly<T, SIGN, 2>(a, b, lbase, js, bi, nb, ns, tws); break;
        case 3: butterfly<T, SIGN, 3>(a, b, lbase, js, bi, nb, ns, tws); break;
        case 4: butterfly<T, SIGN, 4>(a, b, lbase, js, bi, nb, ns, tws); break;
        default: butterfly<T, SIGN, 8>(a, b, lbase, js, bi, nb, ns, tws); break;
      }
    }
    __syncthreads();
    cplx<T>* t = a; a = b; b = t;
  }
  return a;
}

// The transform of lines whose length N and count NL per block are compile-time constants:
// every stage's radix, stride and twiddle offset is a constant of plan_of(N), so butterfly
// indices need no runtime division and LDS offsets become instruction immediates.  Same
// butterflies, in the same order, as fft_lds.  Returns the buffer holding the result.
template <typename T, int SIGN, int N, int NL, bool LINE_FASTEST, int S = 0>
__device__ inline cplx<T>* fft_lds_static(cplx<T>* a, cplx<T>* b, const cplx<T>* __restrict__ tw) {
  constexpr FftPlan P = plan_of(N);
  if constexpr (S == P.nstages) {
    return a;
  } else {
    constexpr int R = P.radix[S], NS = P.ns[S], NB = N / R, TOTAL = NL * NB;
    constexpr int LS = LINE_FASTEST ? 1 : N, JS = LINE_FASTEST ? NL : 1;
    const cplx<T>* tws = tw + P.twoff[S];
#pragma unroll
    for (int w0 = 0; w0 < TOTAL; w0 += kBlock) {
      const int w = w0 + (int)threadIdx.x;
      if (TOTAL % kBlock == 0 || w < TOTAL) {
        const int l = LINE_FASTEST ? w % NL : w / NB;
        const int bi = LINE_FASTEST ? w / NL : w % NB;
        butterfly<T, SIGN, R>(a, b, l * LS, JS, bi, NB, NS, tws);
      }
    }
    __syncthreads();
    return fft_lds_static<T, SIGN, N, NL, LINE_FASTEST, S + 1>(b, a, tw);
  }
}

// The same stages in one LDS buffer: every thread first takes the inputs of all its butterflies
// of a stage into registers, and writes the outputs after the block's barrier.  Half the LDS of
// the two-buffer form for the same tile, at one more barrier per stage.
template <typename T, int SIGN, int N, int NL, bool LINE_FASTEST, int S = 0>
__device__ inline void fft_lds_static_inplace(cplx<T>* a, const cplx<T>* __restrict__ tw) {
  constexpr FftPlan P = plan_of(N);
  if constexpr (S < P.nstages) {
    constexpr int R = P.radix[S], NS = P.ns[S], NB = N / R, TOTAL = NL * NB;
    constexpr int LS = LINE_FASTEST ? 1 : N, JS = LINE_FASTEST ? NL : 1;
    constexpr int IT = (TOTAL + kBlock - 1) / kBlock;
    const cplx<T>* tws = tw + P.twoff[S];
    cplx<T> v[IT][R];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int w = it * kBlock + (int)threadIdx.x;
      if (TOTAL % kBlock == 0 || w < TOTAL) {
        const int l = LINE_FASTEST ? w % NL : w / NB;
        const int bi = LINE_FASTEST ? w / NL : w % NB;
#pragma unroll
        for (int r = 0; r < R; ++r) v[it][r] = a[l * LS + (bi + r * NB) * JS];
        if (NS > 1) {
          const int k = bi % NS;
#pragma unroll
          for (int r = 1; r < R; ++r) {
            cplx<T> t = tws[k * (R - 1) + r - 1];
            if (SIGN > 0) t.y = -t.y;
            v[it][r] = cmul(v[it][r], t);
          }
        }
        dft<T, SIGN, R>(v[it]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int w = it * kBlock + (int)threadIdx.x;
      if (TOTAL % kBlock == 0 || w < TOTAL) {
        const int l = LINE_FASTEST ? w % NL : w / NB;
        const int bi = LINE_FASTEST ? w / NL : w % NB;
        const int j0 = (bi / NS) * NS * R + bi % NS;
#pragma unroll
        for (int r = 0; r < R; ++r) a[l * LS + (j0 + r * NS) * JS] = v[it][r];
      }
    }
    __syncthreads();
    fft_lds_static_inplace<T, SIGN, N, NL, LINE_FASTEST, S + 1>(a, tw);
  }
}

// The centering stencil of LineCenter along the lines of an LDS tile (element (l, j) of NL lines
// of N points at l * LS + j * JS), in place: every thread forms the outputs of its elements from
// LDS into registers, then writes them after the block's barrier.  SHIFT is the stencil's (0
// before a forward transform, -1 after an inverse one).
template <typename T, int N, int NL, bool LINE_FASTEST, int SHIFT>
__device__ inline void center_tile(cplx<T>* a, const LineCenter<T>& lc) {
  constexpr int LS = LINE_FASTEST ? 1 : N, JS = LINE_FASTEST ? NL : 1;
  constexpr int TOTAL = N * NL, IT = (TOTAL + kBlock - 1) / kBlock;
  cplx<T> o[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int w = it * kBlock + (int)threadIdx.x;
    T sx = 0, sy = 0;
    if (TOTAL % kBlock == 0 || w < TOTAL) {
      const int l = LINE_FASTEST ? w % NL : w / N;
      const int j = LINE_FASTEST ? w / NL : w % N;
      const cplx<T>* line = a + l * LS;
      for (int n = 1; n <= lc.m; ++n) {
        int jp = j + n + SHIFT, jm = j - n + 1 + SHIFT;
        jp -= jp >= N ? N : 0;
        jm += jm < 0 ? N : 0;
        const cplx<T> u = line[jp * JS], v = line[jm * JS];
        sx = fma(lc.c[n - 1], u.x + v.x, sx);
        sy = fma(lc.c[n - 1], u.y + v.y, sy);
      }
    }
    o[it] = cmake(sx, sy);
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int w = it * kBlock + (int)threadIdx.x;
    if (TOTAL % kBlock == 0 || w < TOTAL) {
      const int l = LINE_FASTEST ? w % NL : w / N;
      const int j = LINE_FASTEST ? w / NL : w % N;
      a[l * LS + j * JS] = o[it];
    }
  }
  __syncthreads();
}

// Largest element count per thread of one block's LDS tile (two buffers of kLdsBudget
// bytes in all): every thread issues all its global loads (those inside the tile) before it
// stores any to LDS.
#ifndef PIC_FFT_LDS_BUDGET
#define PIC_FFT_LDS_BUDGET 65536
#endif
constexpr size_t kLdsBudget = PIC_FFT_LDS_BUDGET;
// Elements per z-pass block (line pairs times the line length) and the largest strided tile.
#ifndef PIC_FFT_ZPASS_ELEMS
#define PIC_FFT_ZPASS_ELEMS 2048
#endif
#ifndef PIC_FFT_MAX_TL_SHIFT
#define PIC_FFT_MAX_TL_SHIFT 4
#endif
template <typename T>
constexpr int kPerThread = (int)(kLdsBudget / (2 * sizeof(cplx<T>)) / kBlock);

// The plan's twiddles, copied to LDS behind the two tile buffers.
template <typename T>
__device__ inline cplx<T>* stage_twiddles(cplx<T>* lds, const cplx<T>* __restrict__ tw, int count) {
  for (int e = threadIdx.x; e < count; e += blockDim.x) lds[e] = tw[e];
  return lds;
}

// z pass, real -> half spectrum.  Block = P line pairs of one array (blockIdx.y).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_r2c_z(Batch<const T*> in, Batch<cplx<T>*> out, FftPlan p,
                                                  const cplx<T>* __restrict__ tw, int nlines, int pz, int P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = p.n;
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* b = a + (size_t)P * N;
  const T* __restrict__ src = in.p[blockIdx.y];
  cplx<T>* __restrict__ dst = out.p[blockIdx.y];
  const int pair0 = blockIdx.x * P;
  const int np = min(P, nlines / 2 - pair0);
  const int total = np * N;
  constexpr int PER = kPerThread<T>;
  T v0[PER], v1[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = (int)threadIdx.x + u * kBlock;
    if (e < total) {
      const int q = e / N, j = e - q * N;
      const size_t l = 2 * (size_t)(pair0 + q);
      v0[u] = src[l * N + j];
      v1[u] = src[(l + 1) * N + j];
    }
  }
  const cplx<T>* twl = stage_twiddles(b + (size_t)P * N, tw, p.twcount);
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * kBlock;
    if (e < total) a[e] = cmake(v0[u], v1[u]);
  }
  __syncthreads();
  cplx<T>* res = fft_lds<T, -1>(a, b, np, N, 1, p, twl, false);
  const int nh = N / 2 + 1;
  for (int e = threadIdx.x; e < np * nh; e += blockDim.x) {
    const int q = e / nh, k = e - q * nh;
    const cplx<T> zk = res[q * N + k];
    const cplx<T> zn = res[q * N + (k == 0 ? 0 : N - k)];
    const cplx<T> F = cmake((T)0.5 * (zk.x + zn.x), (T)0.5 * (zk.y - zn.y));
    const cplx<T> G = cmake((T)0.5 * (zk.y + zn.y), (T)0.5 * (zn.x - zk.x));
    const size_t l = 2 * (size_t)(pair0 + q);
    dst[l * pz + k] = F;
    dst[(l + 1) * pz + k] = G;
  }
}

// z pass, half spectrum -> real (scaled).  The imaginary parts of the kz = 0 and
// kz = nz/2 bins are dropped (real-output convention).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_c2r_z(Batch<const cplx<T>*> in, Batch<T*> out, FftPlan p,
                                                  const cplx<T>* __restrict__ tw, int nlines, int pz, int P, T scale,
                                                  T scale_lo) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = p.n;
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* b = a + (size_t)P * N;
  const cplx<T>* __restrict__ src = in.p[blockIdx.y];
  T* __restrict__ dst = out.p[blockIdx.y];
  const int pair0 = blockIdx.x * P;
  const int np = min(P, nlines / 2 - pair0);
  const int half = N / 2;
  const int total = np * N;
  constexpr int PER = kPerThread<T>;
  cplx<T> f[PER], g[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = (int)threadIdx.x + u * kBlock;
    if (e < total) {
      const int q = e / N, k = e - q * N;
      const size_t l = 2 * (size_t)(pair0 + q);
      const int kk = k <= half ? k : N - k;
      f[u] = src[l * pz + kk];
      g[u] = src[(l + 1) * pz + kk];
    }
  }
  const cplx<T>* twl = stage_twiddles(b + (size_t)P * N, tw, p.twcount);
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * kBlock;
    if (e < total) {
      const int k = e % N;
      cplx<T> F = f[u], G = g[u];
      if (k > half) {
        F = cconj(F);
        G = cconj(G);
      } else if (k == 0 || k == half) {
        F.y = 0;
        G.y = 0;
      }
      a[e] = cmake(F.x - G.y, F.y + G.x);
    }
  }
  __syncthreads();
  cplx<T>* res = fft_lds<T, +1>(a, b, np, N, 1, p, twl, false);
  for (int e = threadIdx.x; e < np * N; e += blockDim.x) {
    const int q = e / N, j = e - q * N;
    const size_t l = 2 * (size_t)(pair0 + q);
    const cplx<T> v = res[q * N + j];
    dst[l * N + j] = mul_const(v.x, scale, scale_lo);
    dst[(l + 1) * N + j] = mul_const(v.y, scale, scale_lo);
  }
}

// y or x pass, complex -> complex along a strided axis, TL = 2^tl_shift adjacent lines
// per block.
template <typename T, int SIGN>
__global__ void __launch_bounds__(kBlock) k_fft_strided(Batch<const cplx<T>*> in, Batch<cplx<T>*> out, FftPlan p,
                                                        const cplx<T>* __restrict__ tw, int tl_shift, int inner_count,
                                                        int tiles_per_outer, long long outer_stride,
                                                        long long elem_stride) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = p.n;
  const int TL = 1 << tl_shift;
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* b = a + (size_t)TL * N;
  const cplx<T>* __restrict__ src = in.p[blockIdx.y];
  cplx<T>* __restrict__ dst = out.p[blockIdx.y];
#ifndef PIC_FFT_XCD
#define PIC_FFT_XCD 1
#endif
  // tiles next to each other read and write the two halves of the same memory lines: one XCD
  const int tile = PIC_FFT_XCD ? xcd_major(blockIdx.x, gridDim.x) : blockIdx.x;
  const int outer = tile / tiles_per_outer;
  const int inner0 = (tile - outer * tiles_per_outer) * TL;
  const int nl = min(TL, inner_count - inner0);
  const size_t base = (size_t)outer * outer_stride + inner0;
  const int total = N * TL;
  constexpr int PER = kPerThread<T>;
  cplx<T> v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = (int)threadIdx.x + u * kBlock;
    if (e < total) {
      const int j = e >> tl_shift, i = min(e & (TL - 1), nl - 1);
      v[u] = src[base + i + (size_t)j * elem_stride];
    }
  }
  const cplx<T>* twl = stage_twiddles(b + (size_t)TL * N, tw, p.twcount);
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * kBlock;
    if (e < total) a[e] = ((e & (TL - 1)) < nl) ? v[u] : cmake((T)0, (T)0);
  }
  __syncthreads();
  cplx<T>* res = fft_lds<T, SIGN>(a, b, TL, 1, TL, p, twl, true);
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int j = e >> tl_shift, i = e & (TL - 1);
    if (i < nl) dst[base + i + (size_t)j * elem_stride] = res[e];
  }
}


// ------------------------------------------------- kernels for compile-time axis lengths
// The passes above with the axis length N, the pairs per z-pass block P and the lines per
// strided tile TL as template constants (same data layout, LDS use and arithmetic).

// Largest P (z pass) and TL (strided pass) that fit the LDS budget with the twiddles.
template <typename T>
constexpr int static_pairs(int n) {
  int P = PIC_FFT_ZPASS_ELEMS / n;
  if (P < 1) P = 1;
  while (P > 1 && (2 * (size_t)P * n + n) * sizeof(cplx<T>) > kLdsBudget) P /= 2;
  return P;
}
#ifndef PIC_FFT_INPLACE
#define PIC_FFT_INPLACE 1
#endif
// Tile buffers of the strided kernels for compile-time lengths: two (stages from one buffer to
// the other) or one (PIC_FFT_INPLACE: stages in place).
constexpr int kStaticBuffers = PIC_FFT_INPLACE ? 1 : 2;
template <typename T>
constexpr int static_lines(int n, int buffers = 2) {
  int sh = PIC_FFT_MAX_TL_SHIFT;
  while (sh > 0 && (buffers * ((size_t)1 << sh) * n + n) * sizeof(cplx<T>) > kLdsBudget) --sh;
  return 1 << sh;
}

template <typename T, int N>
__global__ void __launch_bounds__(kBlock) k_r2c_z_n(Batch<const T*> in, Batch<cplx<T>*> out,
                                                    const cplx<T>* __restrict__ tw, int nlines, int pz,
                                                    LineCenter<T> lc, unsigned cmask) {
  constexpr int P = static_pairs<T>(N);
  constexpr int TW = plan_of(N).twcount;
  constexpr int PER = (P * N + kBlock - 1) / kBlock;
  constexpr int NH = N / 2 + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* b = a + (size_t)P * N;
  const int pair0 = blockIdx.x * P;
  const int np = min(P, nlines / 2 - pair0);
  const unsigned total = (unsigned)(np * N);
  const T* __restrict__ src = in.p[blockIdx.y] + (size_t)2 * pair0 * N;  // line 2 pair0 of this block
  cplx<T>* __restrict__ dst = out.p[blockIdx.y] + (size_t)2 * pair0 * pz;
  T v0[PER], v1[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const unsigned e = threadIdx.x + u * kBlock;
    if (e < total) {
      const unsigned q = e / N, j = e - q * N;
      v0[u] = src[2 * q * N + j];
      v1[u] = src[(2 * q + 1) * N + j];
    }
  }
  const cplx<T>* twl = stage_twiddles(b + (size_t)P * N, tw, TW);
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const unsigned e = threadIdx.x + u * kBlock;
    if (e < total) a[e] = cmake(v0[u], v1[u]);
  }
  __syncthreads();
  if ((cmask >> blockIdx.y) & 1u) center_tile<T, N, P, false, 0>(a, lc);
  cplx<T>* res = fft_lds_static<T, -1, N, P, false>(a, b, twl);
  constexpr int OUTER = (P * NH + kBlock - 1) / kBlock;
#pragma unroll
  for (int u = 0; u < OUTER; ++u) {
    const unsigned e = threadIdx.x + u * kBlock;
    if (e < (unsigned)(np * NH)) {
      const unsigned q = e / NH, k = e - q * NH;
      const cplx<T> zk = res[q * N + k];
      const cplx<T> zn = res[q * N + (k == 0 ? 0 : N - k)];
      const cplx<T> F = cmake((T)0.5 * (zk.x + zn.x), (T)0.5 * (zk.y - zn.y));
      const cplx<T> G = cmake((T)0.5 * (zk.y + zn.y), (T)0.5 * (zn.x - zk.x));
      dst[2 * q * pz + k] = F;
      dst[(2 * q + 1) * pz + k] = G;
    }
  }
}

template <typename T, int N>
__global__ void __launch_bounds__(kBlock) k_c2r_z_n(Batch<const cplx<T>*> in, Batch<T*> out,
                                                    const cplx<T>* __restrict__ tw, int nlines, int pz, T scale,
                                                    T scale_lo, LineCenter<T> lc, unsigned cmask) {
  constexpr int P = static_pairs<T>(N);
  constexpr int TW = plan_of(N).twcount;
  constexpr int PER = (P * N + kBlock - 1) / kBlock;
  constexpr int HALF = N / 2;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* b = a + (size_t)P * N;
  const int pair0 = blockIdx.x * P;
  const int np = min(P, nlines / 2 - pair0);
  const unsigned total = (unsigned)(np * N);
  const cplx<T>* __restrict__ src = in.p[blockIdx.y] + (size_t)2 * pair0 * pz;
  T* __restrict__ dst = out.p[blockIdx.y] + (size_t)2 * pair0 * N;
  cplx<T> f[PER], g[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const unsigned e = threadIdx.x + u * kBlock;
    if (e < total) {
      const unsigned q = e / N, k = e - q * N;
      const unsigned kk = k <= HALF ? k : N - k;
      f[u] = src[2 * q * pz + kk];
      g[u] = src[(2 * q + 1) * pz + kk];
    }
  }
  const cplx<T>* twl = stage_twiddles(b + (size_t)P * N, tw, TW);
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const unsigned e = threadIdx.x + u * kBlock;
    if (e < total) {
      const unsigned k = e % N;
      cplx<T> F = f[u], G = g[u];
      if (k > HALF) {
        F = cconj(F);
        G = cconj(G);
      } else if (k == 0 || k == HALF) {
        F.y = 0;
        G.y = 0;
      }
      a[e] = cmake(F.x - G.y, F.y + G.x);
    }
  }
  __syncthreads();
  cplx<T>* res = fft_lds_static<T, +1, N, P, false>(a, b, twl);
  if ((cmask >> blockIdx.y) & 1u) center_tile<T, N, P, false, -1>(res, lc);
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const unsigned e = threadIdx.x + u * kBlock;
    if (e < total) {
      const unsigned q = e / N, j = e - q * N;
      const cplx<T> v = res[e];
      dst[2 * q * N + j] = mul_const(v.x, scale, scale_lo);
      dst[(2 * q + 1) * N + j] = mul_const(v.y, scale, scale_lo);
    }
  }
}

// Strided pass with N and TL constant.  Thread t holds line i = t mod TL of the tile (kBlock
// is a multiple of TL) at elements j = t / TL + u kBlock / TL, so its global address advances
// by a constant number of rows per u.
template <typename T, int SIGN, int N>
__global__ void __launch_bounds__(kBlock) k_fft_strided_n(Batch<const cplx<T>*> in, Batch<cplx<T>*> out,
                                                          const cplx<T>* __restrict__ tw, int inner_count,
                                                          int tiles_per_outer, long long outer_stride,
                                                          long long elem_stride, LineCenter<T> lc, unsigned cmask) {
  constexpr int TL = static_lines<T>(N, kStaticBuffers);
  static_assert(kBlock % TL == 0, "a block covers whole rows of the tile");
  constexpr int TW = plan_of(N).twcount;
  constexpr int TOTAL = N * TL;
  constexpr int PER = (TOTAL + kBlock - 1) / kBlock;
  constexpr int ROWS = kBlock / TL;  // rows advanced per u
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* b = a + (size_t)TL * N;  // second buffer (two-buffer stages) or the twiddles
  const int tile = PIC_FFT_XCD ? xcd_major(blockIdx.x, gridDim.x) : blockIdx.x;
  const int outer = tile / tiles_per_outer;
  const int inner0 = (tile - outer * tiles_per_outer) * TL;
  const int nl = min(TL, inner_count - inner0);
  const int i = (int)threadIdx.x % TL, j0 = (int)threadIdx.x / TL;
  const long long row0 = (long long)outer * outer_stride + inner0 + min(i, nl - 1) + (long long)j0 * elem_stride;
  const long long step = (long long)ROWS * elem_stride;
  const cplx<T>* __restrict__ src = in.p[blockIdx.y] + row0;
  cplx<T> v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u)
    if (TOTAL % kBlock == 0 || (int)threadIdx.x + u * kBlock < TOTAL) v[u] = src[u * step];
  const cplx<T>* twl = stage_twiddles(PIC_FFT_INPLACE ? b : b + (size_t)TL * N, tw, TW);
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = (int)threadIdx.x + u * kBlock;
    if (TOTAL % kBlock == 0 || e < TOTAL) a[e] = i < nl ? v[u] : cmake((T)0, (T)0);
  }
  __syncthreads();
  const bool cen = (cmask >> blockIdx.y) & 1u;
  if (SIGN < 0 && cen) center_tile<T, N, TL, true, 0>(a, lc);  // forward: centre, then transform
  cplx<T>* res = a;
  if constexpr (PIC_FFT_INPLACE)
    fft_lds_static_inplace<T, SIGN, N, TL, true>(a, twl);
  else
    res = fft_lds_static<T, SIGN, N, TL, true>(a, b, twl);
  if (SIGN > 0 && cen) center_tile<T, N, TL, true, -1>(res, lc);  // inverse: transform, then centre
  if (i < nl) {
    cplx<T>* __restrict__ dst = out.p[blockIdx.y] + row0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = (int)threadIdx.x + u * kBlock;
      if (TOTAL % kBlock == 0 || e < TOTAL) dst[u * step] = res[e];
    }
  }
}

// Tiles fit the LDS budget of a launch together with the twiddles (fewer than n of them).
template <typename T>
int pairs_per_block(int n) {
  return static_pairs<T>(n);
}
template <typename T>
int lines_per_tile_shift(int n) {
  int sh = 0;
  while ((1 << sh) < static_lines<T>(n)) ++sh;
  return sh;
}

// LDS bytes of a block: two tile buffers of ``elems`` elements and the twiddles.
template <typename T>
size_t fft_lds_bytes(size_t elems, const FftPlan& p) {
  return (2 * elems + (size_t)(p.twcount > 0 ? p.twcount : 1)) * sizeof(cplx<T>);
}

#ifndef PIC_FFT_STATIC
#define PIC_FFT_STATIC 1
#endif
// Calls f(std::integral_constant<int, n>) for the axis lengths that have kernels of their own
// (those of the configurations this library is tuned on) and returns whether it did; other
// lengths take the generic kernels.
template <typename F>
bool with_static_length(int n, F&& f) {
  if (!PIC_FFT_STATIC) return false;
  switch (n) {
    case 64: f(std::integral_constant<int, 64>{}); return true;
    case 128: f(std::integral_constant<int, 128>{}); return true;
    case 256: f(std::integral_constant<int, 256>{}); return true;
    case 384: f(std::integral_constant<int, 384>{}); return true;
    case 768: f(std::integral_constant<int, 768>{}); return true;
    default: return false;
  }
}

template <typename T, int SIGN>
void strided_pass(const Batch<const cplx<T>*>& in, const Batch<cplx<T>*>& out, int count, const FftPlan& p,
                  const cplx<T>* tw, int outer_count, int inner_count, long long outer_stride, long long elem_stride,
                  hipStream_t s, const LineCenter<T>& lc = LineCenter<T>(), int axis = 0) {
  if (with_static_length(p.n, [&](auto nc) {
        constexpr int N = decltype(nc)::value;
        constexpr int TL = static_lines<T>(N, kStaticBuffers);
        const int tpo = (inner_count + TL - 1) / TL;
        dim3 grid(outer_count * tpo, count);
        const size_t lds = (kStaticBuffers * (size_t)TL * N + (size_t)(p.twcount > 0 ? p.twcount : 1)) *
                           sizeof(cplx<T>);
        allow_lds((const void*)k_fft_strided_n<T, SIGN, N>, lds);
        hipLaunchKernelGGL((k_fft_strided_n<T, SIGN, N>), grid, dim3(kBlock), lds, s, in, out, tw, inner_count, tpo,
                           outer_stride, elem_stride, lc, lc.m > 0 ? lc.mask[axis] : 0u);
      }))
    return;
  const int sh = lines_per_tile_shift<T>(p.n);
  const int TL = 1 << sh;
  const int tpo = (inner_count + TL - 1) / TL;
  dim3 grid(outer_count * tpo, count);
  const size_t lds = fft_lds_bytes<T>((size_t)TL * p.n, p);
  allow_lds((const void*)k_fft_strided<T, SIGN>, lds);
  hipLaunchKernelGGL((k_fft_strided<T, SIGN>), grid, dim3(kBlock), lds, s, in, out, p, tw, sh, inner_count, tpo,
                     outer_stride, elem_stride);
}

// A twiddle (c, s) = (cos, sin) of an exact angle in the run precision.  Rounding c and s
// separately leaves |w|^2 - 1 up to ~1e-7 in FP32, the same factor on every pass through that
// twiddle, which the field energy carried by those modes then gains or loses step after step.  In
// FP32 the pair is chosen among the roundings of c and s and their neighbours (each within one
// unit in the last place) as the one whose squared modulus is closest to 1; FP64 rounds directly.
template <typename T>
cplx<T> unit_twiddle(double c, double s) {
  if (sizeof(T) == 8) return cmake((T)c, (T)s);
  cplx<T> best = cmake((T)c, (T)s);
  double err = std::fabs((double)best.x * best.x + (double)best.y * best.y - 1.0);
  const float c0 = (float)c, s0 = (float)s;
  const float cs[3] = {std::nextafter(c0, -2.0f), c0, std::nextafter(c0, 2.0f)};
  const float ss[3] = {std::nextafter(s0, -2.0f), s0, std::nextafter(s0, 2.0f)};
  for (float cc : cs)
    for (float sc : ss) {
      const double e = std::fabs((double)cc * cc + (double)sc * sc - 1.0);
      if (e < err) {
        err = e;
        best = cmake((T)cc, (T)sc);
      }
    }
  return best;
}

}  // namespace

template <typename T>
hipError_t Fft3D<T>::init(int nx_, int ny_, int nz_) {
  nx = nx_; ny = ny_; nz = nz_;
  nzh = nz / 2 + 1;
  const int align = (int)(128 / sizeof(cplx<T>));
  pz = (nzh + align - 1) / align * align;
  const int n[3] = {nx, ny, nz};
  for (int d = 0; d < 3; ++d) {
    plan[d] = make_fft_plan(n[d]);
    if (plan[d].nstages < 0) return hipErrorInvalidValue;
    const int cnt = plan[d].twcount > 0 ? plan[d].twcount : 1;
    double* h = new double[2 * (size_t)cnt]();
    fft_twiddles(plan[d], h);
    cplx<T>* hc = new cplx<T>[cnt];
    for (int i = 0; i < cnt; ++i) hc[i] = unit_twiddle<T>(h[2 * i], h[2 * i + 1]);
    hipError_t e = hipMalloc(&tw[d], cnt * sizeof(cplx<T>));
    if (e == hipSuccess) e = hipMemcpy(tw[d], hc, cnt * sizeof(cplx<T>), hipMemcpyHostToDevice);
    delete[] h;
    delete[] hc;
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
void Fft3D<T>::release() {
  for (int d = 0; d < 3; ++d) {
    if (tw[d]) (void)hipFree(tw[d]);
    tw[d] = nullptr;
  }
}

template <typename T>
bool Fft3D<T>::centering_fusable() const {
  auto has = [](int n) { return with_static_length(n, [](auto) {}); };
  return has(nx) && has(ny) && has(nz);
}

template <typename T>
void Fft3D<T>::forward(const Batch<const T*>& in, const Batch<cplx<T>*>& out, int count, hipStream_t s,
                       const LineCenter<T>* lcp) const {
  const LineCenter<T> lc = lcp ? *lcp : LineCenter<T>();
  const int nlines = nx * ny;
  if (!with_static_length(nz, [&](auto nc) {
        constexpr int N = decltype(nc)::value;
        constexpr int P = static_pairs<T>(N);
        dim3 grid((nlines / 2 + P - 1) / P, count);
        const size_t lds = fft_lds_bytes<T>((size_t)P * N, plan[2]);
        allow_lds((const void*)k_r2c_z_n<T, N>, lds);
        hipLaunchKernelGGL((k_r2c_z_n<T, N>), grid, dim3(kBlock), lds, s, in, out, tw[2], nlines, pz, lc,
                           lc.m > 0 ? lc.mask[2] : 0u);
      })) {
    const int P = pairs_per_block<T>(nz);
    dim3 grid((nlines / 2 + P - 1) / P, count);
    const size_t lds = fft_lds_bytes<T>((size_t)P * nz, plan[2]);
    allow_lds((const void*)k_r2c_z<T>, lds);
    hipLaunchKernelGGL((k_r2c_z<T>), grid, dim3(kBlock), lds, s, in, out, plan[2], tw[2], nlines, pz, P);
  }
  Batch<const cplx<T>*> cin;
  for (int i = 0; i < count; ++i) cin.p[i] = out.p[i];
  strided_pass<T, -1>(cin, out, count, plan[1], tw[1], nx, nzh, (long long)ny * pz, pz, s, lc, 1);
  strided_pass<T, -1>(cin, out, count, plan[0], tw[0], 1, ny * pz, 0, (long long)ny * pz, s, lc, 0);
}

template <typename T>
void Fft3D<T>::inverse(const Batch<const cplx<T>*>& in, const Batch<cplx<T>*>& scratch, const Batch<T*>& out,
                       int count, double scale, hipStream_t s, const LineCenter<T>* lcp) const {
  const LineCenter<T> lc = lcp ? *lcp : LineCenter<T>();
  const T sc_hi = (T)scale, sc_lo = (T)(scale - (double)sc_hi);
  strided_pass<T, +1>(in, scratch, count, plan[0], tw[0], 1, ny * pz, 0, (long long)ny * pz, s, lc, 0);
  Batch<const cplx<T>*> cs;
  for (int i = 0; i < count; ++i) cs.p[i] = scratch.p[i];
  strided_pass<T, +1>(cs, scratch, count, plan[1], tw[1], nx, nzh, (long long)ny * pz, pz, s, lc, 1);
  const int nlines = nx * ny;
  if (!with_static_length(nz, [&](auto nc) {
        constexpr int N = decltype(nc)::value;
        constexpr int P = static_pairs<T>(N);
        dim3 grid((nlines / 2 + P - 1) / P, count);
        const size_t lds = fft_lds_bytes<T>((size_t)P * N, plan[2]);
        allow_lds((const void*)k_c2r_z_n<T, N>, lds);
        hipLaunchKernelGGL((k_c2r_z_n<T, N>), grid, dim3(kBlock), lds, s, cs, out, tw[2], nlines, pz, sc_hi, sc_lo,
                           lc, lc.m > 0 ? lc.mask[2] : 0u);
      })) {
    const int P = pairs_per_block<T>(nz);
    dim3 grid((nlines / 2 + P - 1) / P, count);
    const size_t lds = fft_lds_bytes<T>((size_t)P * nz, plan[2]);
    allow_lds((const void*)k_c2r_z<T>, lds);
    hipLaunchKernelGGL((k_c2r_z<T>), grid, dim3(kBlock), lds, s, cs, out, plan[2], tw[2], nlines, pz, P, sc_hi,
                       sc_lo);
  }
}

template struct Fft3D<float>;
template struct Fft3D<double>;

}  // namespace pic
