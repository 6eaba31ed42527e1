// Host-side launchers of the HIP kernels (internal to libpic).
#pragma once

#include "common.h"

namespace pic {

// ---------------------------------------------------------------- FFT (fft.hip)
// Real 3D transforms of (nx, ny, nz) arrays, z contiguous.  The half spectrum is
// stored (nx, ny, pz) with kz contiguous, kz < nz/2+1 used, pz >= nz/2+1 the row
// pitch.  Forward: X[k] = sum_j x[j] exp(-2 pi i j.k / n) per axis (unnormalised).
// Finite-order centering (Sec. 3) folded into the transform passes: array i of a batch is
// centred along axis a (0 x, 1 y, 2 z) when bit i of mask[a] is set, by the periodic stencil
//   out_j = sum_{n=1}^{m} c[n-1] (in_{j+n+shift} + in_{j-n+1+shift})
// applied to the whole lines of that axis a pass holds in LDS (before the forward transform
// along a, after the inverse one).  A stencil along one axis commutes with the transforms
// along the others, so this is the real-space centering of the array, up to rounding.
template <typename T>
struct LineCenter {
  int m = 0;      // half order (0: no centering)
  int shift = 0;  // 0: nodes -> cell centres, -1: centres -> nodes
  unsigned mask[3] = {0u, 0u, 0u};
  T c[16] = {};
};

template <typename T>
struct Fft3D {
  int nx = 0, ny = 0, nz = 0, nzh = 0, pz = 0;
  FftPlan plan[3];
  cplx<T>* tw[3] = {nullptr, nullptr, nullptr};
  hipError_t init(int nx, int ny, int nz);   // builds plans, uploads twiddles
  void release();
  size_t spectrum_elems() const { return (size_t)nx * ny * pz; }
  // Whether every axis length has transform kernels of its own (LineCenter needs them).
  bool centering_fusable() const;
  // count <= kMaxBatch arrays, real -> spectrum; lc (optional, centering_fusable() only):
  // centering of the inputs folded into the passes
  void forward(const Batch<const T*>& in, const Batch<cplx<T>*>& out, int count, hipStream_t s,
               const LineCenter<T>* lc = nullptr) const;
  // spectrum -> real; ``scratch`` receives the partially transformed spectra (``in`` is preserved);
  // the result is scaled by ``scale`` (given in FP64 and applied to twice the run precision: 1/N is
  // inexact in binary when N has a factor 3, and a rounded scale would change the field energy by
  // the same factor on every inverse transform).
  void inverse(const Batch<const cplx<T>*>& in, const Batch<cplx<T>*>& scratch, const Batch<T*>& out, int count,
               double scale, hipStream_t s, const LineCenter<T>* lc = nullptr) const;
};

// ---------------------------------------------------------------- centering (centering.hip)
// out = centering of in along ``axis`` at order 2m with coefficients c[n-1] = alpha^s_{m,n}/2
// (accumulate: out += it).  shift = 0: nodes -> cell centres; shift = -1: cell centres -> nodes.
template <typename T>
void center_axis(const T* in, T* out, int nx, int ny, int nz, int axis, int shift, int m, const double* c,
                 hipStream_t s, bool accumulate = false);
// out = centering of in along ``axis`` (0 or 1), then along z, both with ``shift``, in one pass
// (the same sums in the same order as two center_axis calls).  Returns false, launching
// nothing, when no row block fits the LDS.
template <typename T>
bool center_axis_then_z(const T* in, T* out, int nx, int ny, int nz, int axis, int shift, int m, const double* c,
                        hipStream_t s);

// ---------------------------------------------------------------- PSATD update (psatd.hip)
template <typename T>
struct PsatdTables {
  T* C = nullptr;        // [nx*ny*nzh] each
  T* Sw = nullptr;
  T* X1 = nullptr;
  T* X2 = nullptr;
  T* X3 = nullptr;
  cplx<T>* Dp[3] = {nullptr, nullptr, nullptr};  // i [k_d]_s exp(+i k_d d_d / 2), per axis (z: nzh entries)
  cplx<T>* Dm[3] = {nullptr, nullptr, nullptr};  // i [k_d]_s exp(-i k_d d_d / 2)
  // Fourier symbol of the nodes -> centres centering along each axis (index-space DFT):
  // sum_n c_n (e^{i theta n} + e^{-i theta (n-1)}); centres -> nodes is its conjugate.
  cplx<T>* Tc[3] = {nullptr, nullptr, nullptr};
  // Standard Galilean PSATD (Sec. 4.3), complex per mode: theta^2 C, theta^2 S/w_s, X1, X2,
  // theta^2 X3, X4 (all null for standard PSATD)
  cplx<T>* G[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  // Averaged Galilean PSATD (Sec. 4.4): Psi1, Psi2, Y1, Y2, Y3, Y4 (null unless averaging)
  cplx<T>* Av[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  // Spectral current correction (standard PSATD): project J onto the Fourier-space
  // continuity equation with (rho^{n+1} - rho^n) / dt before the update
  int cc = 0;
  T inv_dt = 0;
};
// With nodal != nullptr (spectral centering): J holds the NODAL current spectra, centred
// to the Yee grid by the symbols Tc inside the update, and nodal[0..5] receive the
// centred spectra of the updated E (0..2) and B (3..5), ready for the inverse FFT.
template <typename T>
// With averaged tables (t.Av), ``nodal`` instead receives the averaged spectra <E>, <B> of
// Sec. 4.4 (Yee grid, 6 arrays), computed from the fields at the step's start.
void psatd_update(const PsatdTables<T>& t, cplx<T>* const E[3], cplx<T>* const B[3], const cplx<T>* const J[3],
                  const cplx<T>* rho_old, const cplx<T>* rho_new, int nx, int ny, int nzh, int pz,
                  cplx<T>* const* nodal, hipStream_t s);
// Conjugate transpose of the update per mode (reverse mode): E, B hold the adjoints of the
// updated fields and receive those of the old fields; J, rho_old, rho_new receive the
// adjoints of the sources.
template <typename T>
void psatd_adjoint(const PsatdTables<T>& t, cplx<T>* const E[3], cplx<T>* const B[3], cplx<T>* const J[3],
                   cplx<T>* rho_old, cplx<T>* rho_new, int nx, int ny, int nzh, int pz, hipStream_t s);

// Workgroups of a launch go to the eight XCDs of the device round-robin (workgroup b
// to XCD b mod 8), and each XCD has its own L2.  xcd_major renumbers the workgroups
// 0..n-1 so that every XCD receives one contiguous range of logical indices: tiles
// next to each other, which share halo nodes or halves of memory lines, then share an L2.
// (A bijection for any n; only the speed depends on the dispatch order.)
__device__ inline int xcd_major(int b, int n) {
  constexpr int kXcds = 8;
  const int q = n / kXcds, r = n % kXcds;
  const int x = b % kXcds, s = b / kXcds;
  return x * q + min(x, r) + s;
}

// Lets a kernel launch with more than the default 64 KiB of dynamic LDS (gfx950: up to 160 KiB
// per workgroup); a failure is cleared and left to the launch to report.
void allow_lds(const void* kernel, size_t bytes);

// ---------------------------------------------------------------- particles (particles.hip)
// Division by a fixed divisor d (1 <= d < 2^31) as a multiply-high and a shift:
// n / d == (mulhi(n, m) + n) >> s for 0 <= n < 2^31, with s = ceil(log2 d) and
// m = floor(2^32 (2^s - d) / d) + 1 (Granlund and Montgomery, PLDI 1994, Sec. 4).
struct FastDiv {
  uint32_t d, m, s;
};
FastDiv make_fastdiv(uint32_t d);

struct GridGeom {
  int nx, ny, nz;
  double dx, dy, dz, dt;
  int shape_order;
  FastDiv ny_div, nz_div;  // decode of linear cell indices
  // Galilean frame (Sec. 4.3): the grid moves with v_gal, so a particle moves by
  // (v - v_gal) dt per step; sg = v_gal dt / (dx, dy, dz) in cells (0 for standard PSATD)
  double sgx, sgy, sgz;
  // Deterministic depositions: each tile's fixed-point scale comes from the particle count
  // times the largest contribution (a maximum and a count do not depend on the order in
  // which the tile's particles are visited) instead of the floating-point sum of the
  // contributions, whose rounding does.  Everything else of the deposition is integer
  // arithmetic, exact in any order.
  int det;
};
GridGeom make_geom(int nx, int ny, int nz, double dx, double dy, double dz, double dt, int shape_order);

// Edge of the deposition / gather tiles in cells.  A compile-time constant, so that
// every LDS offset inside a tile's box is an instruction immediate.
constexpr int kTile = 8;
template <typename T>
struct SpeciesView {
  int64_t n;
  int32_t* cell;
  T* off[3];
  T* u[3];
  T* w;         // may be null
  double w_const, q, m;
};
struct TileGeom {
  int ntx, nty, ntz, ntiles;
  int* scan_tmp = nullptr;  // device scratch of the bucket scan: (ntiles + 1) / 8192 + 2 ints
};
TileGeom make_tiles(const GridGeom& g);  // tiles of kTile^3 cells
// Edge length (nodes) of the LDS boxes of one tile: the tile, the shape support and a
// one-cell margin on each side (particles move less than one cell per step).
int deposit_box(int shape_order);
// Elements per component of a tile's slot in the staging buffer of deposit_tiled: B x B rows
// (B = deposit_box) of 16 values, row (lx, ly) holding box nodes lz = 0 .. B-1 at positions
// lz + ((BASE + 3) mod 4) (BASE = -1 cubic, 0 linear) and zeros elsewhere.  The offset puts grid
// nodes z = 4g .. 4g+3 at positions 4h .. 4h+3 of every box that covers them, so that the
// reduction reads four nodes of a box as one aligned vector.
int deposit_stage_slot(int shape_order);
// Counting sort by tile of the particles' current cells: counts[ntiles+1],
// starts[ntiles+2], cursor[ntiles+1] (scratch), dst[n] = each particle's slot in
// tile order (tiles in order, then particles with invalid cells, counted in *bad).
void tile_sort(const GridGeom& g, const TileGeom& t, const int32_t* cell, int64_t n, int* counts, int* starts,
               int* cursor, int* dst, int* bad, hipStream_t s);
void invert_perm(const int* dst, int* perm, int64_t n, hipStream_t s);
// Exclusive scan of counts[ntiles + 1] into starts[ntiles + 2] and cursor[ntiles + 1].
void scan_counts(const TileGeom& t, const int* counts, int* starts, int* cursor, hipStream_t s);
// Slot runs of the regrouping: from the per-(source tile, neighbour) counts a deposition
// published (nbr_counts, source grouping old_starts) and the new grouping's starts,
// bases[27 S + nb] = first slot of source S's particles bound for neighbour nb, and
// cursor[D] = first slot of tile D after all its runs (for particles that moved further).
void neighbour_bases(const TileGeom& t, const int* old_starts, const int* nbr_counts, const int* new_starts,
                     int* bases, int* cursor, hipStream_t s);

// Tile-ordered gather + push.  Either through a permutation (home_cursor == nullptr):
// slot q of tile t (q in [starts[t], starts[t+1]), tiles of the current cells) reads
// particle perm[q] of ``in`` and writes it to slot q of ``out`` (write_sorted) or to
// perm[q] (in place when out == in); or, in pic_step's steady state, ``in`` grouped by
// home tile (starts = home ranges) is written to ``out`` grouped by the tile of each
// particle's current cell, slots reserved per block from home_cursor (the new starts);
// nbr_bases (optional, from neighbour_bases) holds, per home tile, the first slot of
// its particles bound for each neighbour tile [27 * ntiles]; without it each block
// counts its particles and reserves the runs with atomics on home_cursor.
template <typename T>
void gather_push_tiled(const GridGeom& g, const TileGeom& t, const T* const E[3], const T* const B[3],
                       const SpeciesView<T>& in, const SpeciesView<T>& out, const int* perm, const int* starts,
                       bool write_sorted, int* home_cursor, const int* nbr_bases, hipStream_t s);
template <typename T>
void permute_species(const SpeciesView<T>& in, const SpeciesView<T>& out, const int* dst, hipStream_t s);
// Deposition of one species in two launches.  deposit_tiled accumulates rho (at the
// particles' positions) and, when with_j, J (at x - dt v/2) tile by tile (tile t owns
// sorted slots [starts[t], starts[t+1]); slot q holds particle perm[q], perm == nullptr:
// q) into per-tile boxes in ``stage`` (ntiles * (with_j ? 4 : 1) * deposit_stage_slot
// elements, row layout); particles that left the one-cell margin go straight to rho/J.
// deposit_reduce with ReduceArgs::rows = 1 then sums the overlapping boxes into the nodal arrays.
// With next_counts != nullptr, the particles are also counted per tile of their cells
// (the grouping of the next step), into next_counts[ntiles + 1] (invalid cells last),
// and, when nbr_counts != nullptr, per tile t of this grouping and neighbour nb of t
// (0..26, the tile offsets in {-1,0,1}^3 in x-major order) into nbr_counts[27 t + nb].
// ``work`` is one int of device scratch (the tile counter of the persistent launch).
// ``spill_flag`` (optional) is set to 1 whenever a particle goes to rho/J directly.  With
// ``box_faces`` (ntiles ints, optional; used on grids of whole tiles) each tile stages only
// the layers of its box that hold a nonzero value and records which outer faces it staged,
// for a deposit_reduce with the same array in ReduceArgs::box_faces.
template <typename T>
void deposit_tiled(const GridGeom& g, const TileGeom& t, const SpeciesView<T>& sp, const int* perm, const int* starts,
                   bool with_j, T* stage, int* bad, int* next_counts, int* nbr_counts, int* work, T* rho,
                   T* const J[3], hipStream_t s, int* spill_flag = nullptr, int* box_faces = nullptr);
// How deposit_reduce starts each node and what else it folds in.  By default it adds to the
// nodal arrays.  With bit 0 (rho) or bit 1 (J) of acc_mask clear it overwrites them instead,
// rho starting from ``base`` when given, else from zero.  When *flag != 0, the ``spill``
// arrays (which hold what a deposit_tiled with rho/J = spill sent past its boxes, and are zero
// otherwise) are added and cleared.  *next_flag is zeroed for the deposition after this one.
template <typename T>
struct ReduceArgs {
  int acc_mask = 3;
  const T* base = nullptr;
  T* spill[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  const int* flag = nullptr;
  int* next_flag = nullptr;
  const int* box_faces = nullptr;  // per tile, the outer faces its deposition staged (null: all)
  // Staging layout: 0 = node-major boxes (B^3 per component); 1 = the zero-padded rows that
  // deposit_tiled writes (deposit_stage_slot elements per component).
  int rows = 0;
  __device__ T start(int q, const T* o, size_t idx) const {
    if (acc_mask & (q == 0 ? 1 : 2)) return o[idx];
    return (q == 0 && base) ? base[idx] : (T)0;
  }
  __device__ T take_spill(int q, size_t idx) const {
    const T v = spill[q][idx];
    spill[q][idx] = 0;
    return v;
  }
};
template <typename T>
void deposit_reduce(const GridGeom& g, const TileGeom& t, const int* starts, const T* stage, bool with_j, T* rho,
                    T* const J[3], hipStream_t s, const ReduceArgs<T>& ra = ReduceArgs<T>());

// Reverse mode of gather + push + move + deposition of one species, particles at time n
// visited in slot order (slot q -> particle perm[q]; perm == nullptr: q); with the tile
// grouping of their cells (starts != nullptr) one workgroup per tile reads the fields from
// LDS boxes when they fit, else one particle per thread reads them from the grids.
// lam[0..2] (dL/d offsets, cells) and lam[3..5] (dL/du) hold the adjoints of x^{n+1}, u^{n+1/2}
// and receive those of x^n, u^{n-1/2}.  F: nodal E (0..2) and B (3..5) of the state at n;
// L: dL/drho^{n+1} (0) and dL/dJ_nod (1..3).  lamF[0..5][p] receives dL/d(E_p, B_p), the
// adjoints of the fields gathered at the particle (zero for immobile species).
template <typename T>
void particle_adjoint(const GridGeom& g, const TileGeom& t, const SpeciesView<T>& sp, const Batch<T*>& lam,
                      const int* perm, const int* starts, const T* const F[6], const T* const L[4],
                      const Batch<T*>& lamF, hipStream_t s);
// out[v] += sum_p val[v][p] S(x_p - x_i), v = 0..5 (the transpose of the gather), with the
// grouping (perm, starts) of the particles' current cells; stage: ntiles * 6 * deposit_box^3.
template <typename T>
void scatter_tiled(const GridGeom& g, const TileGeom& t, const SpeciesView<T>& sp, const int* perm, const int* starts,
                   const T* const val[6], T* const out[6], T* stage, hipStream_t s);

// The fully staggered comparison cycle: gather + push with every component of E, B (Yee-grid
// arrays) interpolated from its own Yee positions, in place, one particle per thread; and the
// deposition of rho^{n+1} (nodes) and J (each component onto its own Yee positions) with global
// atomics (adds to rho and J).
template <typename T>
void gather_push_yee(const GridGeom& g, const T* const E[3], const T* const B[3], const SpeciesView<T>& sp,
                     hipStream_t s);
template <typename T>
void deposit_yee(const GridGeom& g, const SpeciesView<T>& sp, bool with_j, T* rho, T* const J[3], hipStream_t s);
// The same through per-tile fixed-point LDS boxes (grouping of the current cells: perm, starts;
// stage as deposit_tiled's with 4 components) and the deposition's box reduction.
template <typename T>
void deposit_yee_tiled(const GridGeom& g, const TileGeom& t, const SpeciesView<T>& sp, const int* perm,
                       const int* starts, bool with_j, T* stage, T* rho, T* const J[3], hipStream_t s);
// gather_push_yee through the grouping of the particles' cells and per-tile LDS boxes of E, B.
template <typename T>
void gather_push_yee_tiled(const GridGeom& g, const TileGeom& t, const T* const E[3], const T* const B[3],
                           const SpeciesView<T>& sp, const int* perm, const int* starts, hipStream_t s);

// ---------------------------------------------------------------- reductions (diag.hip)
// acc[0] += sum of squares over ``count`` arrays of n elements; acc[1] += sum of ``sum_arr``.
template <typename T>
void sum_squares(const Batch<const T*>& arrs, int count, int64_t n, double* acc, hipStream_t s);
template <typename T>
void sum_plain(const T* arr, int64_t n, double* acc, hipStream_t s);
template <typename T>
void add_into(T* dst, const T* src, int64_t n, hipStream_t s);
// Zeroes count (<= 8) arrays of n elements in one launch.
template <typename T>
void zero_arrays(const Batch<T*>& arrs, int count, int64_t n, hipStream_t s);
// acc[0] += sum |sum_d D-_d V_d + ca A + cb B|^2, acc[1] += sum |ca A + cb B|^2 over the
// half-spectrum modes (index-space spectra of the Yee components V and of A, B; B may be null),
// weighted as full-spectrum sums.
template <typename T>
void div_residual(const PsatdTables<T>& t, const cplx<T>* const V[3], const cplx<T>* A, double ca, const cplx<T>* B,
                  double cb, int nx, int ny, int nzh, int pz, int nz, double* acc, hipStream_t s);

}  // namespace pic
